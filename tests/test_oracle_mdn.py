"""Pins of the oracle's E_MDN term from supplied mixture parameters: a plain
loop over residues and atoms, a single-Gaussian closed form, central finite
differences of the gradient, and invariance under a rigid motion of the
whole complex."""
import math

import numpy as np

import synth
from oracle import mdn as MDN


def _system(seed=0, n_rec=30, n_lig=5, P=6, K=3):
    rng = np.random.default_rng(seed)
    rec = rng.uniform(-6, 6, size=(n_rec, 3))
    residue = np.sort(rng.integers(0, 7, size=n_rec)).astype(np.int32)
    residue = np.unique(residue, return_inverse=True)[1].astype(np.int32)
    n_res = residue.max() + 1
    params = synth.make_mdn_params(n_lig, n_res, K, seed=seed).astype(np.float64)
    x = rng.uniform(-4, 4, size=(P, n_lig, 3))
    return rec, residue, params, x


def test_against_plain_loops():
    rec, residue, params, x = _system()
    E, _, _, _ = MDN.mdn_energy(x, rec, residue, params)
    for p in range(len(x)):
        tot = 0.0
        for i in range(residue.max() + 1):
            atoms = [a for a in range(len(rec)) if residue[a] == i]
            for j in range(x.shape[1]):
                d = min(math.dist(x[p, j], rec[a]) for a in atoms)
                if d < 5.0:
                    tot -= sum(pi * math.exp(-(d - mu) ** 2 / (2 * s * s)) for pi, mu, s in params[j, i])
        assert abs(E[p] - tot) <= 1e-12 * max(1.0, abs(tot))


def test_single_gaussian_closed_form():
    rec = np.zeros((1, 3))
    residue = np.zeros(1, np.int32)
    params = np.array([[[[1.0, 3.2, 0.5]]]])
    for d in (0.0, 1.0, 3.2, 4.9, 5.1):
        E, g, _, _ = MDN.mdn_energy(np.array([[[d, 0.0, 0.0]]]), rec, residue, params)
        want = -math.exp(-(d - 3.2) ** 2 / 0.5) if d < 5.0 else 0.0
        assert abs(E[0] - want) < 1e-15
        if 0 < d < 5.0:
            # E = -P(d), dE/dd = P (d - mu) / sigma^2, and dd/dx = 1 on the axis
            want_g = math.exp(-(d - 3.2) ** 2 / 0.5) * (d - 3.2) / 0.25
            assert abs(g[0, 0, 0] - want_g) < 1e-12


def test_gradient_against_finite_differences():
    rec, residue, params, x = _system(seed=3)
    E, g, _, margin = MDN.mdn_energy(x, rec, residue, params)
    h = 1e-6
    checked = 0
    for p in range(len(x)):
        if margin[p] < 1e-3:
            continue
        for j in range(x.shape[1]):
            for c in range(3):
                xp, xm = x.copy(), x.copy()
                xp[p, j, c] += h
                xm[p, j, c] -= h
                fd = (MDN.mdn_energy(xp[p:p + 1], rec, residue, params)[0][0]
                      - MDN.mdn_energy(xm[p:p + 1], rec, residue, params)[0][0]) / (2 * h)
                assert abs(fd - g[p, j, c]) <= 1e-6 * max(1.0, abs(fd))
                checked += 1
    assert checked >= 30


def test_rigid_motion_invariance():
    rec, residue, params, x = _system(seed=5)
    E0, _, _, _ = MDN.mdn_energy(x, rec, residue, params)
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1.0]])
    t = np.array([1.5, -2.0, 0.25])
    E1, _, _, _ = MDN.mdn_energy(x @ R.T + t, rec @ R.T + t, residue, params)
    np.testing.assert_allclose(E1, E0, rtol=1e-12, atol=1e-12)
