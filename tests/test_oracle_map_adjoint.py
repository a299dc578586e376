"""Pins of the oracle's map-build adjoint (TRIDS terms): the explicit-constant
map build equals the map build of maps.py, and the analytic adjoint equals
central finite differences of L = sum(lam * G) with respect to every term
constant and to receptor coordinates away from the fixed cutoffs."""
import numpy as np
import pytest

from oracle import map_adjoint as MA, maps as MAPS, params as P
from tests._tiny import tiny_pocket


def _pocket():
    return tiny_pocket(n=12, radius=5.0, grid=14, seed=7)


def test_explicit_constants_reproduce_the_map_build():
    pk = _pocket()
    G = MA.map_terms(pk, MA.default_theta())
    ref = MAPS.build_maps(pk, P.PRESET_TRIDS).reshape(8, 3, -1)
    np.testing.assert_allclose(G, ref, rtol=1e-12, atol=1e-12)


def _loss(pk, lam, theta, decide=None):
    return float(np.sum(lam * MA.map_terms(pk, theta, decide=decide)))


def test_theta_gradient_against_finite_differences():
    pk = _pocket()
    rng = np.random.default_rng(0)
    n = int(np.prod(pk.dims))
    lam = rng.normal(size=(8, 3, n))
    th = MA.default_theta()
    _, dth = MA.map_adjoint(pk, lam, th)
    h = 1e-6
    for j in range(MA.N_THETA):
        e = np.zeros(MA.N_THETA)
        e[j] = h
        # clash cutoff decisions held at theta (the term is zero where d_c
        # moves them)
        fd = (_loss(pk, lam, th + e, th) - _loss(pk, lam, th - e, th)) / (2 * h)
        assert abs(fd - dth[j]) <= 1e-6 * max(1.0, abs(fd)), (MA.THETA_NAMES[j], fd, dth[j])


def test_receptor_gradient_against_finite_differences():
    pk = _pocket()
    rng = np.random.default_rng(1)
    n = int(np.prod(pk.dims))
    lam = rng.normal(size=(8, 3, n))
    th = MA.default_theta()
    dr, _ = MA.map_adjoint(pk, lam, th)
    margin = MA.fixed_cutoff_margin(pk)
    h = 1e-7
    checked = 0
    for i in range(len(pk.type)):
        if margin[i] < 1e-4:
            continue
        for c in range(3):
            xyz = np.array(pk.xyz, np.float64)
            plus, minus = pk.__class__(**{**pk.__dict__}), pk.__class__(**{**pk.__dict__})
            xp, xm = xyz.copy(), xyz.copy()
            xp[i, c] += h
            xm[i, c] -= h
            plus.xyz, minus.xyz = xp, xm
            fd = (_loss(plus, lam, th) - _loss(minus, lam, th)) / (2 * h)
            assert abs(fd - dr[i, c]) <= 1e-5 * max(1.0, abs(fd)), (i, c, fd, dr[i, c])
            checked += 1
    assert checked >= 6


def test_adjoint_is_linear_in_lam():
    pk = _pocket()
    rng = np.random.default_rng(2)
    n = int(np.prod(pk.dims))
    a, b = rng.normal(size=(8, 3, n)), rng.normal(size=(8, 3, n))
    ra, ta = MA.map_adjoint(pk, a)
    rb, tb = MA.map_adjoint(pk, b)
    rs, ts = MA.map_adjoint(pk, 2.0 * a - b)
    np.testing.assert_allclose(rs, 2.0 * ra - rb, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(ts, 2.0 * ta - tb, rtol=1e-9, atol=1e-9)
