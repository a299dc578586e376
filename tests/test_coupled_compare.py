"""CPU checks of the coupled-trajectory comparison (tests/_coupled.py) that the
GPU sampler tests rely on.

The "device" side here is the oracle itself run a second time with
FP32-like noise on every evaluation (poses rounded to float32, energies and
gradients perturbed at the size of the GPU's measured errors).  With that
noise alone every parting must be explained by a decision margin or by
gradual drift.  With a mistake planted in the second run (a wrong Armijo
constant, a wrong Adam moment rate, an energy offset, a wrong Metropolis
beta) the comparison must report partings it cannot explain.
"""
import numpy as np
import pytest

from oracle import topology, score as SC, sampler as SM, optim, params as P
from tests import _coupled as C
from tests._tiny import tiny_pocket, tiny_ligand


class _Noisy:
    """Scorer wrapper: float32 poses, relative noise on E and dE/dq, and an
    optional energy offset (a planted mistake)."""

    def __init__(self, base, seed, e_off=0.0):
        self.b = base
        self.rng = np.random.default_rng(seed)
        self.e_off = e_off

    def score(self, topo, q):
        q32 = np.asarray(q, np.float32).astype(np.float64)
        r = dict(self.b.score(topo, q32))
        r["E"] = r["E"] + 3e-7 * r["S_abs"] * self.rng.normal(size=len(q32)) + self.e_off * r["S_abs"]
        gn = np.linalg.norm(r["dEdq"], axis=1, keepdims=True)
        r["dEdq"] = r["dEdq"] + 3e-6 * gn * self.rng.normal(size=r["dEdq"].shape)
        return r

    def energy(self, topo, q):
        return self.score(topo, q)["E"]


@pytest.fixture(scope="module")
def system():
    pk = tiny_pocket(n=20, radius=6.0, grid=28)
    L = tiny_ligand(9, 3, seed=6)
    w = np.asarray(P.TRIDS_WEIGHTS, np.float32).astype(np.float64)
    return SC.Scorer(pk, weights=w), topology.from_ligands(L, 0)


def _run(sc, topo, prm):
    ev, tr = SM.EvalLog(prm.n_traj), []
    SM.sample(sc, topo, 0, prm, trace=tr, evlog=ev)
    return ev, tr


def _as_trace(ev, n_dof):
    qs = n_dof + 2
    T = len(ev.rows)
    cap = max(len(r) for r in ev.rows)
    out = np.full((T, cap, 2 * qs + 1), np.nan, np.float32)
    nev = np.zeros(T, np.int64)
    for t, rows in enumerate(ev.rows):
        for k, (q, E, g, *_rest) in enumerate(rows):
            out[t, k, :n_dof] = q
            out[t, k, qs:qs + n_dof] = g
            out[t, k, 2 * qs] = E
        nev[t] = len(rows)
    return out, nev


KINDS = {"adam": (SM.LOCAL_ADAM, 10, 0.1), "linesearch": (SM.LOCAL_LINESEARCH, 3, 0.1),
         "sgd": (SM.LOCAL_SGD, 4, 0.002)}


def _compare(system, kind, planted=None, seed=1):
    sc, topo = system
    opt, nl, lr = KINDS[kind]
    prm = SM.SamplerParams(n_traj=24, n_steps=4, n_local=nl, seed=4, local_opt=opt, lr=lr)
    ev, tr = _run(sc, topo, prm)
    noisy = _Noisy(sc, seed, e_off=1e-4 if planted == "energy" else 0.0)
    prm2 = SM.SamplerParams(**{**prm.__dict__})
    saved = optim.ARMIJO_C
    try:
        if planted == "armijo":
            optim.ARMIJO_C = 2e-2
        if planted == "adam":
            prm2.beta1 = 0.8
        if planted == "beta":
            prm2.mc_beta = 0.5
        ev2, _ = _run(noisy, topo, prm2)
    finally:
        optim.ARMIJO_C = saved
    gt, nev = _as_trace(ev2, topo.n_dof)
    return C.compare_run(gt, nev, ev, tr, kind, nl, lr, topo.n_dof)


@pytest.mark.parametrize("kind", ["adam", "linesearch", "sgd"])
def test_fp32_noise_partings_are_explained(system, kind):
    res = _compare(system, kind)
    assert res["unexplained"] == [], res["unexplained"][:3]
    assert res["whole"] >= res["T"] // 2, res


@pytest.mark.parametrize("kind,planted", [("linesearch", "armijo"), ("adam", "adam"), ("adam", "energy"),
                                          ("sgd", "beta")])
def test_planted_mistakes_are_reported(system, kind, planted):
    res = _compare(system, kind, planted)
    assert len(res["unexplained"]) >= 3, (planted, res)


def test_linesearch_log_replay(system):
    """The line-search replay used on the GPU's log accepts the oracle's own
    log and rejects a log made with a different Armijo constant."""
    sc, topo = system
    prm = SM.SamplerParams(n_traj=12, n_steps=4, n_local=3, seed=4, local_opt=SM.LOCAL_LINESEARCH)
    ev, _ = _run(sc, topo, prm)
    gt, nev = _as_trace(ev, topo.n_dof)
    tot = np.zeros(3, int)
    for t in range(prm.n_traj):
        tot += C.check_linesearch_log(gt[t], int(nev[t]), topo.n_dof, 3, topo.box_min, topo.box_max)
    assert tot[1] > 0 and tot[0] > tot[1]
    saved = optim.ARMIJO_C
    try:
        optim.ARMIJO_C = 0.3
        ev2, _ = _run(sc, topo, prm)
    finally:
        optim.ARMIJO_C = saved
    gt, nev = _as_trace(ev2, topo.n_dof)
    with pytest.raises(AssertionError):
        for t in range(prm.n_traj):
            C.check_linesearch_log(gt[t], int(nev[t]), topo.n_dof, 3, topo.box_min, topo.box_max)
