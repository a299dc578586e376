"""Pins of the oracle's optimiser, Philox stream, Metropolis sampler, best-pose
selection and adjoint (CPU).

* Adam against torch.optim.Adam in FP64 (library routine);
* Armijo line search on a quadratic with a closed-form answer;
* Philox4x32-10 against rocRAND's engine (library routine, built for the host);
* acceptance frequency at dE = 10 against exp(-0.69) (the paper's beta);
* resume equality, E_best monotone, L = 0 pure Metropolis;
* RMSD / clustering by hand and by brute force;
* adjoint: exact finite differences in the linear inputs, central FD in x.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import torch

import synth
from oracle import optim, philox as PX, sampler as SM, best as BEST, topology, adjoint as ADJ
from oracle import score as SC, params as P, fk as FK, maps as MAPS
from tests._tiny import tiny_pocket, tiny_ligand


def test_adam_matches_torch_fp64():
    rng = np.random.default_rng(0)
    A = rng.normal(size=(7, 7)); A = A @ A.T + np.eye(7)
    c = rng.normal(size=7) * 0.1
    f = lambda q: 0.5 * np.einsum("pi,ij,pj->p", q, A, q) + q @ c + 0.1 * (q ** 4).sum(1)
    df = lambda q: q @ A + c + 0.4 * q ** 3
    q0 = rng.uniform(-0.3, 0.3, (1, 7))
    q0[0, :3] = 0.0
    box = (np.full(3, -100.0), np.full(3, 100.0))
    q, E = optim.adam_refine(lambda q: (f(q), df(q)), q0, 10, *box)
    t = torch.tensor(q0[0], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=0.1, betas=(0.9, 0.999), eps=1e-8)
    At = torch.tensor(A); ct = torch.tensor(c)
    for _ in range(10):
        opt.zero_grad()
        loss = 0.5 * t @ At @ t + t @ ct + 0.1 * (t ** 4).sum()
        loss.backward()
        opt.step()
    np.testing.assert_allclose(q[0], t.detach().numpy(), rtol=1e-12, atol=1e-13)


def test_adam_first_step_is_lr_times_sign():
    g = np.array([[3.0, -0.2, 1e-3, -50.0, 7.0, 0.5]])
    q0 = np.zeros((1, 6))
    box = (np.full(3, -9.0), np.full(3, 9.0))
    q, _ = optim.adam_refine(lambda q: (np.zeros(1), g), q0, 1, *box)
    np.testing.assert_allclose(q, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_armijo_line_search_on_quadratic():
    qs = np.array([[0.3, -0.2, 0.1, 0.0, 0.0, 0.0]])
    f = lambda q: (0.5 * ((q - qs) ** 2).sum(1), q - qs)
    box = (np.full(3, -9.0), np.full(3, 9.0))
    # distance 3 > 0.5001: alpha = 1 accepted -> moves exactly 1 toward qs
    q0 = qs + np.array([[3.0, 0, 0, 0, 0, 0]])
    q, E = optim.linesearch_refine(f, q0, 1, *box)
    np.testing.assert_allclose(q, qs + np.array([[2.0, 0, 0, 0, 0, 0]]), atol=1e-14)
    # distance 0.3: alpha = 1 overshoots, alpha = 0.5 satisfies Armijo
    q0 = qs + np.array([[0.0, 0.3, 0, 0, 0, 0]])
    q, E = optim.linesearch_refine(f, q0, 1, *box)
    np.testing.assert_allclose(q, qs + np.array([[0.0, -0.2, 0, 0, 0, 0]]), atol=1e-14)
    # at the minimum nothing moves
    q, E = optim.linesearch_refine(f, qs.copy(), 3, *box)
    np.testing.assert_allclose(q, qs, atol=0)


def test_wrap_and_clamp():
    q = np.array([[5.0, -5.0, 0.5, np.pi, -np.pi, 3 * np.pi + 0.1, -7.0]])
    w = optim.wrap_clamp(q, np.array([-1.0, -1.0, -1.0]), np.array([1.0, 1.0, 1.0]))
    np.testing.assert_allclose(w[0, :3], [1.0, -1.0, 0.5])
    assert np.all(w[0, 3:] >= -np.pi) and np.all(w[0, 3:] < np.pi)
    np.testing.assert_allclose(np.cos(w[0, 3:]), np.cos(q[0, 3:]), atol=1e-12)


_RR_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int a = 1; a + 2 < argc; a += 3) {
    unsigned long long seed = strtoull(argv[a], 0, 0), sub = strtoull(argv[a + 1], 0, 0),
                       off = strtoull(argv[a + 2], 0, 0);
    rocrand_state_philox4x32_10 s;
    rocrand_init(seed, sub, off, &s);
    for (int i = 0; i < 8; i++) printf("%u ", rocrand(&s));
    printf("\n");
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_host_exe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host reference")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "rr.cpp")
    exe = os.path.join(d, "rr")
    open(src, "w").write(_RR_SRC)
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-I/opt/rocm/include",
                           src, "-o", exe], stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand_engine(rocrand_host_exe):
    # rocRAND's engine: key = (seed lo, seed hi); counter = (offset/4 as 64-bit
    # in words 0-1, subsequence as 64-bit in words 2-3); 4 outputs per counter.
    cases = [(0, 0, 0), (0x0000000500000007, 0, 0), (0xdeadbeefcafef00d, 3, 0),
             (123456789, 0x0000000900000002, 40), (0xffffffffffffffff, 0xffffffffffffffff, 8)]
    args = []
    for c in cases:
        args += [str(v) for v in c]
    out = subprocess.check_output([rocrand_host_exe] + args).decode().strip().splitlines()
    for (seed, sub, off), line in zip(cases, out):
        ref = [int(v) for v in line.split()]
        got = []
        for blk in range(2):
            ctr = off // 4 + blk
            w = PX.philox4x32_10([ctr & PX.M32, ctr >> 32, sub & PX.M32, sub >> 32],
                                 [seed & PX.M32, seed >> 32])
            got += [int(v) for v in w]
        assert got == ref


def test_unit_and_index_maps():
    x = np.array([0, 255, 256, 0xFFFFFFFF], np.uint32)
    u = PX.to_unit(x)
    assert u[0] == 0.0 and u[1] == 0.0 and u[2] == 2.0 ** -24 and u[3] == 1.0 - 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    assert list(PX.mulhi_index(np.array([0, 0xFFFFFFFF], np.uint32), 7)) == [0, 6]
    w = PX.draw(3, 9, np.arange(20000), 1, PX.PURPOSE_STEP)
    cnt = np.bincount(PX.mulhi_index(w[0], 10), minlength=10)
    assert cnt.min() > 1800 and cnt.max() < 2200


class _MockScorer:
    """E(q) = c for every pose -> every proposal has dE = 0 (or a fixed offset)."""

    def __init__(self, fn):
        self.fn = fn

    def score(self, topo, q):
        E = self.fn(q)
        return dict(E=E, dEdq=np.zeros_like(q))

    def energy(self, topo, q):
        return self.fn(q)


def _topo():
    return topology.from_ligands(tiny_ligand(6, 2, seed=1), 0)


def test_metropolis_acceptance_frequency_at_delta_10():
    topo = _topo()
    n = 20000
    prm = SM.SamplerParams(n_traj=n, n_steps=1, n_local=0, seed=5)
    st = SM.init_state(_MockScorer(lambda q: np.zeros(len(q))), topo, 0, prm)
    st = SM.run_steps(_MockScorer(lambda q: np.full(len(q), 10.0)), topo, 0, prm, st, 1)
    frac = np.mean(st.E_cur == 10.0)
    p = math.exp(-0.069 * 10.0)
    assert abs(frac - p) < 4 * math.sqrt(p * (1 - p) / n)


def test_downhill_always_accepted_and_one_dof_changes():
    topo = _topo()
    prm = SM.SamplerParams(n_traj=500, n_steps=1, n_local=0, seed=2)
    st = SM.init_state(_MockScorer(lambda q: np.zeros(len(q))), topo, 0, prm)
    q0 = st.q_cur.copy()
    st = SM.run_steps(_MockScorer(lambda q: np.full(len(q), -1.0)), topo, 0, prm, st, 1)
    assert np.all(st.E_cur == -1.0)
    changed = (st.q_cur != q0).sum(1)
    assert np.all(changed <= 1) and changed.sum() > 450
    lo, hi = SM.dof_range(topo)
    assert np.all(q0 >= lo) and np.all(q0 < hi + 1e-12)


def test_sampler_resume_and_monotone_best():
    pk = tiny_pocket(n=20, radius=6.0, grid=28)
    sc = SC.Scorer(pk)
    topo = _topo()
    prm = SM.SamplerParams(n_traj=6, n_steps=6, n_local=3, seed=4)
    full = SM.sample(sc, topo, 7, prm)
    st = SM.init_state(sc, topo, 7, prm)
    hist = [st.E_best.copy()]
    for _ in range(6):
        st = SM.run_steps(sc, topo, 7, prm, st, 1)
        hist.append(st.E_best.copy())
        assert np.all(st.E_best <= st.E_cur)
    assert np.all(np.diff(np.array(hist), axis=0) <= 0)
    for a in ("q_cur", "E_cur", "q_best", "E_best"):
        assert np.array_equal(getattr(full, a), getattr(st, a))


def test_linesearch_sampler_runs_and_improves():
    pk = tiny_pocket(n=20, radius=6.0, grid=28)
    sc = SC.Scorer(pk)
    topo = _topo()
    prm = SM.SamplerParams(n_traj=4, n_steps=3, n_local=2, seed=4, local_opt=SM.LOCAL_LINESEARCH)
    st0 = SM.init_state(sc, topo, 7, prm)
    st = SM.run_steps(sc, topo, 7, prm, SM.init_state(sc, topo, 7, prm), 3)
    assert np.all(st.E_best <= st0.E_best)


def test_rmsd_and_clustering():
    x = np.random.default_rng(0).normal(size=(10, 3))
    assert BEST.rmsd(x, x + np.array([1.0, 0, 0])) == pytest.approx(1.0)
    assert BEST.rmsd(x, x) == 0.0
    L = synth.make_ligands(3, 12, 3, seed=4)
    rng = np.random.default_rng(5)
    for i in range(3):
        topo = topology.from_ligands(L, i)
        T = 64
        q = synth.random_poses(topo.n_dof, topo.box_min, topo.box_max, T, rng).astype(np.float64)
        q[T // 2:] = q[:T // 2] + rng.normal(size=(T // 2, topo.n_dof)) * 0.02   # near-duplicates
        E = rng.normal(size=T)
        E[5] = E[9]                                      # a tie: lower id first
        out = BEST.best_poses(topo, E, q, top_n=8, rmsd_cut=1.0)
        sel = out["idx"]
        X = FK.fk(topo, q)
        # brute-force greedy reference
        order = sorted(range(T), key=lambda k: (E[k], k))
        ref = []
        for k in order:
            if len(ref) == 8:
                break
            if all(BEST.rmsd(X[k], X[r]) >= 1.0 for r in ref):
                ref.append(k)
        assert list(sel) == ref
        assert np.all(np.diff(out["E"]) >= 0)
        np.testing.assert_allclose(out["E_screen"], E[sel] / (1 + 0.01 * topo.n_tors))


@pytest.mark.parametrize("preset", [P.PRESET_TRIDS, P.PRESET_VINA])
def test_adjoint_exact_in_linear_inputs_and_fd_in_x(preset):
    pk = tiny_pocket(n=20, radius=6.0, grid=20)
    grid = SC.grid_of(pk)
    G = MAPS.build_maps(pk, preset)
    K = P.n_terms(preset)
    rng = np.random.default_rng(8)
    w = np.asarray(P.default_weights(preset)) * (1 + 0.1 * rng.normal(size=K))
    topo = topology.from_ligands(tiny_ligand(6, 2, seed=3), 0)
    q = synth.random_poses(topo.n_dof, topo.box_min, topo.box_max, 5, rng).astype(np.float64)
    dLdE = rng.normal(size=5)
    L = lambda G, w, q=q, x=None: dLdE @ ADJ.energy(G, w, grid, preset, topo, q=q, x=x)
    A = ADJ.adjoint(G, w, grid, preset, topo, dLdE, q=q)
    # weights: E linear in w -> difference quotient exact up to rounding
    for k in range(K):
        e = np.zeros(K); e[k] = 1.0
        np.testing.assert_allclose((L(G, w + e) - L(G, w - e)) / 2, A["dLdw"][k], rtol=1e-9, atol=1e-9)
    # map values: perturb nodes with nonzero and zero adjoint
    nz = np.argwhere(np.abs(A["dLdG"]) > 0)
    picks = [tuple(nz[i]) for i in rng.choice(len(nz), 6, replace=False)] + [(0, 0, 0, 0, 0)]
    for idx in picks:
        Gp = G.copy(); Gp[idx] += 1.0
        Gm = G.copy(); Gm[idx] -= 1.0
        np.testing.assert_allclose((L(Gp, w) - L(Gm, w)) / 2, A["dLdG"][idx], rtol=1e-8, atol=1e-9)
    # coordinates: central FD
    x = FK.fk(topo, q)
    Ax = ADJ.adjoint(G, w, grid, preset, topo, dLdE, x=x)
    h = 1e-6
    for a in range(topo.n_atoms):
        for c in range(3):
            xp = x.copy(); xp[:, a, c] += h
            xm = x.copy(); xm[:, a, c] -= h
            fd = (dLdE * (ADJ.energy(G, w, grid, preset, topo, x=xp) - ADJ.energy(G, w, grid, preset, topo, x=xm))) / (2 * h)
            np.testing.assert_allclose(Ax["dLdx"][:, a, c], fd, rtol=1e-5, atol=1e-5)
    # q path agrees with the grid scorer's chain rule
    sc = SC.Scorer(pk, preset, weights=w, G=G)
    np.testing.assert_allclose(A["dLdq"], dLdE[:, None] * sc.score(topo, q)["dEdq"], rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("kind", [optim.SGD, optim.RMSPROP, optim.ADAGRAD, optim.ADAMW])
def test_optimizer_variants_match_torch_fp64(kind):
    rng = np.random.default_rng(kind)
    A = rng.normal(size=(7, 7)); A = A @ A.T + np.eye(7)
    c = rng.normal(size=7) * 0.1
    f = lambda q: 0.5 * np.einsum("pi,ij,pj->p", q, A, q) + q @ c + 0.1 * (q ** 4).sum(1)
    df = lambda q: q @ A + c + 0.4 * q ** 3
    q0 = rng.uniform(-0.3, 0.3, (1, 7))
    q0[0, :3] = 0.05
    box = (np.full(3, -100.0), np.full(3, 100.0))
    q, E = optim.first_order_refine(kind, lambda q: (f(q), df(q)), q0, 8, *box, lr=0.01)
    t = torch.tensor(q0[0], dtype=torch.float64, requires_grad=True)
    opt = {optim.SGD: lambda: torch.optim.SGD([t], lr=0.01),
           optim.RMSPROP: lambda: torch.optim.RMSprop([t], lr=0.01, alpha=0.99, eps=1e-8),
           optim.ADAGRAD: lambda: torch.optim.Adagrad([t], lr=0.01, eps=1e-8),
           optim.ADAMW: lambda: torch.optim.AdamW([t], lr=0.01, betas=(0.9, 0.999), eps=1e-8,
                                                   weight_decay=0.01)}[kind]()
    At = torch.tensor(A); ct = torch.tensor(c)
    for _ in range(8):
        opt.zero_grad()
        loss = 0.5 * t @ At @ t + t @ ct + 0.1 * (t ** 4).sum()
        loss.backward()
        opt.step()
    np.testing.assert_allclose(q[0], t.detach().numpy(), rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------- screening rank

def _rank_brute(v, k):
    # a plain sort with an explicit key, independent of screen_rank's lexsort
    items = sorted(range(len(v)), key=lambda i: (math.isnan(v[i]), 0.0 if math.isnan(v[i]) else v[i], i))
    s = [v[i] for i in items[:k]] + [math.inf] * max(0, k - len(v))
    idx = items[:k] + [-1] * max(0, k - len(v))
    return s, idx


@pytest.mark.parametrize("seed", range(6))
def test_screen_rank_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 40))
    v = rng.choice([-3.0, -1.5, -0.0, 0.0, 2.0, np.inf, np.nan, -np.inf], size=n)
    v = np.where(rng.random(n) < 0.5, rng.normal(size=n), v)
    for k in (1, 5, 50):
        s, idx = BEST.screen_rank(v, k)
        bs, bidx = _rank_brute(list(v), k)
        assert list(idx) == bidx
        np.testing.assert_array_equal(np.asarray(s), np.asarray(bs))


def test_screen_rank_ties_and_specials():
    v = [1.0, -0.0, 0.0, np.nan, -2.0, 1.0, np.inf, -2.0]
    s, idx = BEST.screen_rank(v, 10)
    assert list(idx) == [4, 7, 1, 2, 0, 5, 6, 3, -1, -1]
    assert np.isinf(s[-1]) and np.isnan(s[7])
