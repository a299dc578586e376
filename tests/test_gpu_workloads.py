"""GPU tests of the two largest workloads at full size, in the launch
configuration the bench times (batched form, persistent launches over every
lane bucket).

* Batching: 65,536 ligands of 15-50 heavy atoms (skewed toward 25-35), 0-12
  torsions, 1 pocket of 2,000 atoms with 64^3 x 8 maps, 32 trajectories x 150
  MC steps x 10 Adam steps.
* Mixed pockets: 16 pockets (800-3,000 atoms, grids 48^3-96^3 x 8), 4,096
  ligands each of 10-70 heavy atoms assigned round-robin, 64 trajectories x
  200 MC steps, all in one dock_sample call; then the adjoint across the 16
  pockets in one call.

Every trajectory's evaluation count, the best/current bookkeeping and the
lane plan are checked in full.  A subset of trajectories (every 4,096th /
4,097th ligand, its first two trajectories; for the mixed workload one ligand
in each pocket) logs its evaluations on the GPU during the full run; the
oracle runs the same ligands and trajectories itself (same Philox stream, its
own FP64 arithmetic, no GPU value as input) for the first MC steps, and the
two logs are compared row by row (tests/_coupled.py).  Over all 150 / 200
steps, each logged trajectory's best energy equals the minimum of its
per-step final energies.  The mixed-pocket adjoint is checked by exact
identities at full size and against the oracle's adjoint on seeded poses of
two ligands per pocket.
"""
import multiprocessing as mp
import time

import numpy as np
import pytest

import synth
from oracle import topology, maps as MAPS, score as SC, adjoint as ADJ, params as P, atomtype as AT
from tests import _gpu as G
from tests import _coupled as CP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ORACLE_STEPS = 8


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G.lib()


def _full_run_checks(D, run, H, L, T, S, stride, tt):
    st = D.dock_run_state(run, trace=True)
    torch.cuda.synchronize()
    nev = st["n_evals"].cpu().numpy()
    assert np.all(nev == 1 + S * 11), np.unique(nev)
    Eb, Ec = st["E_best"].cpu().numpy(), st["E_cur"].cpu().numpy()
    assert np.all(np.isfinite(Eb)) and np.all(Eb <= Ec)
    tr = st["trace"].cpu().numpy()
    traced = np.arange(0, L.n_ligands, stride)
    assert tr.shape[:2] == (len(traced), tt)
    # the best energy of a logged trajectory is the least of its initial
    # energy and its MC steps' final energies (rows 0, 11, 22, ...)
    qs = st["q_stride"]
    for a, l in enumerate(traced):
        for t in range(tt):
            finals = tr[a, t, 0:1 + S * 11:11, 2 * qs]
            assert Eb[l, t] == finals.min(), (l, t, Eb[l, t], finals.min())
    return st, tr, traced


def _coupled_oracle(jobs, tr, nev, traced_ids, tt, n_dof_of, workers):
    kw = dict(kind="adam", n_local=10, lr=0.1)
    t0 = time.time()
    with mp.get_context("spawn").Pool(workers) as pool:
        outs = pool.map(CP.oracle_run, jobs)
    G.say("oracle: %d ligands x %d trajectories x %d MC steps in %.1f s" % (len(jobs), tt, ORACLE_STEPS,
                                                                              time.time() - t0))
    tot = dict(whole=0, parted=0, explained=0, rows=0)
    for a, (rows, margins) in enumerate(outs):
        res = CP.compare_prefix(tr[a], nev[a], rows, margins, n_dof=n_dof_of[a], **kw)
        for k in tot:
            tot[k] += res[k]
        for t, why in res["unexplained"]:
            G.say("  ligand", traced_ids[a], "trajectory", t, "unexplained:", why)
        assert res["unexplained"] == [], (traced_ids[a], res["unexplained"])
    G.say("coupled with the oracle: %d of %d trajectories whole over %d steps, %d parted (all explained), "
          "%d rows agree" % (tot["whole"], len(jobs) * tt, ORACLE_STEPS, tot["parted"], tot["rows"]))
    return tot


def test_batching_workload_full_size(D):
    workers = synth.default_workers()
    t0 = time.time()
    pks, L, wl = synth.workload("C4", workers=workers)
    G.say("batching workload: %d ligands drawn in %.1f s" % (L.n_ligands, time.time() - t0))
    T, S = wl["T"], wl["S"]
    w = G.weights32(P.PRESET_TRIDS)
    p = G.load_pocket(pks[0], P.PRESET_TRIDS, w)
    H = G.load_ligands(L)
    stride, tt, seed = 4096, 2, 7
    torch.cuda.synchronize()
    t0 = time.time()
    run = D.dock_sample(p, H, n_traj=T, n_steps=S, seed=seed, record_trace=1, trace_lig_stride=stride,
                        trace_traj=tt)
    ms = D.dock_run_kernel_ms(run)
    G.say("batching workload: %d trajectories x %d steps, sampler %.0f ms (%.0f M evals/s), call %.1f s"
          % (L.n_ligands * T, S, ms, L.n_ligands * T * (1 + S * 11) / ms / 1e3, time.time() - t0))
    plan = D.dock_run_plan(run)
    G.say("lane buckets", list(zip(plan["lanes"].tolist(), plan["apl"].tolist())))
    assert (32, 2) in list(zip(plan["lanes"].tolist(), plan["apl"].tolist()))
    st, tr, traced = _full_run_checks(D, run, H, L, T, S, stride, tt)
    sub = L.subset(traced)
    jobs, ndof = [], []
    for a, l in enumerate(traced):
        ndof.append(topology.from_ligands(sub, a).n_dof)
        jobs.append((pks[0], P.PRESET_TRIDS, w.astype(np.float64), sub, a, int(l),
                     dict(n_traj=T, n_steps=ORACLE_STEPS, n_local=10, seed=seed), list(range(tt))))
    nev = st["n_evals"].cpu().numpy()[traced, :tt]
    tot = _coupled_oracle(jobs, tr, nev, traced, tt, ndof, workers)
    assert tot["rows"] >= len(jobs) * tt * 12


def test_mixed_pockets_workload_full_size(D):
    workers = synth.default_workers()
    t0 = time.time()
    pks, L, wl = synth.workload("C5", workers=workers)
    G.say("mixed pockets: %d pockets, %d ligands drawn in %.1f s" % (len(pks), L.n_ligands, time.time() - t0))
    T, S = wl["T"], wl["S"]
    w = G.weights32(P.PRESET_TRIDS)
    ps = [G.load_pocket(pk, P.PRESET_TRIDS, w, keep=True) for pk in pks]
    H = G.load_ligands(L)
    stride, tt, seed = 4097, 1, 5   # ligands 0, 4097, 8194, ... land in pockets 0, 1, 2, ...
    torch.cuda.synchronize()
    t0 = time.time()
    run = D.dock_sample(ps, H, n_traj=T, n_steps=S, seed=seed, record_trace=1, trace_lig_stride=stride,
                        trace_traj=tt)
    ms = D.dock_run_kernel_ms(run)
    G.say("mixed pockets: %d trajectories x %d steps over 16 pockets, sampler %.0f ms (%.0f M evals/s), "
          "call %.1f s" % (L.n_ligands * T, S, ms, L.n_ligands * T * (1 + S * 11) / ms / 1e3, time.time() - t0))
    st, tr, traced = _full_run_checks(D, run, H, L, T, S, stride, tt)
    assert sorted(L.pocket_index[traced].tolist()) == list(range(16))
    sub = L.subset(traced)
    jobs, ndof = [], []
    for a, l in enumerate(traced):
        ndof.append(topology.from_ligands(sub, a).n_dof)
        jobs.append((pks[int(L.pocket_index[l])], P.PRESET_TRIDS, w.astype(np.float64), sub, a, int(l),
                     dict(n_traj=T, n_steps=ORACLE_STEPS, n_local=10, seed=seed), list(range(tt))))
    nev = st["n_evals"].cpu().numpy()[traced, :tt]
    tot = _coupled_oracle(jobs, tr, nev, traced, tt, ndof, workers)
    assert tot["rows"] >= len(jobs) * tt * 12

    # ---- adjoint across the 16 pockets in one call: L = sum of every
    # ligand's best-pose energy, gradients to each pocket's per-term maps and
    # weights (deterministic mode)
    best = D.dock_best_poses(H, T, st["E_best"], st["q_best"], top_n=1, rmsd_cluster=1.0, want_xyz=False)
    qb = best["q"][:, 0].contiguous()
    lig = torch.arange(L.n_ligands, dtype=torch.int32, device="cuda")
    Gs = [D.dock_pocket_maps(pp, per_term=True) for pp in ps]
    wt = torch.tensor(np.tile(w, (16, 1)), device="cuda")
    ones = torch.ones(L.n_ligands, device="cuda")
    dG = [torch.zeros_like(g) for g in Gs]
    dw = torch.zeros_like(wt)
    torch.cuda.synchronize()
    t0 = time.time()
    D.dock_score_adjoint(ps, H, lig, wt, ones, q=qb, G=Gs, dLdG=dG, dLdw=dw, deterministic=1)
    torch.cuda.synchronize()
    G.say("adjoint over %d best poses and 16 pockets: %.1f ms" % (L.n_ligands, (time.time() - t0) * 1e3))
    # node sums: sum_nodes dL/dG[t][k] = w_k * (# atoms of type t over the pocket's poses)
    counts = np.zeros((16, 8))
    for l in range(L.n_ligands):
        lg = L.ligand(l)
        counts[L.pocket_index[l]] += np.bincount(AT.type_atoms(lg["element"], lg["n_h"], lg["bonds"]), minlength=8)
    dw = dw.cpu().numpy().astype(np.float64)
    for pi in range(16):
        got = dG[pi].cpu().numpy().astype(np.float64).reshape(8, 3, -1).sum(-1)
        expect = counts[pi][:, None] * w[None].astype(np.float64)
        assert np.allclose(got, expect, rtol=1e-5, atol=1e-5 * np.abs(expect).max()), pi
    # dL/dw from the forward's linearity in w (GPU forward, FP64 sums)
    for k in range(3):
        e = np.zeros((16, 3), np.float32)
        e[:, k] = 1.0
        Ep = D.dock_score_terms(ps, H, lig, wt + torch.tensor(e, device="cuda"), q=qb, G=Gs).cpu().numpy()
        Em = D.dock_score_terms(ps, H, lig, wt - torch.tensor(e, device="cuda"), q=qb, G=Gs).cpu().numpy()
        fd = np.zeros(16)
        np.add.at(fd, L.pocket_index, (Ep.astype(np.float64) - Em) / 2.0)
        scale = np.abs(Ep).astype(np.float64)
        tol = np.zeros(16)
        np.add.at(tol, L.pocket_index, scale)
        assert np.all(np.abs(fd - dw[:, k]) <= 2e-5 * tol + 1e-3), (k, fd, dw[:, k])

    # ---- seeded poses of two ligands per pocket: the adjoint of those poses
    # alone against the oracle's, pocket by pocket (maps filled where touched)
    rng = np.random.default_rng(77)
    pick = [l for pi in range(16) for l in np.flatnonzero(L.pocket_index == pi)[1:3]]
    subL = L.subset(pick)
    topos = [topology.from_ligands(subL, a) for a in range(len(pick))]
    n_per = 4
    Q = np.zeros((len(pick) * n_per, H.q_stride), np.float32)
    pl = np.repeat(np.asarray(pick, np.int32), n_per)
    for a, t in enumerate(topos):
        Q[a * n_per:(a + 1) * n_per, :t.n_dof] = G.poses_for(t, n_per, rng, "near")
    dLdE = rng.normal(size=len(Q)).astype(np.float32)
    dG = [torch.zeros_like(g) for g in Gs]
    dw = torch.zeros_like(wt)
    D.dock_score_adjoint(ps, H, torch.tensor(pl, device="cuda"), wt, torch.tensor(dLdE, device="cuda"),
                         q=torch.tensor(Q, device="cuda"), G=Gs, dLdG=dG, dLdw=dw, deterministic=1)
    torch.cuda.synchronize()
    dw = dw.cpu().numpy()
    worst = 0.0
    for pi in range(16):
        pk = pks[pi]
        grid = SC.grid_of(pk)
        mine = [a for a in range(len(pick)) if L.pocket_index[pick[a]] == pi]
        xs = [_fk(topos[a], Q[a * n_per:(a + 1) * n_per]) for a in mine]
        Gd = _lazy_terms(pk, P.PRESET_TRIDS, grid, xs)
        refG, refw = np.zeros_like(Gd), np.zeros(3)
        for a in mine:
            t = topos[a]
            sl = slice(a * n_per, (a + 1) * n_per)
            A = ADJ.adjoint(Gd, w.astype(np.float64), grid, P.PRESET_TRIDS, t, dLdE[sl].astype(np.float64),
                            q=Q[sl, :t.n_dof].astype(np.float64))
            refG += A["dLdG"]
            refw += A["dLdw"]
        got = dG[pi].cpu().numpy().astype(np.float64)
        sc = np.abs(refG).max()
        worst = max(worst, np.abs(got - refG).max() / sc)
        assert np.abs(got - refG).max() <= 1e-5 * sc + 1e-7, pi
        np.testing.assert_allclose(dw[pi], refw, rtol=1e-5, atol=1e-4 * np.abs(refw).max())
    G.say("seeded poses, 16 pockets: dL/dG worst max |diff| / max %.3g" % worst)


def _fk(topo, Q):
    from oracle import fk as FK
    return FK.fk(topo, Q[:, :topo.n_dof].astype(np.float64))


def _lazy_terms(pk, preset, grid, xs):
    """Oracle per-term maps filled at the nodes the given coordinates touch."""
    nx, ny, nz = pk.dims
    Gd = np.zeros((8, P.n_terms(preset), nz, ny, nx))
    c = np.concatenate([SC.cells(grid, x.reshape(-1, 3)) for x in xs])
    idx = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                idx.append(((c[:, 2] + dz) * ny + c[:, 1] + dy) * nx + c[:, 0] + dx)
    flat = np.unique(np.concatenate(idx))
    vals = MAPS.build_maps(pk, preset, nodes=flat)
    z, rem = np.divmod(flat, nx * ny)
    y, x = np.divmod(rem, nx)
    Gd[:, :, z, y, x] = vals
    return Gd
