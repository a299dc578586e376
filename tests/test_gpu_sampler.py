"""GPU tests of the sampler forms, resume, best-pose selection and whole-run
distributions.  Run on an MI355X.

* plain, batched, hipGraph-replayed and chunked launches give bit-identical
  trajectories (random streams depend on ligand, trajectory and step only);
* a run large enough for two atoms per lane (33-64-atom ligands) uses that
  layout, its logged evaluations match the oracle and its forms agree;
* run(S) == run(s) + advance(S - s) == restore(state at s) + advance, bitwise;
* live runs sharing the device's bucket streams (interleaved advances, two
  caller streams) reach the states each reaches alone;
* the recorded trace is self-consistent (score kernel at the logged q, Adam
  update rule between consecutive rows, Armijo condition for line search);
* best poses (rank, RMSD clustering, top N, E_screen) against the oracle on
  seeded candidate sets;
* best-pose energy and RMSD distributions over seeds against the oracle's
  (stored by tests/golden/make_c1_best_distribution.py);
* short Adam trajectories coupled with the oracle's.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import topology, score as SC, sampler as SM, best as BEST, fk as FK, params as P
from tests import _gpu as G
from tests._tiny import tiny_pocket, tiny_ligand
from tests import _coupled as CP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G.lib()


@pytest.fixture(scope="module")
def mixed(D):
    """A 2,000-atom pocket and 12 ligands spanning every lane configuration."""
    pk = synth.make_pocket(2000, grid=64, seed=0)
    spec = [(10, 0), (15, 6), (20, 3), (28, 9), (33, 5), (40, 15), (52, 8), (60, 14), (64, 2),
            (66, 6), (70, 12), (24, 4)]
    L = synth.pack_ligands([synth.make_ligand(n, t, np.random.default_rng(70 + n)) for n, t in spec])
    L.pocket_index = np.zeros(L.n_ligands, np.int32)
    w = G.weights32(P.PRESET_TRIDS)
    return G.load_pocket(pk, P.PRESET_TRIDS, w), G.load_ligands(L), L, pk


def _state(D, run):
    st = D.dock_run_state(run)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in st.items()}


def _same(a, b, tag):
    for k in ("q_cur", "E_cur", "q_best", "E_best", "n_evals"):
        assert np.array_equal(a[k], b[k]), (tag, k, np.argwhere(a[k] != b[k])[:4])


def test_forms_are_bitwise_identical(D, mixed):
    p, H, L, _ = mixed
    kw = dict(n_traj=24, n_steps=6, n_local=4, seed=9)
    G.say("forms: plain")
    ref = _state(D, D.dock_sample(p, H, form=D.FORM_PLAIN, use_graph=0, **kw))
    for form, graph, chunk in ((D.FORM_BATCHED, 0, 0), (D.FORM_BATCHED, 1, 0), (D.FORM_BATCHED, 1, 2),
                               (D.FORM_BATCHED, 0, 4)):
        G.say("forms: batched graph", graph, "chunk", chunk)
        got = _state(D, D.dock_sample(p, H, form=form, use_graph=graph, steps_per_launch=chunk, **kw))
        _same(ref, got, (form, graph, chunk))
    assert np.all(ref["n_evals"] == 1 + 6 * 5)
    assert np.all(ref["E_best"] <= ref["E_cur"])


def test_forced_wider_groups_agree(D, mixed):
    p, H, L, _ = mixed
    kw = dict(n_traj=8, n_steps=3, n_local=3, seed=2)
    G.say("lanes: auto vs 64")
    a = _state(D, D.dock_sample(p, H, **kw))
    b = _state(D, D.dock_sample(p, H, lanes_per_pose=64, **kw))
    # different reduction trees: close, not bitwise
    np.testing.assert_allclose(a["E_cur"][:, :], b["E_cur"], rtol=2e-3, atol=1e-3)


def _two_per_lane_traj(mid):
    """Trajectories per ligand at which a run lays out the 33-64-atom ligands
    two atoms per lane: two poses per wavefront must fill at least two waves
    per wave slot (12 waves per CU)."""
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    need = 2 * 2 * 12 * n_cu
    return 64 * (-(-need // (64 * mid)) + 1)


def test_two_atoms_per_lane_runs_against_oracle(D, mixed):
    """A run that fills the chip with two poses per wavefront lays out the
    33-64-atom ligands two atoms per lane in 32-lane groups; a small run keeps
    one atom per lane.  The large run's logged evaluations match the oracle
    at sampled rows, and its plain and batched forms agree bitwise."""
    p, H, L, pk = mixed
    topos = [topology.from_ligands(L, i) for i in range(L.n_ligands)]
    mid = [i for i, t in enumerate(topos) if 32 < t.n_atoms <= 64 and t.n_dof <= 32]
    assert len(mid) == 5
    T = _two_per_lane_traj(len(mid))
    kw = dict(n_steps=2, n_local=3, seed=21)
    G.say("two per lane: plans, T =", T)
    small = D.dock_sample(p, H, n_traj=16, **kw)
    big = D.dock_sample(p, H, n_traj=T, record_trace=1, **kw)
    for run, want in ((small, (64, 1)), (big, (32, 2))):
        plan = D.dock_run_plan(run)
        for i in mid:
            b = plan["lig_bucket"][i]
            assert (plan["lanes"][b], plan["apl"][b]) == want, (i, plan)
    st = D.dock_run_state(big, trace=True)
    torch.cuda.synchronize()
    tr = st["trace"].cpu().numpy()
    qs = st["q_stride"]
    nev = st["n_evals"].cpu().numpy()
    assert np.all(nev == 1 + 2 * 4)
    sc = SC.LazyScorer(pk, P.PRESET_TRIDS, weights=G.weights32(P.PRESET_TRIDS).astype(np.float64))
    checked = 0
    for i in mid:
        t = topos[i]
        # every trajectory's first evaluation (its Philox initial pose, drawn
        # by the oracle on its own) against the oracle at that pose
        q0 = SM.initial_q(t, i, 21, np.arange(T))
        ref = sc.score(t, q0)
        c, _, we, wg = G.compare_eval(tr[i, :, 0, 2 * qs], tr[i, :, 0, qs:2 * qs], ref, t.n_dof,
                                      "two per lane init lig %d" % i)
        checked += c
        # the first trajectories coupled with the oracle's own runs
        evlog, mct = SM.EvalLog(8), []
        SM.sample(sc, t, i, SM.SamplerParams(n_traj=8, n_steps=2, n_local=3, seed=21), traj=np.arange(8),
                  trace=mct, evlog=evlog)
        res = CP.compare_run(tr[i, :8], nev[i, :8], evlog, mct, "adam", 3, 0.1, t.n_dof)
        G.say("lig", i, "N", t.n_atoms, "init worst E/tol %.3g g/tol %.3g;" % (we, wg), CP.summary(res))
        assert res["unexplained"] == [], res["unexplained"][:3]
    assert checked >= 0.9 * T * len(mid)
    G.say("two per lane: forms")
    a = _state(D, D.dock_sample(p, H, n_traj=T, form=D.FORM_PLAIN, use_graph=0, **kw))
    b = _state(D, D.dock_sample(p, H, n_traj=T, form=D.FORM_BATCHED, use_graph=0, **kw))
    _same(a, b, "two per lane plain/batched")
    for k in ("q_cur", "E_cur", "q_best", "E_best"):
        assert np.array_equal(a[k], st[k].cpu().numpy()), k


def test_live_runs_share_bucket_streams(D, mixed):
    """Batched runs share their device's pool of bucket streams.  Two live
    runs advanced in interleaved order, and two runs enqueued on different
    streams without a synchronisation between them, reach the states each
    run reaches alone."""
    p, H, L, _ = mixed
    kw = dict(n_traj=16, n_local=3, form=D.FORM_BATCHED)
    G.say("shared streams: references")
    ref_a = _state(D, D.dock_sample(p, H, n_steps=6, seed=31, **kw))
    ref_b = _state(D, D.dock_sample(p, H, n_steps=5, seed=32, **kw))
    assert len(D.dock_run_plan(D.dock_sample(p, H, n_steps=0, seed=31, **kw))["lanes"]) > 1
    G.say("shared streams: interleaved advances")
    a = D.dock_sample(p, H, n_steps=2, seed=31, **kw)
    b = D.dock_sample(p, H, n_steps=2, seed=32, **kw)
    D.dock_run_advance(a, 3)
    D.dock_run_advance(b, 3)
    D.dock_run_advance(a, 1)
    _same(ref_a, _state(D, a), "interleaved a")
    _same(ref_b, _state(D, b), "interleaved b")
    G.say("shared streams: two caller streams")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ra = D.dock_sample(p, H, n_steps=6, seed=31, stream=s1, **kw)
    rb = D.dock_sample(p, H, n_steps=5, seed=32, stream=s2, **kw)
    torch.cuda.synchronize()
    _same(ref_a, _state(D, ra), "stream a")
    _same(ref_b, _state(D, rb), "stream b")


def test_resume_and_restore_bitwise(D, mixed):
    p, H, L, _ = mixed
    kw = dict(n_traj=16, n_local=3, seed=5)
    G.say("resume")
    full = _state(D, D.dock_sample(p, H, n_steps=7, **kw))
    r = D.dock_sample(p, H, n_steps=3, **kw)
    mid = D.dock_run_state(r)
    D.dock_run_advance(r, 4)
    _same(full, _state(D, r), "advance")
    # restore the step-3 state into a fresh run and finish
    r2 = D.dock_sample(p, H, n_steps=0, **kw)
    D.dock_run_set_state(r2, mid["q_cur"], mid["E_cur"], mid["q_best"], mid["E_best"], 3)
    D.dock_run_advance(r2, 4)
    got = _state(D, r2)
    for k in ("q_cur", "E_cur", "q_best", "E_best"):
        assert np.array_equal(full[k], got[k]), k
    # a restarted run (created with 3 steps, advanced to 7) repeats a new
    # 3-step run with that seed, in its own buffers
    G.say("restart")
    for seed in (5, 12):
        D.dock_run_restart(r, seed)
        _same(_state(D, D.dock_sample(p, H, n_steps=3, **dict(kw, seed=seed))), _state(D, r), ("restart", seed))
    rp = D.dock_sample(p, H, n_steps=2, form=D.FORM_PLAIN, **kw)
    D.dock_run_restart(rp, 31)
    _same(_state(D, D.dock_sample(p, H, n_steps=2, form=D.FORM_PLAIN, **dict(kw, seed=31))), _state(D, rp),
          "restart plain")


def test_traced_subset_matches_full_trace(D, mixed):
    """Logging only every second ligand's first three trajectories gives the
    same rows as logging everything, in the documented block order."""
    p, H, L, _ = mixed
    kw = dict(n_traj=8, n_steps=3, n_local=4, seed=4, record_trace=1)
    full = D.dock_run_state(D.dock_sample(p, H, **kw), trace=True)["trace"].cpu().numpy()
    run = D.dock_sample(p, H, trace_lig_stride=2, trace_traj=3, **kw)
    v = run.view()
    assert (v.trace_lig_stride, v.trace_traj, v.n_trace) == (2, 3, 3 * ((L.n_ligands + 1) // 2))
    sub = D.dock_run_state(run, trace=True)["trace"].cpu().numpy()
    assert sub.shape[:2] == ((L.n_ligands + 1) // 2, 3)
    assert np.array_equal(sub, full[::2, :3], equal_nan=True)
    D.dock_run_restart(run, 4)
    again = D.dock_run_state(run, trace=True)["trace"].cpu().numpy()
    assert np.array_equal(again, sub, equal_nan=True)


def test_trace_self_consistency(D):
    pk = tiny_pocket(n=20, radius=6.0, grid=28)
    L = tiny_ligand(9, 3, seed=6)
    L.pocket_index = np.zeros(1, np.int32)
    w = G.weights32(P.PRESET_TRIDS)
    p = G.load_pocket(pk, P.PRESET_TRIDS, w)
    H = G.load_ligands(L)
    T, S, Lc = 8, 4, 5
    G.say("trace adam")
    run = D.dock_sample(p, H, n_traj=T, n_steps=S, n_local=Lc, seed=1, record_trace=1)
    st = D.dock_run_state(run, trace=True)
    tr = st["trace"].cpu().numpy()[0]           # [T, cap, 2*qs+1]
    qs = st["q_stride"]
    n_dof = 6 + H.max_tors
    rows = tr.reshape(-1, 2 * qs + 1)
    q = torch.tensor(rows[:, :qs].copy(), device="cuda")
    E, g, _ = D.dock_score_grad(p, H, torch.zeros(len(rows), dtype=torch.int32, device="cuda"), q)
    np.testing.assert_allclose(E.cpu().numpy(), rows[:, 2 * qs], rtol=1e-6, atol=1e-5)
    np.testing.assert_allclose(g.cpu().numpy()[:, :n_dof], rows[:, qs:qs + n_dof], rtol=1e-5, atol=1e-4)
    topo = topology.from_ligands(L, 0)
    # Adam rule between consecutive rows of one MC step (FP64 recomputation)
    for t in range(T):
        for s in range(S):
            base = 1 + s * (Lc + 1)
            m = np.zeros(n_dof); v = np.zeros(n_dof)
            for k in range(Lc):
                qk = tr[t, base + k, :n_dof].astype(np.float64)
                gk = tr[t, base + k, qs:qs + n_dof].astype(np.float64)
                m = 0.9 * m + 0.1 * gk
                v = 0.999 * v + 0.001 * gk * gk
                step = 0.1 * (m / (1 - 0.9 ** (k + 1))) / (np.sqrt(v / (1 - 0.999 ** (k + 1))) + 1e-8)
                nxt = qk - step
                nxt[:3] = np.clip(nxt[:3], topo.box_min, topo.box_max)
                nxt[3:] = nxt[3:] - 2 * np.pi * np.floor((nxt[3:] + np.pi) / (2 * np.pi))
                got = tr[t, base + k + 1, :n_dof]
                d = np.abs(np.angle(np.exp(1j * (got - nxt))))
                d[:3] = np.abs(got[:3] - nxt[:3])
                assert d.max() < 2e-4, (t, s, k, d.max())


def test_best_poses_match_oracle(D):
    L = synth.make_ligands(4, lambda r: int(r.integers(8, 40)), lambda r: int(r.integers(0, 8)), seed=31)
    H = G.load_ligands(L)
    rng = np.random.default_rng(7)
    T = 96
    qs = H.q_stride
    Eall = np.zeros((L.n_ligands, T), np.float32)
    Qall = np.zeros((L.n_ligands, T, qs), np.float32)
    topos = []
    for i in range(L.n_ligands):
        t = topology.from_ligands(L, i)
        topos.append(t)
        q = synth.random_poses(t.n_dof, t.box_min, t.box_max, T, rng)
        q[T // 2:] = q[:T // 2] + (rng.normal(size=(T // 2, t.n_dof)) * 0.05).astype(np.float32)
        Qall[i, :, :t.n_dof] = q
        e = rng.normal(size=T).astype(np.float32)
        e[3] = e[7]
        e[11] = np.inf
        Eall[i] = e
    G.say("best poses", L.n_ligands, "ligands x", T)
    out = D.dock_best_poses(H, T, torch.tensor(Eall, device="cuda"), torch.tensor(Qall, device="cuda"),
                            top_n=8, rmsd_cluster=1.0)
    got = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    n_checked = 0
    for i, t in enumerate(topos):
        ref = BEST.best_poses(t, Eall[i].astype(np.float64), Qall[i, :, :t.n_dof].astype(np.float64),
                              top_n=8, rmsd_cut=1.0, margins=True)
        n = len(ref["idx"])
        if ref["rmsd_margin"] > 1e-4:
            n_checked += 1
            assert got["n"][i] == n
            assert list(got["idx"][i, :n]) == list(ref["idx"])
            np.testing.assert_array_equal(got["E"][i, :n], Eall[i][ref["idx"]])
            np.testing.assert_allclose(got["E_screen"][i, :n], ref["E_screen"], rtol=1e-6)
            np.testing.assert_array_equal(got["q"][i, :n, :t.n_dof], Qall[i, ref["idx"], :t.n_dof])
            np.testing.assert_allclose(got["xyz"][i, :n, :t.n_atoms], ref["xyz"], atol=2e-5)
            assert np.all(got["idx"][i, n:] == -1) and np.all(np.isinf(got["E"][i, n:]))
    # a ligand whose clustering has an RMSD within 1e-4 of the cut is skipped
    G.say("best poses: %d of %d ligands checked" % (n_checked, len(topos)))
    assert n_checked >= 3


def _tiny_system(D):
    pk = tiny_pocket(n=20, radius=6.0, grid=28)
    L = tiny_ligand(9, 3, seed=6)
    L.pocket_index = np.zeros(1, np.int32)
    w = G.weights32(P.PRESET_TRIDS)
    p = G.load_pocket(pk, P.PRESET_TRIDS, w)
    H = G.load_ligands(L)
    return pk, L, w, p, H, topology.from_ligands(L, 0)


def _coupled_run(D, kind, local_opt, T, S, n_local, lr, seed):
    """GPU run with its evaluation log and the oracle's own run of the same
    trajectories (same Philox stream), compared row by row."""
    pk, L, w, p, H, topo = _tiny_system(D)
    run = D.dock_sample(p, H, n_traj=T, n_steps=S, n_local=n_local, seed=seed, record_trace=1,
                        local_opt=local_opt, lr=lr)
    st = D.dock_run_state(run, trace=True)
    torch.cuda.synchronize()
    tr = st["trace"].cpu().numpy()[0]
    nev = st["n_evals"].cpu().numpy()[0]
    sc = SC.Scorer(pk, weights=w.astype(np.float64))
    evlog, mct = SM.EvalLog(T), []
    ost = SM.sample(sc, topo, 0, SM.SamplerParams(n_traj=T, n_steps=S, n_local=n_local, seed=seed,
                                                  local_opt=local_opt, lr=lr), trace=mct, evlog=evlog)
    res = CP.compare_run(tr, nev, evlog, mct, kind, n_local, lr, topo.n_dof)
    G.say(kind, CP.summary(res))
    for t, why in res["unexplained"]:
        G.say("  unexplained trajectory", t, why)
    return res, tr, nev, evlog, st, ost, topo


def test_linesearch_coupled_with_oracle(D):
    """The Armijo line search (the alternative local rule): GPU and oracle
    trajectories share every random number and are compared evaluation by
    evaluation (pose, energy, gradient); a parting must follow a decision
    within its tolerance band; whole trajectories make the same number of
    evaluations.  On the GPU's own log, every trial's accept / reject
    follows the Armijo test E_trial <= E + 1e-4 alpha (g . d) with d = -g/|g|
    and alpha = 2^-j, and each search ends at its first accepted trial."""
    T, S, nl = 32, 4, 3
    res, tr, nev, evlog, st, ost, topo = _coupled_run(D, "linesearch", D.LOCAL_LINESEARCH, T, S, nl, 0.1, 1)
    assert res["unexplained"] == []
    assert res["whole"] >= T // 2
    whole_n = [t for t in range(T) if len(evlog.rows[t]) == nev[t]]
    assert len(whole_n) >= res["whole"]
    n_trials = n_acc = n_band = 0
    for t in range(T):
        a, b, c = CP.check_linesearch_log(tr[t], int(nev[t]), topo.n_dof, nl, topo.box_min, topo.box_max)
        n_trials, n_acc, n_band = n_trials + a, n_acc + b, n_band + c
    G.say("line search on the GPU log: %d trials, %d accepted, %d within FP32 of the threshold"
          % (n_trials, n_acc, n_band))
    assert n_acc > 0 and n_trials > n_acc


def test_adam_trajectories_coupled(D):
    """Adam refinement (the paper's local rule): GPU and oracle trajectories
    compared evaluation by evaluation; every parting is explained by a
    decision margin (Metropolis, a step direction an FP32 gradient error can
    turn, a cell face or cutoff) or is gradual drift."""
    T, S = 32, 3
    res, tr, nev, evlog, st, ost, topo = _coupled_run(D, "adam", D.LOCAL_ADAM, T, S, 10, 0.1, 4)
    assert res["unexplained"] == []
    assert res["whole"] >= T // 2
    Eb = st["E_best"].cpu().numpy()[0]
    rel = np.abs(Eb - ost.E_best) / np.maximum(1.0, np.abs(ost.E_best))
    G.say("coupled Adam: best energies within 1e-3 for %d of %d" % (np.sum(rel < 1e-3), T))


def test_best_energy_and_rmsd_distributions_over_seeds(D):
    """The 600-atom-pocket / 24-atom-ligand workload, 4 seeds x 64 trajectories
    x 100 MC steps: GPU best energies and RMSDs versus the oracle's."""
    from scipy.stats import ks_2samp
    gold = json.load(open(os.path.join(HERE, "golden", "c1_best_distribution.json")))
    pk, L, wl = synth.workload("C1")
    w = G.weights32(P.PRESET_TRIDS)
    p = G.load_pocket(pk[0], P.PRESET_TRIDS, w)
    H = G.load_ligands(L)
    topo = topology.from_ligands(L, 0)
    Eg, Rg = [], []
    for s in gold["seeds"]:
        G.say("distribution seed", s)
        run = D.dock_sample(p, H, n_traj=gold["n_traj"], n_steps=gold["n_steps"], n_local=gold["n_local"],
                            seed=s)
        st = D.dock_run_state(run)
        qb = st["q_best"][0]
        E, _, xyz = D.dock_score_grad(p, H, torch.zeros(qb.shape[0], dtype=torch.int32, device="cuda"),
                                      qb.contiguous(), want_grad=False, want_xyz=True)
        x = xyz.cpu().numpy()[:, :topo.n_atoms]
        Eg.append(st["E_best"].cpu().numpy()[0])
        Rg.append(np.sqrt(np.mean(np.sum((x - topo.x0[None]) ** 2, axis=2), axis=1)))
    Eg, Rg = np.concatenate(Eg), np.concatenate(Rg)
    Eo, Ro = np.concatenate(gold["E_best"]), np.concatenate(gold["rmsd"])
    pE = ks_2samp(Eg, Eo).pvalue
    pR = ks_2samp(Rg, Ro).pvalue
    # bootstrap CI of the median difference
    rng = np.random.default_rng(0)
    diffs = [np.median(rng.choice(Eg, len(Eg))) - np.median(rng.choice(Eo, len(Eo))) for _ in range(2000)]
    lo, hi = np.percentile(diffs, [2.5, 97.5])
    G.say("KS p(E) %.3g p(RMSD) %.3g; median E gpu %.3f oracle %.3f; CI of diff [%.3f, %.3f]"
          % (pE, pR, np.median(Eg), np.median(Eo), lo, hi))
    assert pE >= 0.01 and pR >= 0.01
    assert lo <= 0.0 <= hi


def test_autotuner_keeps_random_streams_and_runs(D, mixed):
    p, H, L, _ = mixed
    kw = dict(n_traj=16, n_local=3, seed=12)
    D.dock_autotune_clear()
    G.say("autotune")
    base = _state(D, D.dock_sample(p, H, n_steps=0, **kw))
    rep = D.dock_autotune(p, H, trial_steps=1, n_steps=2, **kw)
    G.say("autotune report", rep)
    assert len(rep) >= 3 and all(r["block"] in (64, 128, 256) for r in rep)
    tuned = _state(D, D.dock_sample(p, H, n_steps=0, **kw))
    # initial poses come from the (ligand, trajectory) Philox stream only
    assert np.array_equal(base["q_cur"], tuned["q_cur"])
    run = D.dock_sample(p, H, n_steps=3, **kw)
    st = _state(D, run)
    assert np.all(st["n_evals"] == 1 + 3 * 4) and np.all(np.isfinite(st["E_best"]))
    D.dock_autotune_clear()


@pytest.mark.parametrize("opt", ["SGD", "RMSPROP", "ADAGRAD", "ADAMW"])
def test_optimizer_variants_update_rules(D, opt):
    """The Table S5 alternatives: every recorded step follows the update rule
    (FP64 recomputation from the logged gradients), lr 0.02."""
    pk = tiny_pocket(n=20, radius=6.0, grid=28)
    L = tiny_ligand(9, 3, seed=6)
    L.pocket_index = np.zeros(1, np.int32)
    w = G.weights32(P.PRESET_TRIDS)
    p = G.load_pocket(pk, P.PRESET_TRIDS, w)
    H = G.load_ligands(L)
    T, S, Lc, lr = 8, 3, 4, 0.02
    kind = getattr(D, "LOCAL_" + opt)
    G.say("optimizer", opt)
    run = D.dock_sample(p, H, n_traj=T, n_steps=S, n_local=Lc, seed=2, record_trace=1, local_opt=kind, lr=lr)
    st = D.dock_run_state(run, trace=True)
    tr = st["trace"].cpu().numpy()[0]
    qs = st["q_stride"]
    n = 6 + H.max_tors
    topo = topology.from_ligands(L, 0)
    for t in range(T):
        for s in range(S):
            base = 1 + s * (Lc + 1)
            m = np.zeros(n); v = np.zeros(n)
            for k in range(Lc):
                q = tr[t, base + k, :n].astype(np.float64)
                g = tr[t, base + k, qs:qs + n].astype(np.float64)
                if opt == "SGD":
                    step = lr * g
                elif opt == "RMSPROP":
                    v = 0.99 * v + 0.01 * g * g
                    step = lr * g / (np.sqrt(v) + 1e-8)
                elif opt == "ADAGRAD":
                    v = v + g * g
                    step = lr * g / (np.sqrt(v) + 1e-8)
                else:
                    q = q * (1 - lr * 0.01)
                    m = 0.9 * m + 0.1 * g
                    v = 0.999 * v + 0.001 * g * g
                    step = lr * (m / (1 - 0.9 ** (k + 1))) / (np.sqrt(v / (1 - 0.999 ** (k + 1))) + 1e-8)
                nxt = q - step
                nxt[:3] = np.clip(nxt[:3], topo.box_min, topo.box_max)
                got = tr[t, base + k + 1, :n]
                d = np.abs(np.angle(np.exp(1j * (got - nxt))))
                d[:3] = np.abs(got[:3] - nxt[:3])
                tol = 2e-4 * (1 + np.abs(step).max()) if opt == "SGD" else 2e-4
                assert d.max() < tol, (opt, t, s, k, d.max())
    # the same rule in the oracle's sampler: trajectories coupled row by row
    res = _coupled_run(D, opt.lower(), kind, 16, S, Lc, 0.002, 2)[0]
    assert res["unexplained"] == []
    assert res["whole"] >= 8


@pytest.mark.parametrize("n,k,stride", [(0, 5, 1), (1, 1, 1), (100, 37, 3), (2048, 1024, 1),
                                        (2049, 1024, 2), (70000, 300, 1)])
def test_screen_rank_matches_oracle(D, n, k, stride):
    G.say("screen rank n", n, "k", k, "stride", stride)
    rng = np.random.default_rng(n + k)
    v = rng.normal(size=n * stride).astype(np.float32)
    # ties, signed zeros, infinities and NaNs
    special = rng.choice(np.array([-1.0, -0.0, 0.0, np.inf, -np.inf, np.nan], np.float32), size=v.shape)
    v = np.where(rng.random(v.shape) < 0.2, special, v).astype(np.float32)
    if n > 0:
        v[::7] = np.float32(0.25)
    s, idx = D.dock_screen_rank(torch.tensor(v, device="cuda"), k, stride=stride)
    torch.cuda.synchronize()
    rs, ridx = BEST.screen_rank(v[::stride][:n].astype(np.float64), k)
    assert np.array_equal(idx.cpu().numpy(), ridx.astype(np.int32))
    np.testing.assert_array_equal(s.cpu().numpy(), rs.astype(np.float32))
