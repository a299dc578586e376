"""Edge cases of the C ABI on the GPU: calls over zero poses write nothing,
a zero-step advance leaves a run untouched, and best-pose selection with
more output slots than trajectories pads the unused ones (E = +inf,
idx = -1) while the used ones match the oracle's selection."""
import numpy as np
import pytest

import synth
from oracle import best as BEST, params as P, topology

from tests import _gpu as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SENTINEL = 7.25


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G.lib()


@pytest.fixture(scope="module")
def tiny(D):
    pk = synth.make_pocket(300, grid=32, seed=3)
    L = synth.pack_ligands([synth.make_ligand(n, t, np.random.default_rng(50 + n)) for n, t in
                            ((5, 1), (12, 3), (20, 4))])
    L.pocket_index = np.zeros(L.n_ligands, np.int32)
    w = G.weights32(P.PRESET_TRIDS)
    p = G.load_pocket(pk, P.PRESET_TRIDS, w, keep=True)
    return L, p, G.load_ligands(L), w


def _full(shape, dtype=torch.float32):
    return torch.full(shape, SENTINEL, dtype=dtype, device="cuda")


def test_zero_poses_write_nothing(D, tiny):
    L, p, H, w = tiny
    G.say("zero-pose calls")
    qs = H.q_stride
    arr, npk = D.binding._pocket_array(p)
    lig = torch.zeros(4, dtype=torch.int32, device="cuda")
    q = torch.zeros((4, qs), device="cuda")
    E, g, xyz = _full((4,)), _full((4, qs)), _full((4, H.max_atoms, 3))
    rc = D.lib.dock_score_grad(arr, npk, H.handle, 0, lig.data_ptr(), q.data_ptr(), qs, E.data_ptr(),
                               g.data_ptr(), xyz.data_ptr(), 3 * H.max_atoms, None)
    assert rc == 0
    wt = torch.tensor(w, device="cuda").reshape(1, -1)
    rc = D.lib.dock_score_terms(arr, npk, H.handle, 0, lig.data_ptr(), q.data_ptr(), qs, None, 0, None,
                                wt.data_ptr(), E.data_ptr(), None)
    assert rc == 0
    dLdE = torch.ones(4, device="cuda")
    dLdw, dLdq = _full((1, wt.shape[1])), _full((4, qs))
    n_nodes = int(np.prod(p.dims)) * 8 * wt.shape[1]
    dLdG = _full((n_nodes,))
    for det in (0, 1):
        rc = D.lib.dock_score_adjoint(arr, npk, H.handle, 0, lig.data_ptr(), q.data_ptr(), qs, None, 0, None,
                                      wt.data_ptr(), dLdE.data_ptr(), D.binding._ptr_array([dLdG], 1),
                                      dLdw.data_ptr(), dLdq.data_ptr(), None, det, None)
        assert rc == 0
    torch.cuda.synchronize()
    for t in (E, g, xyz, dLdw, dLdq, dLdG):
        assert bool(torch.all(t == SENTINEL))
    # a negative count is an argument error, and still writes nothing
    rc = D.lib.dock_score_grad(arr, npk, H.handle, -1, lig.data_ptr(), q.data_ptr(), qs, E.data_ptr(),
                               g.data_ptr(), xyz.data_ptr(), 3 * H.max_atoms, None)
    assert rc == -1 and b"negative" in D.lib.dock_last_error()
    torch.cuda.synchronize()
    assert bool(torch.all(E == SENTINEL))


def test_zero_step_advance_leaves_the_run_untouched(D, tiny):
    L, p, H, w = tiny
    G.say("zero-step advance")
    for form in (D.FORM_PLAIN, D.FORM_BATCHED):
        run = D.dock_sample(p, H, n_traj=32, n_steps=3, seed=5, form=form)
        before = D.dock_run_state(run)
        D.dock_run_advance(run, 0)
        after = D.dock_run_state(run)
        torch.cuda.synchronize()
        assert after["step"] == before["step"] == 3
        for k in ("q_cur", "E_cur", "q_best", "E_best", "n_evals"):
            assert torch.equal(before[k], after[k]), (form, k)
        run.free()


def test_best_poses_pad_unused_slots(D, tiny):
    L, p, H, w = tiny
    T, top_n = 4, 8
    G.say("best poses with", top_n, "slots over", T, "trajectories")
    run = D.dock_sample(p, H, n_traj=T, n_steps=4, seed=9)
    st = D.dock_run_state(run)
    out = D.dock_best_poses(H, T, st["E_best"], st["q_best"], top_n=top_n)
    torch.cuda.synchronize()
    E, idx, n = out["E"].cpu().numpy(), out["idx"].cpu().numpy(), out["n"].cpu().numpy()
    Eb, qb = st["E_best"].cpu().numpy(), st["q_best"].cpu().numpy()
    checked = 0
    for i in range(L.n_ligands):
        t = topology.from_ligands(L, i)
        assert 1 <= n[i] <= T
        assert np.all(np.isinf(E[i, n[i]:])) and np.all(E[i, n[i]:] > 0) and np.all(idx[i, n[i]:] == -1)
        # the kept poses: the oracle's greedy selection over the same
        # candidates (same FP32 energies; RMSDs in FP64 from the same q),
        # unless an RMSD lies within 1e-4 A of the clustering cut
        ref = BEST.best_poses(t, Eb[i].astype(np.float64), qb[i][:, :t.n_dof].astype(np.float64), top_n=top_n,
                              rmsd_cut=1.0, w_tor=0.01, margins=True)
        if ref["rmsd_margin"] > 1e-4:
            assert list(idx[i, :n[i]]) == list(ref["idx"]), (i, idx[i], ref["idx"])
            np.testing.assert_array_equal(E[i, :n[i]], Eb[i][ref["idx"]])
            checked += 1
    assert checked >= 2
    run.free()
