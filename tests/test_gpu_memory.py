"""Device memory comes back: repeated cycles of loading a pocket and
ligands, sampling (batched form, graph replay), best poses, the
deterministic adjoint and freeing every handle leave the device's free
memory where the first cycle left it."""
import gc

import numpy as np
import pytest

import synth
from oracle import params as P
from tests import _gpu as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G.lib()


def _cycle(D, pk, L, w):
    p = G.load_pocket(pk, P.PRESET_TRIDS, w, keep=True)
    H = G.load_ligands(L)
    run = D.dock_sample(p, H, n_traj=64, n_steps=4, seed=3, form=D.FORM_BATCHED)
    st = D.dock_run_state(run)
    best = D.dock_best_poses(H, 64, st["E_best"], st["q_best"], top_n=4)
    wt = torch.tensor(w, device="cuda").reshape(1, -1)
    lig = torch.arange(L.n_ligands, dtype=torch.int32, device="cuda")
    G_maps = D.dock_pocket_maps(p, per_term=True)
    dG = torch.zeros_like(G_maps)
    dw = torch.zeros_like(wt)
    D.dock_score_adjoint(p, H, lig, wt, torch.ones(L.n_ligands, device="cuda"), q=best["q"][:, 0].contiguous(),
                         G=[G_maps], dLdG=[dG], dLdw=dw, deterministic=1)
    torch.cuda.synchronize()
    e_sum = float(best["E"][:, 0].sum())
    run.free()
    H.free()
    p.free()
    del run, H, p, st, best, G_maps, dG, dw, wt, lig
    gc.collect()
    torch.cuda.synchronize()
    return e_sum


def test_load_sample_adjoint_free_cycles_return_device_memory(D):
    pk = synth.make_pocket(800, grid=48, seed=6)
    L = synth.pack_ligands([synth.make_ligand(n, t, np.random.default_rng(110 + n)) for n, t in
                            ((9, 1), (21, 4), (40, 7), (58, 9), (67, 5))])
    L.pocket_index = np.zeros(L.n_ligands, np.int32)
    w = G.weights32(P.PRESET_TRIDS)
    first = _cycle(D, pk, L, w)
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]
    for k in range(6):
        assert _cycle(D, pk, L, w) == first          # same seed, same result
    torch.cuda.empty_cache()
    free1 = torch.cuda.mem_get_info()[0]
    G.say("free device memory after 6 more cycles: %+.1f MiB" % ((free1 - free0) / 2**20))
    # one cycle holds ~10 MiB of maps alone: a leak of any handle's buffers
    # over six cycles would show
    assert free1 >= free0 - 8 * 2**20
