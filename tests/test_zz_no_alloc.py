"""GPU test of dock_screen_rank_noalloc, the screening rank that allocates
nothing (its passes run in a static per-device scratch array).

Two calls in a row, the second on a smaller input, each compared bit for bit
with dock_screen_rank (which allocates its scratch) and with the oracle's
lexsort; then the size limit of the static scratch.  Outputs are allocated
before the calls, so the library call itself runs without an allocation.
"""
import numpy as np
import pytest

from oracle import best as BEST
from tests import _gpu as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G.lib()


def _scores(n, stride, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=n * stride).astype(np.float32)
    special = rng.choice(np.array([-1.0, -0.0, 0.0, np.inf, -np.inf, np.nan], np.float32), size=v.shape)
    v = np.where(rng.random(v.shape) < 0.2, special, v).astype(np.float32)
    v[::5] = np.float32(0.5)  # ties
    return v


def test_noalloc_rank_matches_allocating_rank_twice(D):
    cases = [(300_000, 512, 2, 11), (40_000, 100, 1, 12)]  # second call: smaller input
    out_s = torch.empty(1024, dtype=torch.float32, device="cuda")
    out_i = torch.empty(1024, dtype=torch.int32, device="cuda")
    for n, k, stride, seed in cases:
        G.say("noalloc rank n", n, "k", k, "stride", stride)
        v = _scores(n, stride, seed)
        dv = torch.tensor(v, device="cuda")
        out_s.fill_(123.0)
        out_i.fill_(-7)
        torch.cuda.synchronize()
        D.dock_screen_rank_noalloc(dv, k, out_s, out_i, stride=stride)
        ref_s, ref_i = D.dock_screen_rank(dv, k, stride=stride)
        torch.cuda.synchronize()
        gs, gi = out_s[:k].cpu().numpy(), out_i[:k].cpu().numpy()
        assert np.array_equal(gi, ref_i.cpu().numpy())
        assert np.array_equal(gs.view(np.uint32), ref_s.cpu().numpy().view(np.uint32))
        os_, oi = BEST.screen_rank(v[::stride][:n].astype(np.float64), k)
        assert np.array_equal(gi, oi.astype(np.int32))
        np.testing.assert_array_equal(gs, os_.astype(np.float32))
        # entries past top_k are not written
        assert np.all(out_i[k:].cpu().numpy() == -7)


def test_noalloc_rank_single_block_and_limit(D):
    out_s = torch.empty(8, dtype=torch.float32, device="cuda")
    out_i = torch.empty(8, dtype=torch.int32, device="cuda")
    v = _scores(2048, 1, 13)
    dv = torch.tensor(v, device="cuda")
    D.dock_screen_rank_noalloc(dv, 8, out_s, out_i)
    ref_s, ref_i = D.dock_screen_rank(dv, 8)
    torch.cuda.synchronize()
    assert np.array_equal(out_i.cpu().numpy(), ref_i.cpu().numpy())
    # 2^20 + 1 scores in 513 blocks x 1024 kept > 262,144 scratch entries
    big = torch.zeros((1 << 20) + 1, dtype=torch.float32, device="cuda")
    out_s = torch.empty(1024, dtype=torch.float32, device="cuda")
    out_i = torch.empty(1024, dtype=torch.int32, device="cuda")
    with pytest.raises(D.DockError) as ei:
        D.dock_screen_rank_noalloc(big, 1024, out_s, out_i)
    assert ei.value.code == -3
    # the same scores with a smaller top_k fit
    D.dock_screen_rank_noalloc(big, 16, out_s, out_i)
    torch.cuda.synchronize()
    assert np.array_equal(out_i[:16].cpu().numpy(), np.arange(16, dtype=np.int32))
