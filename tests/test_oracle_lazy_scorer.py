"""Pin of the oracle's lazily filled grid scorer (CPU).

`score.LazyScorer` computes a map node by the same brute-force pair sum as
`maps.build_maps`, but only when a pose first reads it; the large parity
cases use it because a full 64^3 x 8 map costs minutes in numpy.  Here it is
pinned to `score.Scorer` (maps built for every node up front), itself pinned
by the node / linear-field / convergence / finite-difference tests of
test_oracle_maps_score.py: energies, DOF gradients, atom gradients, the
absolute-sum scale and the margins must be bit-identical, for both term
presets, for poses inside, across and outside the map box, and for a second
scoring call that reuses nodes filled by the first.
"""
import numpy as np
import pytest

import synth
from oracle import topology, score as SC, params as P
from tests import _gpu as G


@pytest.mark.parametrize("preset", [P.PRESET_TRIDS, P.PRESET_VINA])
def test_lazy_scorer_equals_full_scorer(preset):
    pk = synth.make_pocket(60, radius=8.0, grid=22, seed=11)
    L = synth.make_ligands(3, lambda r: int(r.integers(8, 16)), lambda r: int(r.integers(1, 5)),
                           seed=13, center_jitter=0.5)
    w = np.asarray(P.default_weights(preset), np.float32).astype(np.float64)
    full = SC.Scorer(pk, preset, weights=w)
    lazy = SC.LazyScorer(pk, preset, weights=w)
    rng = np.random.default_rng(17)
    checked = 0
    for i in range(L.n_ligands):
        topo = topology.from_ligands(L, i)
        for kind in ("uniform", "near", "outside"):
            q = G.poses_for(topo, 24, rng, kind).astype(np.float64)
            a = full.score(topo, q)
            b = lazy.score(topo, q)
            for k in ("E", "dEdq", "g", "S_abs", "margin", "margin_E"):
                assert np.array_equal(a[k], b[k]), (preset, i, kind, k)
            checked += len(q)
    # a second pass reads nodes the first pass filled: still identical
    topo = topology.from_ligands(L, 0)
    q = G.poses_for(topo, 24, np.random.default_rng(17), "uniform").astype(np.float64)
    assert np.array_equal(full.score(topo, q)["E"], lazy.score(topo, q)["E"])
    # the lazy maps hold exactly the full maps' values wherever they were filled
    filled = lazy.lazy.done
    assert filled.any() and not filled.all()
    assert np.array_equal(lazy.M[:, filled], full.M[:, filled])
    assert checked == 3 * 3 * 24
