"""Pins of the oracle's maps, interpolation and score (CPU).

* grid value at a node == the direct pairwise sum at that node;
* trilinear interpolation exact on linear fields (value and gradient);
* O(h^2) convergence on a smooth field;
* additivity of the maps over receptor subsets;
* dE/dq against central finite differences on tiny systems;
* rigid-motion invariance of the direct (pairwise) score;
* grid-aligned translation and cube-rotation invariance of the grid score.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from oracle import topology, maps as MAPS, score as SC, fk as FK, params as P
from tests._tiny import tiny_pocket, tiny_ligand


def test_node_values_equal_direct_sum():
    pk = tiny_pocket(n=30, radius=7.0, grid=20)
    rng = np.random.default_rng(0)
    nodes = rng.integers(0, 20 ** 3, 200)
    for preset in (P.PRESET_TRIDS, P.PRESET_VINA):
        G = MAPS.build_maps(pk, preset, nodes=nodes)          # [8, K, n]
        pts = MAPS.node_coords(pk.origin, pk.spacing, pk.dims, nodes)
        for t in range(8):
            # a one-atom ligand of type t placed at each node, scored pairwise
            ds = SC.DirectScorer(pk.xyz, pk.type, preset, weights=np.eye(P.n_terms(preset))[0])
            for k in range(P.n_terms(preset)):
                ds.weights = np.eye(P.n_terms(preset))[k]
                e, _ = ds.inter_atoms([t], pts[:, None, :])
                np.testing.assert_allclose(G[t, k], e[:, 0], rtol=1e-12, atol=1e-12)


def test_trilerp_exact_on_linear_fields():
    grid = SC.Grid(np.array([-3.0, -2.0, -1.5]), 0.375, (11, 9, 13))
    a = np.array([0.7, -1.3, 2.1]); b = 0.4
    nx, ny, nz = grid.dims
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = np.stack([grid.origin[0] + 0.375 * ix, grid.origin[1] + 0.375 * iy, grid.origin[2] + 0.375 * iz], -1)
    M = X @ a + b
    rng = np.random.default_rng(1)
    p = grid.lo + (grid.hi - grid.lo) * rng.random((500, 3))
    v, g, eo, go, _, _ = SC.trilerp(M, grid, p)
    np.testing.assert_allclose(v, p @ a + b, atol=1e-12)
    np.testing.assert_allclose(g, np.broadcast_to(a, g.shape), atol=1e-12)
    assert np.all(eo == 0)
    # outside: value at the clamped point, penalty 10 * L1 distance
    q = np.array([[grid.hi[0] + 0.5, 0.0, 0.0]])
    v, g, eo, go, _, _ = SC.trilerp(M, grid, q)
    np.testing.assert_allclose(v, np.clip(q, grid.lo, grid.hi) @ a + b, atol=1e-12)
    np.testing.assert_allclose(eo, 5.0)
    np.testing.assert_allclose(go[0], [10.0, 0.0, 0.0])
    assert g[0, 0] == 0.0


def test_trilerp_second_order_convergence():
    f = lambda X: np.sin(0.8 * X[..., 0]) * np.cos(0.5 * X[..., 1]) + 0.3 * np.sin(0.6 * X[..., 2])
    rng = np.random.default_rng(2)
    p = rng.uniform(-2.0, 2.0, (2000, 3))
    errs = []
    for h in (0.4, 0.2, 0.1):
        n = int(round(8.0 / h)) + 1
        grid = SC.Grid(np.array([-4.0, -4.0, -4.0]), h, (n, n, n))
        ax = -4.0 + h * np.arange(n)
        Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
        M = f(np.stack([X, Y, Z], -1))
        v, *_ = SC.trilerp(M, grid, p)
        errs.append(np.max(np.abs(v - f(p))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5


def test_maps_additive_over_receptor_subsets():
    pk = tiny_pocket(n=30, radius=7.0, grid=16)
    idx = np.arange(30)
    A = synth.Pocket(pk.xyz[idx < 13], pk.type[idx < 13], pk.origin, pk.spacing, pk.dims, pk.radius)
    B = synth.Pocket(pk.xyz[idx >= 13], pk.type[idx >= 13], pk.origin, pk.spacing, pk.dims, pk.radius)
    G = MAPS.build_maps(pk, P.PRESET_TRIDS)
    np.testing.assert_allclose(G, MAPS.build_maps(A, P.PRESET_TRIDS) + MAPS.build_maps(B, P.PRESET_TRIDS),
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("preset", [P.PRESET_TRIDS, P.PRESET_VINA])
def test_score_gradient_finite_differences(preset):
    pk = tiny_pocket(n=20, radius=6.0, grid=28)
    sc = SC.Scorer(pk, preset)
    rng = np.random.default_rng(3)
    for seed in range(4):
        L = tiny_ligand(n_atoms=6, n_tors=2, seed=seed)
        topo = topology.from_ligands(L, 0)
        q = synth.random_poses(topo.n_dof, topo.box_min, topo.box_max, 16, rng).astype(np.float64)
        r = sc.score(topo, q)
        keep = r["margin"] > 1e-3
        assert keep.sum() >= 8
        h = 1e-6
        for d in range(topo.n_dof):
            qp = q.copy(); qm = q.copy(); qp[:, d] += h; qm[:, d] -= h
            fd = (sc.energy(topo, qp) - sc.energy(topo, qm)) / (2 * h)
            np.testing.assert_allclose(r["dEdq"][keep, d], fd[keep], rtol=1e-5, atol=1e-4)


def _euler_of(R):
    return Rotation.from_matrix(R).as_euler("ZYX")


def test_direct_score_rigid_motion_invariance():
    pk = tiny_pocket(n=20, radius=6.0)
    L = tiny_ligand(n_atoms=6, n_tors=2, seed=7)
    d = L.ligand(0)
    topo = topology.from_ligands(L, 0)
    rng = np.random.default_rng(4)
    R0 = Rotation.random(random_state=5).as_matrix()
    t0 = np.array([1.5, -2.0, 0.7])
    ds = SC.DirectScorer(pk.xyz, pk.type)
    ds2 = SC.DirectScorer(pk.xyz.astype(np.float64) @ R0.T + t0, pk.type)
    xyz2 = d["xyz"].astype(np.float64) @ R0.T + t0
    topo2 = topology.build(d["element"], d["n_h"], xyz2.astype(np.float32), d["bonds"], d["rotatable"])
    # use the exact FP64 moved coordinates in the moved topology
    topo2.x0 = topo.x0 @ R0.T + t0
    topo2.c0 = topo.c0 @ R0.T + t0
    q = synth.random_poses(topo.n_dof, topo.box_min, topo.box_max, 6, rng).astype(np.float64)
    q2 = q.copy()
    R, _, _ = FK.euler_zyx(q[:, 3], q[:, 4], q[:, 5])
    q2[:, 0:3] = q[:, 0:3] @ R0.T + t0
    # world rotation R' with R' (R0 y) = R0 R y for local vectors -> R' = R0 R R0^T
    q2[:, 3:6] = _euler_of(R0[None] @ R @ R0.T[None])
    r1 = ds.score(topo, q)
    r2 = ds2.score(topo2, q2)
    np.testing.assert_allclose(FK.fk(topo2, q2), FK.fk(topo, q) @ R0.T + t0, atol=1e-10)
    np.testing.assert_allclose(r2["E"], r1["E"], rtol=1e-10, atol=1e-9)
    np.testing.assert_allclose(r2["dEdq"][:, 0:3], r1["dEdq"][:, 0:3] @ R0.T, rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(r2["dEdq"][:, 6:], r1["dEdq"][:, 6:], rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(r2["g"], r1["g"] @ R0.T, rtol=1e-8, atol=1e-8)


def test_grid_score_translation_and_cube_rotation_invariance():
    pk = tiny_pocket(n=20, radius=6.0, grid=24)
    sc = SC.Scorer(pk)
    L = tiny_ligand(n_atoms=6, n_tors=2, seed=8)
    topo = topology.from_ligands(L, 0)
    rng = np.random.default_rng(6)
    q = synth.random_poses(topo.n_dof, topo.box_min, topo.box_max, 8, rng).astype(np.float64)
    x = FK.fk(topo, q)
    e0 = sc.inter(topo.types, x)[0].sum(1)
    # grid-aligned translation of receptor, grid and ligand by 3 nodes in y
    s = np.array([0.0, 3 * pk.spacing, 0.0])
    pk2 = synth.Pocket((pk.xyz + s).astype(np.float32), pk.type, (pk.origin + s).astype(np.float32),
                       pk.spacing, pk.dims, pk.radius)
    sc2 = SC.Scorer(pk2)
    # receptor + shift rounds to FP32, so agreement is to FP32 input precision
    np.testing.assert_allclose(sc2.inter(topo.types, x + s)[0].sum(1), e0, rtol=1e-5, atol=1e-4)
    # 90 degree rotation about z of receptor and ligand (grid is centred, cubic)
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    pk3 = synth.Pocket((pk.xyz @ Rz.T).astype(np.float32), pk.type, pk.origin, pk.spacing, pk.dims,
                       pk.radius)
    sc3 = SC.Scorer(pk3)
    np.testing.assert_allclose(sc3.inter(topo.types, x @ Rz.T)[0].sum(1), e0, rtol=1e-12, atol=1e-10)
