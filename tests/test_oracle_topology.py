"""Pins of the oracle's typing, fragments, torsion tree and pair list (CPU).

Fragments and bond distances are checked against scipy's graph routines;
the root choice against brute force over every fragment; typing against
hand-typed molecules.
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components, shortest_path

import synth
from oracle import topology, atomtype as AT


def _line(n):
    xyz = np.stack([np.arange(n) * 1.5, np.zeros(n), np.zeros(n)], 1).astype(np.float32)
    xyz[1::2, 1] = 0.8
    return xyz


def test_typing_hand_cases():
    # ethanol heavy atoms C-C-O: CH3 (C only) -> C_H, CH2 (bonded to O) -> C_P, OH -> O_DA
    t = AT.type_atoms([0, 0, 2], [3, 2, 1], [(0, 1), (1, 2)])
    assert list(t) == [AT.C_H, AT.C_P, AT.O_DA]
    # dimethyl ether C-O-C: O without H -> O_A
    assert list(AT.type_atoms([0, 2, 0], [3, 0, 3], [(0, 1), (1, 2)])) == [AT.C_P, AT.O_A, AT.C_P]
    # trimethylamine: N with 3 heavy neighbours and no H -> N_P
    t = AT.type_atoms([1, 0, 0, 0], [0, 3, 3, 3], [(0, 1), (0, 2), (0, 3)])
    assert t[0] == AT.N_P
    # N with 2 heavy neighbours, no H (imine-like) -> acceptor N_A
    assert AT.type_atoms([0, 1, 0], [3, 0, 3], [(0, 1), (1, 2)])[1] == AT.N_A
    # NH2 -> donor N_D ; chloro -> Cl_H
    t = AT.type_atoms([0, 1, 3], [2, 2, 0], [(0, 1), (0, 2)])
    assert list(t) == [AT.C_P, AT.N_D, AT.CL_H]


def _check_topology(topo, bonds, rot):
    n = topo.n_atoms
    b = np.asarray(bonds).reshape(-1, 2)
    A = csr_matrix((np.ones(len(b)), (b[:, 0], b[:, 1])), shape=(n, n))
    A = A + A.T
    rigid = b[np.asarray(rot) == 0]
    R = csr_matrix((np.ones(len(rigid)), (rigid[:, 0], rigid[:, 1])), shape=(n, n))
    nc, lab = connected_components(R, directed=False)
    assert nc == topo.n_frags
    # same partition, ids ordered by lowest atom index
    first = {}
    for a in range(n):
        first.setdefault(lab[a], len(first))
    assert np.array_equal(np.array([first[l] for l in lab]), topo.atom_frag)
    # pair list = different fragments and >= 4 bonds apart, lexicographic
    sp = shortest_path(A, unweighted=True, directed=False)
    ref = [(i, j) for i in range(n) for j in range(i + 1, n)
           if topo.atom_frag[i] != topo.atom_frag[j] and sp[i, j] >= 4]
    assert [tuple(p) for p in topo.pairs] == ref
    # root minimises the fragment-tree height, lowest id on ties
    F = topo.n_frags
    if F > 1:
        fe = [(topo.atom_frag[i], topo.atom_frag[j]) for (i, j), r in zip(b, rot) if r]
        fe = np.array(fe)
        FA = csr_matrix((np.ones(len(fe)), (fe[:, 0], fe[:, 1])), shape=(F, F))
        ecc = shortest_path(FA, unweighted=True, directed=False).max(axis=1)
        assert topo.root == int(np.flatnonzero(ecc == ecc.min())[0])
        assert topo.height == ecc.min()
    # every torsion's axis joins its child fragment to the parent fragment;
    # parents precede children in BFS order
    pos = {f: i for i, f in enumerate(topo.bfs)}
    for k in range(topo.n_tors):
        f = topo.tors_frag[k]
        p = topo.frag_parent[f]
        assert topo.atom_frag[topo.tors_a[k]] == p
        assert topo.atom_frag[topo.tors_b[k]] == f
        assert pos[p] < pos[f]
        assert topo.frag_tors[f] == k
    # torsion k is the k-th non-root fragment in BFS order
    assert list(topo.tors_frag) == list(topo.bfs[1:])


def test_generated_ligands_against_scipy():
    L = synth.make_ligands(40, lambda r: int(r.integers(3, 40)), lambda r: int(r.integers(0, 12)),
                           seed=11)
    for i in range(L.n_ligands):
        d = L.ligand(i)
        topo = topology.from_ligands(L, i)
        _check_topology(topo, d["bonds"], d["rotatable"])
        np.testing.assert_allclose(topo.c0, d["xyz"][topo.atom_frag == topo.root].astype(np.float64).mean(0))


def test_ring_and_branch_molecule():
    # 6-ring (0..5) with a chain 5-6-7-8 and a branch 7-9-10
    bonds = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0), (5, 6), (6, 7), (7, 8), (7, 9), (9, 10)]
    rot = [0, 0, 0, 0, 0, 0, 1, 1, 0, 1, 0]
    xyz = np.random.default_rng(0).normal(size=(11, 3)).astype(np.float32) * 3
    topo = topology.build([0] * 11, [1] * 11, xyz, bonds, rot)
    assert topo.n_frags == 4 and topo.n_tors == 3
    _check_topology(topo, bonds, rot)


def test_errors():
    xyz = _line(4)
    with pytest.raises(topology.TopologyError):      # rotatable ring bond
        topology.build([0] * 3, [2] * 3, xyz[:3], [(0, 1), (1, 2), (2, 0)], [1, 0, 0])
    with pytest.raises(topology.TopologyError):      # disconnected
        topology.build([0] * 4, [2] * 4, xyz, [(0, 1), (2, 3)], [0, 0])
    with pytest.raises(topology.TopologyError):      # duplicate bond
        topology.build([0] * 2, [2] * 2, xyz[:2], [(0, 1), (1, 0)], [0, 0])
    with pytest.raises(topology.TopologyError):      # NaN coordinate
        bad = xyz.copy(); bad[0, 0] = np.nan
        topology.build([0] * 4, [2] * 4, bad, [(0, 1), (1, 2), (2, 3)], [0, 0, 0])
    with pytest.raises(topology.LimitError):         # too many atoms
        n = 129
        topology.build([0] * n, [2] * n, _line(n), [(i, i + 1) for i in range(n - 1)], [0] * (n - 1))


def test_single_atom_and_rigid_ligands():
    t = topology.build([0], [4], np.zeros((1, 3), np.float32), np.zeros((0, 2)), [])
    assert t.n_frags == 1 and t.n_tors == 0 and len(t.pairs) == 0 and t.n_dof == 6
    t = topology.build([0] * 6, [2] * 6, _line(6), [(i, i + 1) for i in range(5)], [0] * 5)
    assert t.n_frags == 1 and len(t.pairs) == 0      # same fragment -> no intra pairs
