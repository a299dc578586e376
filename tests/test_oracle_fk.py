"""Pins of the oracle's forward kinematics and chain rule (CPU).

Rotation conventions against scipy's Rotation; geometric invariants of the
torsion tree; the chain rule against central finite differences of a test
energy with a known coordinate gradient.
"""
import numpy as np
from scipy.spatial.transform import Rotation

import synth
from oracle import topology, fk as FK


def _ligs():
    return synth.make_ligands(12, lambda r: int(r.integers(5, 40)), lambda r: int(r.integers(0, 10)),
                              seed=21)


def _rand_q(topo, n, rng):
    return synth.random_poses(topo.n_dof, topo.box_min, topo.box_max, n, rng).astype(np.float64)


def test_euler_is_intrinsic_zyx():
    rng = np.random.default_rng(0)
    a, b, g = rng.uniform(-np.pi, np.pi, (3, 20))
    R, _, _ = FK.euler_zyx(a, b, g)
    ref = Rotation.from_euler("ZYX", np.stack([a, b, g], 1)).as_matrix()
    np.testing.assert_allclose(R, ref, atol=1e-14)


def test_axis_rotation_is_rodrigues():
    rng = np.random.default_rng(1)
    u = rng.normal(size=3); u /= np.linalg.norm(u)
    th = rng.uniform(-np.pi, np.pi, 10)
    ref = Rotation.from_rotvec(u[None] * th[:, None]).as_matrix()
    np.testing.assert_allclose(FK.rot_axis(u, th), ref, atol=1e-14)


def test_zero_dofs_reproduce_input():
    L = _ligs()
    for i in range(L.n_ligands):
        topo = topology.from_ligands(L, i)
        q = np.zeros((1, topo.n_dof)); q[0, :3] = topo.c0
        np.testing.assert_allclose(FK.fk(topo, q)[0], topo.x0, atol=1e-12)


def test_bond_lengths_and_rigid_fragments_invariant():
    L = _ligs()
    rng = np.random.default_rng(2)
    for i in range(L.n_ligands):
        d = L.ligand(i)
        topo = topology.from_ligands(L, i)
        x = FK.fk(topo, _rand_q(topo, 5, rng))
        for a, b in d["bonds"]:
            ref = np.linalg.norm(topo.x0[a] - topo.x0[b])
            np.testing.assert_allclose(np.linalg.norm(x[:, a] - x[:, b], axis=1), ref, rtol=1e-12)
        for f in range(topo.n_frags):
            idx = np.flatnonzero(topo.atom_frag == f)
            D0 = np.linalg.norm(topo.x0[idx, None] - topo.x0[None, idx], axis=-1)
            D = np.linalg.norm(x[:, idx, None] - x[:, None, idx], axis=-1)
            np.testing.assert_allclose(D, np.broadcast_to(D0, D.shape), atol=1e-11)


def test_two_pi_periodicity():
    L = _ligs()
    rng = np.random.default_rng(3)
    topo = topology.from_ligands(L, 3)
    q = _rand_q(topo, 4, rng)
    for d in range(3, topo.n_dof):
        q2 = q.copy(); q2[:, d] += 2 * np.pi
        np.testing.assert_allclose(FK.fk(topo, q2), FK.fk(topo, q), atol=1e-11)


def test_torsion_moves_only_its_subtree_and_keeps_axis():
    L = _ligs()
    rng = np.random.default_rng(4)
    for i in range(L.n_ligands):
        topo = topology.from_ligands(L, i)
        q = _rand_q(topo, 3, rng)
        x = FK.fk(topo, q)
        for k in range(topo.n_tors):
            q2 = q.copy(); q2[:, 6 + k] += 0.7
            x2 = FK.fk(topo, q2)
            m = topo.subtree_atoms(k)
            np.testing.assert_allclose(x2[:, ~m], x[:, ~m], atol=1e-12)
            b = topo.tors_b[k]
            np.testing.assert_allclose(x2[:, b], x[:, b], atol=1e-12)
            if m.sum() > 1:
                assert np.max(np.abs(x2[:, m] - x[:, m])) > 1e-3


def test_chain_rule_against_finite_differences():
    # E(x) = sum_i c_i . x_i + 0.5 sum_i s_i |x_i|^2 ; dE/dx_i = c_i + s_i x_i
    L = _ligs()
    rng = np.random.default_rng(5)
    for i in range(L.n_ligands):
        topo = topology.from_ligands(L, i)
        c = rng.normal(size=(topo.n_atoms, 3))
        s = rng.uniform(0.1, 1.0, topo.n_atoms)
        E = lambda q: (FK.fk(topo, q) * c).sum((1, 2)) + 0.5 * (s * (FK.fk(topo, q) ** 2).sum(2)).sum(1)
        q = _rand_q(topo, 3, rng)
        x = FK.fk(topo, q)
        g = c[None] + s[None, :, None] * x
        an = FK.dof_gradient(topo, q, x, g)
        h = 1e-6
        for d in range(topo.n_dof):
            qp = q.copy(); qm = q.copy(); qp[:, d] += h; qm[:, d] -= h
            fd = (E(qp) - E(qm)) / (2 * h)
            np.testing.assert_allclose(an[:, d], fd, rtol=1e-6, atol=1e-5)
