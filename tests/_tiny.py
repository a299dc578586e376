"""Tiny seeded systems shared by the CPU tests (inputs only)."""
import numpy as np
import synth


def tiny_pocket(n=20, radius=6.0, grid=24, seed=3):
    return synth.make_pocket(n, radius=radius, grid=grid, seed=seed)


def tiny_ligand(n_atoms=6, n_tors=2, seed=5):
    rng = np.random.default_rng(seed)
    return synth.pack_ligands([synth.make_ligand(n_atoms, n_tors, rng)])
