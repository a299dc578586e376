"""Helpers shared by the GPU tests: load synthetic inputs through the C ABI
and compare against the oracle with the parity tolerances.

Tolerances (per evaluation, FP32 GPU vs FP64 oracle):
  |E - E_ref| <= 1e-5 * max(|E_ref|, S_abs)      S_abs = sum of |per-atom|
                                                   and |per-pair| energies
  ||g - g_ref||_2 <= 1e-4 * ||g_ref||_2 (+1e-4 absolute floor)
The energy is compared unless a pair sits within MARGIN of a hard cutoff
(where E itself jumps); the gradient is compared unless some decision
(cell face, box face, cutoff, kink of a piecewise term) lies within MARGIN.
FP32 and FP64 atom positions differ by a few 1e-6 A; MARGIN = 3e-5 A.
"""
import sys

import numpy as np

import synth
from oracle import topology, score as SC, params as P

E_RTOL = 1e-5
G_RTOL = 1e-4
MARGIN = 3e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lib():
    import paper_2510_24186_amd as D
    return D


def load_pocket(pk, preset=P.PRESET_TRIDS, weights=None, keep=False, direct=False, residue=None):
    D = lib()
    return D.dock_load_pocket(pk.xyz, pk.type, pk.origin, pk.spacing, pk.dims, preset=preset,
                              weights=weights, keep_per_term=keep,
                              inter_mode=D.INTER_DIRECT if direct else D.INTER_GRID, residue=residue)


def load_ligands(L, host_only=False):
    D = lib()
    return D.dock_load_ligands(L.atom_off, L.element, L.n_h, L.xyz, L.bond_off, L.bonds,
                               L.rotatable, pocket_index=L.pocket_index, host_only=host_only)


def weights32(preset):
    return np.asarray(P.default_weights(preset), np.float32)


def poses_for(topo, n, rng, kind="uniform"):
    """Seeded pose draws for one ligand (inputs only)."""
    if kind == "uniform":
        return synth.random_poses(topo.n_dof, topo.box_min, topo.box_max, n, rng)
    q = np.zeros((n, topo.n_dof))
    q[:, 0:3] = topo.c0 + rng.normal(size=(n, 3)) * 0.5
    q[:, 3:6] = rng.normal(size=(n, 3)) * 0.3
    q[:, 6:] = rng.normal(size=(n, topo.n_dof - 6)) * 0.5
    if kind == "outside":
        q[:, 0] += 30.0
    return q.astype(np.float32)


def compare_eval(E, g, ref, n_dof, tag=""):
    """Returns (n_checked, n_margin_skipped, worst E ratio, worst g ratio)."""
    Er, gr = ref["E"], ref["dEdq"][:, :n_dof]
    scale = np.maximum(np.abs(Er), ref["S_abs"])
    e_ratio = np.abs(E - Er) / (E_RTOL * scale + 1e-30)
    gn = np.linalg.norm(gr, axis=1)
    g_ratio = np.linalg.norm(g[:, :n_dof] - gr, axis=1) / (G_RTOL * gn + 1e-4)
    ok_margin = ref["margin"] > MARGIN
    ok_e = ref["margin_E"] > MARGIN
    bad = (ok_e & (e_ratio > 1)) | (ok_margin & (g_ratio > 1))
    # poses within the bound only thanks to the absolute floor (reported)
    dg = np.linalg.norm(g[:, :n_dof] - gr, axis=1)
    floor_only = ok_margin & (dg > G_RTOL * gn) & (g_ratio <= 1)
    if np.any(floor_only):
        say("%s: %d of %d poses within the gradient bound only by its 1e-4 floor (|g| %s, |dg| %s)"
            % (tag, int(floor_only.sum()), int(ok_margin.sum()), np.array2string(gn[floor_only][:4], precision=3),
               np.array2string(dg[floor_only][:4], precision=3)))
    if np.any(bad):
        i = int(np.flatnonzero(bad)[0])
        raise AssertionError(
            "%s pose %d: E %r vs %r (S_abs %r) ratio %.3g; |dg|/|g| ratio %.3g; margin %.3g"
            % (tag, i, float(E[i]), float(Er[i]), float(ref["S_abs"][i]), e_ratio[i], g_ratio[i],
               ref["margin"][i]))
    return int(ok_margin.sum()), int((~ok_margin).sum()), float(e_ratio[ok_e].max(initial=0)), \
        float(g_ratio[ok_margin].max(initial=0))
