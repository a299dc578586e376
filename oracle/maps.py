"""Receptor grid maps, brute force in FP64 (oracle side).

The paper sums the physics terms over receptor-ligand atom pairs within a
cutoff (Methods, E_long / E_clash / E_Hbond; Discussion item 4, the cutoff
pair kernel).  Those terms depend on the ligand atom only through its type,
so Sum_receptor phi_k(|p - r_i|) can be tabulated per ligand type on a
lattice.  A map node is defined as exactly that pair sum at the node:

  G[t][k][node] = sum_{receptor i inside cutoff_k} phi_k(|node - r_i|; t, type_i)
  M[t]          = sum_k w_k G[t][k]

Nodes: origin + h * (ix, iy, iz); layout [t][k][iz][iy][ix].  Node and
receptor coordinates are exact FP32 numbers; the inside-cutoff decision is
taken on the FP32 squared distance (see terms.within_fp32), the values in FP64.
"""
import numpy as np
from scipy.spatial import cKDTree

from . import params as P
from . import terms


def node_coords(origin, spacing, dims, idx):
    """FP64 coordinates of flat node indices idx (x fastest)."""
    nx, ny, nz = dims
    idx = np.asarray(idx, np.int64)
    ix = idx % nx
    iy = (idx // nx) % ny
    iz = idx // (nx * ny)
    o = np.asarray(origin, np.float64)
    return np.stack([o[0] + spacing * ix, o[1] + spacing * iy, o[2] + spacing * iz], axis=1)


def node_values(rec_xyz, rec_type, points, preset, ligand_types=range(8),
                decision="fp32"):
    """Per-term pair sums at `points` [n,3] for each ligand type.

    Returns [len(ligand_types), K, n].  decision="fp32" takes the cutoff
    decision on FP32 squared distances (exact FP32 points), "fp64" on FP64
    distances (arbitrary points, the direct pairwise mode).
    """
    rec = np.asarray(rec_xyz, np.float32).astype(np.float64)
    rtype = np.asarray(rec_type).astype(np.int64)
    pts = np.asarray(points, np.float64)
    K = P.n_terms(preset)
    ltypes = list(ligand_types)
    out = np.zeros((len(ltypes), K, len(pts)))
    cmax = P.TRIDS_LONG_DMAX if preset == P.PRESET_TRIDS else P.VINA_CUTOFF
    tree = cKDTree(rec)
    nb = tree.query_ball_point(pts, cmax + 1e-3)
    pi = np.repeat(np.arange(len(pts)), [len(v) for v in nb])
    ri = np.concatenate([np.asarray(v, np.int64) for v in nb]) if len(pi) else np.zeros(0, np.int64)
    if len(pi) == 0:
        return out
    d = np.sqrt(np.sum((pts[pi] - rec[ri]) ** 2, axis=1))
    if decision == "fp32":
        d2f = terms.d2_fp32(pts[pi].astype(np.float32), rec[ri].astype(np.float32))
    for a, t in enumerate(ltypes):
        for tr in range(P.N_TYPES):
            sel = rtype[ri] == tr
            if not np.any(sel):
                continue
            if decision == "fp32":
                within = terms.within_fp32(preset, d2f[sel], t, tr)
            else:
                within = terms.within_fp64(preset, d[sel], t, tr)
            vals, _ = terms.pair_energy_terms(preset, d[sel], t, tr, within)
            for k in range(K):
                out[a, k] += np.bincount(pi[sel], weights=vals[k], minlength=len(pts))
    return out


def build_maps(pocket, preset, nodes=None, chunk=20000):
    """Per-term maps G [8, K, nz, ny, nx] (or [8, K, len(nodes)] for a subset)."""
    nx, ny, nz = pocket.dims
    total = nx * ny * nz
    idx = np.arange(total) if nodes is None else np.asarray(nodes, np.int64)
    K = P.n_terms(preset)
    out = np.zeros((8, K, len(idx)))
    for s in range(0, len(idx), chunk):
        pts = node_coords(pocket.origin, pocket.spacing, pocket.dims, idx[s:s + chunk])
        out[:, :, s:s + chunk] = node_values(pocket.xyz, pocket.type, pts, preset)
    if nodes is None:
        return out.reshape(8, K, nz, ny, nx)
    return out


def combine(G, weights):
    """M[t] = sum_k w_k G[t][k]."""
    w = np.asarray(weights, np.float64)
    return np.einsum("k,tk...->t...", w, G)
