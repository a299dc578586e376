"""Differentiable form: gradients of summed scores, FP64 (oracle side).

The score is linear in the per-term maps and in the weights:
  E(G, w, q) = sum_i sum_k w_k trilerp(G[t_i][k], x_i(q)) + E_out(x)
             + sum_pairs sum_k w_k phi_k(r_ij)
so for L = sum_p dL/dE_p * E_p:
  dL/dG[t][k][node] = sum over atoms i of type t whose cell has `node` as a
                      corner of dL/dE_p * w_k * (trilinear corner weight),
  dL/dw_k           = sum_p dL/dE_p * (sum_i trilerp(G[t_i][k], x_i) + sum_pairs phi_k),
  dL/dx_i           = dL/dE_p * dE/dx_i,   dL/dq = dL/dE_p * dE/dq.
The paper differentiates the score only w.r.t. ligand coordinates for
sampling (Methods, after E_dock; Discussion item 3); the map and weight
adjoints extend the same linear structure.
"""
import numpy as np

from . import params as P
from . import terms
from . import fk as FK
from .score import trilerp, corner_weights


def per_term_intra(topo, preset, x):
    """Per-term intra sums [P, K] and per-term atom gradients [K, P, N, 3]."""
    K = P.n_terms(preset)
    Pn = x.shape[0]
    Ek = np.zeros((Pn, K))
    gk = np.zeros((K,) + x.shape)
    for i, j in topo.pairs:
        ti, tj = int(topo.types[i]), int(topo.types[j])
        r = x[:, i] - x[:, j]
        d = np.sqrt(np.sum(r * r, axis=1))
        within = terms.within_fp64(preset, d, ti, tj)
        vals, dvals = terms.pair_energy_terms(preset, d, ti, tj, within)
        Ek += vals.T
        f = (dvals / d)[:, :, None] * r[None]
        gk[:, :, i] += f
        gk[:, :, j] -= f
    return Ek, gk


def forward_terms(G, grid, preset, topo, x):
    """Per-term energies [P, K] (inter + intra) and E_out [P] for coordinates x."""
    K = P.n_terms(preset)
    Pn, N, _ = x.shape
    Ek = np.zeros((Pn, K))
    eout = np.zeros(Pn)
    for a in range(N):
        t = int(topo.types[a])
        for k in range(K):
            v, _, eo, _, _, _ = trilerp(G[t, k], grid, x[:, a])
            Ek[:, k] += v
        eout += eo
    Ei, _ = per_term_intra(topo, preset, x)
    return Ek + Ei, eout


def energy(G, w, grid, preset, topo, q=None, x=None):
    if x is None:
        x = FK.fk(topo, q)
    Ek, eout = forward_terms(G, grid, preset, topo, x)
    return Ek @ np.asarray(w, np.float64) + eout


def adjoint(G, w, grid, preset, topo, dLdE, q=None, x=None):
    """Returns dict(dLdG [8,K,nz,ny,nx], dLdw [K], dLdx [P,N,3], dLdq [P,n_dof] or None)."""
    w = np.asarray(w, np.float64)
    dLdE = np.asarray(dLdE, np.float64)
    if x is None:
        x = FK.fk(topo, q)
    Pn, N, _ = x.shape
    K = P.n_terms(preset)
    dLdG = np.zeros_like(G, dtype=np.float64)
    nx, ny, nz = grid.dims
    dLdw = np.zeros(K)
    gat = np.zeros_like(x)
    for a in range(N):
        t = int(topo.types[a])
        for k in range(K):
            v, g, eo, go, _, (c, f) = trilerp(G[t, k], grid, x[:, a])
            dLdw[k] += np.sum(dLdE * v)
            gat[:, a] += w[k] * g
            for dx, dy, dz, cw in corner_weights(f):
                np.add.at(dLdG[t, k], (c[:, 2] + dz, c[:, 1] + dy, c[:, 0] + dx),
                          dLdE * w[k] * cw)
        gat[:, a] += go
    Ei, gi = per_term_intra(topo, preset, x)
    dLdw += dLdE @ Ei
    gat += np.einsum("k,kpnc->pnc", w, gi)
    dLdx = dLdE[:, None, None] * gat
    dLdq = None if q is None else dLdE[:, None] * FK.dof_gradient(topo, q, x, gat)
    return dict(dLdG=dLdG, dLdw=dLdw, dLdx=dLdx, dLdq=dLdq)
