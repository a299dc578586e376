"""Adjoint of the receptor grid-map build, FP64 (oracle side).

Test infrastructure only: the GPU library never imports it.

For the TRIDS preset (Methods, "Scoring functions"), the per-term maps

    G[t][k][node] = sum_i phi_k(|node - r_i|; t, u_i)

depend on the receptor coordinates r_i and on the term constants

    theta = (mu_long, sigma_long, mu_hb, sigma_hb, d_clash_hb, R_0 .. R_7)

through
    E_long : -exp(-(s - mu_long)^2 / (2 sigma_long^2)),  s = d - R_t - R_u,  d < 10
    E_clash: -log(max(d, 0.1) / d_c),  d_c = d_clash_hb for a donor/acceptor
             pair, else R_t + R_u,  d < d_c
    E_Hbond: -exp(-(d - mu_hb)^2 / (2 sigma_hb^2)),  donor/acceptor,  d < 3.4
(the Vina-like width of E_long, 2 A, is sigma_long = sqrt(2)).  Given
lam = dL/dG for a loss L, `map_adjoint` returns dL/dr_i and dL/dtheta by the
chain rule through every (node, receptor atom) pair inside the cutoffs.

Cutoff decisions are those of the map build (FP32 squared distance against
fl32(c)^2, see maps.py).  The fixed cutoffs (10 A, 3.4 A) are not
differentiated: the terms jump there and a derivative exists only away from
them.  d_c moves its own cutoff, where the clash term is zero, so moving it
adds nothing beyond the term's own derivative.
"""
import math
import numpy as np
from scipy.spatial import cKDTree

from . import params as P
from . import maps as MAPS
from . import terms

N_THETA = 5 + P.N_TYPES
THETA_NAMES = ("mu_long", "sigma_long", "mu_hb", "sigma_hb", "d_clash_hb") + tuple(
    "R_" + n for n in P.TYPE_NAMES)


def default_theta():
    return np.array([P.TRIDS_LONG_MU, math.sqrt(P.TRIDS_LONG_2SIG2 / 2.0), P.TRIDS_HB_MU,
                     P.TRIDS_HB_SIGMA, P.TRIDS_CLASH_DHB] + [P.radius(t) for t in range(P.N_TYPES)])


def _pairs(pocket, idx, reach):
    """(node index, receptor index) pairs within `reach` of each other."""
    pts = MAPS.node_coords(pocket.origin, pocket.spacing, pocket.dims, idx)
    # values from the coordinates as given (FP32 inputs are exact in FP64);
    # the cutoff decisions round them to FP32 like the map build
    rec = np.asarray(pocket.xyz, np.float64)
    nb = cKDTree(rec).query_ball_point(pts, reach)
    pi = np.repeat(np.arange(len(pts)), [len(v) for v in nb])
    ri = np.concatenate([np.asarray(v, np.int64) for v in nb]) if len(pi) else np.zeros(0, np.int64)
    return pts, rec, pi, ri


def _cut32(c):
    c32 = np.float32(c)
    return np.float32(c32 * c32)


def _chunks(total, chunk):
    for s in range(0, total, chunk):
        yield np.arange(s, min(total, s + chunk))


def map_terms(pocket, theta, chunk=20000, decide=None):
    """TRIDS per-term maps [8, 3, n_nodes] at constants theta (the map build of
    maps.py with the constants made explicit).  `decide` (default theta)
    gives the constants the clash cutoff decisions are taken with: holding
    them fixed turns the maps into smooth functions of theta, whose
    derivative is what map_adjoint returns (a decision that d_c moves flips a
    term that is zero at the cutoff)."""
    th = np.asarray(theta, np.float64)
    mu_l, sig_l, mu_h, sig_h, dc_hb = th[:5]
    R = th[5:]
    thd = th if decide is None else np.asarray(decide, np.float64)
    Rd = thd[5:]
    nx, ny, nz = pocket.dims
    total = nx * ny * nz
    out = np.zeros((8, 3, total))
    rtype = np.asarray(pocket.type, np.int64)
    for idx in _chunks(total, chunk):
        pts, rec, pi, ri = _pairs(pocket, idx, P.TRIDS_LONG_DMAX + 1e-3)
        if len(pi) == 0:
            continue
        d = np.sqrt(np.sum((pts[pi] - rec[ri]) ** 2, axis=1))
        d2f = terms.d2_fp32(pts[pi].astype(np.float32), rec[ri].astype(np.float32))
        u = rtype[ri]
        for t in range(8):
            hb = np.array([P.hbond_pair(t, x) for x in range(8)])[u]
            s = d - R[t] - R[u]
            x = s - mu_l
            v0 = np.where(d2f < _cut32(P.TRIDS_LONG_DMAX), -np.exp(-x * x / (2 * sig_l ** 2)), 0.0)
            dc = np.where(hb, dc_hb, R[t] + R[u])
            dcd = np.where(hb, thd[4], Rd[t] + Rd[u])
            inside_c = d2f < np.array([_cut32(c) for c in dcd], np.float32)
            v1 = np.where(inside_c, -np.log(np.maximum(d, P.CLASH_DMIN) / dc), 0.0)
            xh = d - mu_h
            v2 = np.where(hb & (d2f < _cut32(P.TRIDS_HB_DMAX)), -np.exp(-xh * xh / (2 * sig_h ** 2)), 0.0)
            for k, v in enumerate((v0, v1, v2)):
                out[t, k, idx] += np.bincount(pi, weights=v, minlength=len(idx))
    return out


def map_adjoint(pocket, lam, theta=None, chunk=20000):
    """dL/dr [n_rec, 3] and dL/dtheta [13] for lam = dL/dG [8, 3, n_nodes]."""
    th = default_theta() if theta is None else np.asarray(theta, np.float64)
    mu_l, sig_l, mu_h, sig_h, dc_hb = th[:5]
    R = th[5:]
    lam = np.asarray(lam, np.float64).reshape(8, 3, -1)
    nx, ny, nz = pocket.dims
    total = nx * ny * nz
    rtype = np.asarray(pocket.type, np.int64)
    n_rec = len(rtype)
    dr = np.zeros((n_rec, 3))
    dth = np.zeros(N_THETA)
    for idx in _chunks(total, chunk):
        pts, rec, pi, ri = _pairs(pocket, idx, P.TRIDS_LONG_DMAX + 1e-3)
        if len(pi) == 0:
            continue
        diff = rec[ri] - pts[pi]
        d = np.sqrt(np.sum(diff ** 2, axis=1))
        unit = np.where(d[:, None] > 0, diff / np.where(d > 0, d, 1.0)[:, None], 0.0)
        d2f = terms.d2_fp32(pts[pi].astype(np.float32), rec[ri].astype(np.float32))
        u = rtype[ri]
        dphi = np.zeros(len(pi))       # sum_t,k lam * dphi/dd per pair
        for t in range(8):
            l0, l1, l2 = (lam[t, k, idx][pi] for k in range(3))
            hb = np.array([P.hbond_pair(t, x) for x in range(8)])[u]
            # long
            inside = d2f < _cut32(P.TRIDS_LONG_DMAX)
            x = d - R[t] - R[u] - mu_l
            g = np.where(inside, np.exp(-x * x / (2 * sig_l ** 2)), 0.0)
            dphi += l0 * g * x / sig_l ** 2
            dth[0] += np.sum(l0 * -g * x / sig_l ** 2)
            dth[1] += np.sum(l0 * -g * x * x / sig_l ** 3)
            dR = l0 * -g * x / sig_l ** 2
            dth[5 + t] += np.sum(dR)
            np.add.at(dth, 5 + u, dR)
            # clash
            dc = np.where(hb, dc_hb, R[t] + R[u])
            inside = d2f < np.array([_cut32(c) for c in dc], np.float32)
            dd = np.maximum(d, P.CLASH_DMIN)
            dphi += np.where(inside & (d > P.CLASH_DMIN), l1 * -1.0 / dd, 0.0)
            ddc = np.where(inside, l1 / dc, 0.0)
            dth[4] += np.sum(np.where(hb, ddc, 0.0))
            dRc = np.where(hb, 0.0, ddc)
            dth[5 + t] += np.sum(dRc)
            np.add.at(dth, 5 + u, dRc)
            # hydrogen bond
            inside = hb & (d2f < _cut32(P.TRIDS_HB_DMAX))
            xh = d - mu_h
            gh = np.where(inside, np.exp(-xh * xh / (2 * sig_h ** 2)), 0.0)
            dphi += l2 * gh * xh / sig_h ** 2
            dth[2] += np.sum(l2 * -gh * xh / sig_h ** 2)
            dth[3] += np.sum(l2 * -gh * xh * xh / sig_h ** 3)
        np.add.at(dr, ri, dphi[:, None] * unit)
    return dr, dth


def fixed_cutoff_margin(pocket):
    """Per receptor atom, the smallest |d - c| over nodes and the fixed cutoffs
    (10 A, 3.4 A): a finite difference of size h on r_i is valid only when it
    stays well below this."""
    nx, ny, nz = pocket.dims
    total = nx * ny * nz
    rec_n = len(pocket.type)
    m = np.full(rec_n, np.inf)
    for idx in _chunks(total, 20000):
        pts, rec, pi, ri = _pairs(pocket, idx, P.TRIDS_LONG_DMAX + 0.5)
        if len(pi) == 0:
            continue
        d = np.sqrt(np.sum((rec[ri] - pts[pi]) ** 2, axis=1))
        mm = np.minimum(np.abs(d - P.TRIDS_LONG_DMAX), np.abs(d - P.TRIDS_HB_DMAX))
        np.minimum.at(m, ri, mm)
    return m
