"""Pair functions phi_k(d) of the scoring function, FP64 (oracle side).

TRIDS physics preset (Methods, "Scoring functions": E_long, E_clash, E_Hbond):
  long : -exp(-(s - 3)^2 / 4),  s = d - (R_i + R_j)            d < 10
  clash: -log(max(d, 0.1) / d_clash)                            d < d_clash
  hbond: -exp(-(d - 2.88)^2 / (2 * 0.3^2))     donor/acceptor,  d < 3.4
The printed exponents of E_long and E_Hbond lack the minus sign; they are
read as decaying Gaussians (otherwise the sums diverge).  E_long's (mu,
sigma) are "as in Vina": Vina's second Gaussian, offset 3 A, width 2 A.

Vina-form preset (five terms, cutoff 8 A, s = surface distance):
  gauss1 = exp(-(s/0.5)^2), gauss2 = exp(-((s-3)/2)^2), repulsion = s^2 (s<0),
  hydrophobic = 1 (s<0.5) .. linear .. 0 (s>=1.5), both atoms hydrophobic,
  hbond = 1 (s<-0.7) .. linear .. 0 (s>=0), donor/acceptor pairs.

Each function returns (value, d value / d d).  Cutoffs are NOT applied here:
the caller decides which pairs are inside each term's cutoff (see
`params.term_cutoffs`) and in which precision that decision is taken.
"""
import numpy as np
from . import params as P


def _gauss(x, two_sig2):
    v = np.exp(-(x * x) / two_sig2)
    return v, v * (-2.0 * x / two_sig2)


def trids_long(d, rsum):
    s = d - rsum
    v, dv = _gauss(s - P.TRIDS_LONG_MU, P.TRIDS_LONG_2SIG2)
    return -v, -dv


def trids_clash(d, dclash):
    dd = np.maximum(d, P.CLASH_DMIN)
    v = -np.log(dd / dclash)
    dv = np.where(d > P.CLASH_DMIN, -1.0 / dd, 0.0)
    return v, dv


def trids_hbond(d):
    v, dv = _gauss(d - P.TRIDS_HB_MU, 2.0 * P.TRIDS_HB_SIGMA ** 2)
    return -v, -dv


def vina_gauss1(s):
    return _gauss(s, 0.25)          # (s/0.5)^2 = s^2/0.25


def vina_gauss2(s):
    return _gauss(s - 3.0, 4.0)     # ((s-3)/2)^2


def vina_repulsion(s):
    neg = s < 0.0
    return np.where(neg, s * s, 0.0), np.where(neg, 2.0 * s, 0.0)


def vina_hydrophobic(s):
    v = np.where(s < 0.5, 1.0, np.where(s < 1.5, 1.5 - s, 0.0))
    dv = np.where((s >= 0.5) & (s < 1.5), -1.0, 0.0)
    return v, dv


def vina_hbond(s):
    v = np.where(s < -0.7, 1.0, np.where(s < 0.0, -s / 0.7, 0.0))
    dv = np.where((s >= -0.7) & (s < 0.0), -1.0 / 0.7, 0.0)
    return v, dv


def phi(preset, k, d, ti, tj):
    """Term k of `preset` for pairs at distance d (arrays), types ti, tj (ints)."""
    d = np.asarray(d, np.float64)
    rsum = P.radius(ti) + P.radius(tj)
    if preset == P.PRESET_TRIDS:
        if k == 0:
            return trids_long(d, rsum)
        if k == 1:
            dcl = P.TRIDS_CLASH_DHB if P.hbond_pair(ti, tj) else rsum
            return trids_clash(d, dcl)
        return trids_hbond(d)
    s = d - rsum
    return (vina_gauss1, vina_gauss2, vina_repulsion, vina_hydrophobic,
            vina_hbond)[k](s)


def pair_energy_terms(preset, d, ti, tj, within):
    """Per-term values and derivatives for one type pair.

    within[k]: boolean array, True where the pair is inside term k's cutoff
    (None when the term does not apply to this type pair).
    Returns (vals [K, ...], dvals [K, ...]).
    """
    K = P.n_terms(preset)
    d = np.asarray(d, np.float64)
    vals = np.zeros((K,) + d.shape)
    dvals = np.zeros((K,) + d.shape)
    for k in range(K):
        if within[k] is None:
            continue
        v, dv = phi(preset, k, d, ti, tj)
        vals[k] = np.where(within[k], v, 0.0)
        dvals[k] = np.where(within[k], dv, 0.0)
    return vals, dvals


def within_fp64(preset, d, ti, tj):
    """Cutoff decisions taken on the FP64 distance (ligand-internal pairs)."""
    cuts = P.term_cutoffs(preset, ti, tj)
    return [None if c is None else (np.asarray(d) < c) for c in cuts]


def within_fp32(preset, d2_f32, ti, tj):
    """Cutoff decisions taken on an FP32 squared distance.

    Used for map nodes, where both the node and the receptor atom are exact
    FP32 numbers: the decision is d2 < fl32(c)*fl32(c), with d2 and the
    product evaluated in FP32, so the GPU library and the oracle include
    exactly the same receptor atoms at every node.
    """
    cuts = P.term_cutoffs(preset, ti, tj)
    out = []
    for c in cuts:
        if c is None:
            out.append(None)
        else:
            c32 = np.float32(c)
            out.append(np.asarray(d2_f32, np.float32) < np.float32(c32 * c32))
    return out


def d2_fp32(a, b):
    """Squared distance in FP32, fixed order ((dx*dx + dy*dy) + dz*dz)."""
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    dx = (a[..., 0] - b[..., 0]).astype(np.float32)
    dy = (a[..., 1] - b[..., 1]).astype(np.float32)
    dz = (a[..., 2] - b[..., 2]).astype(np.float32)
    return ((dx * dx + dy * dy) + dz * dz).astype(np.float32)
