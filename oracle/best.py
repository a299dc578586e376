"""Ranking, clustering and screening score, FP64 (oracle side).

Methods, "Conformation sampling": samples are ranked, clustered to drop
duplicates, and the top N are kept (the PyMOL plugin shows 8 by default,
Section 3.4).  E_screen = E_dock / (1 + w_tor * N_tor), w_tor = 0.01
(Methods, E_screen; Table S6).  Readings: rank by energy, ties to the lower
trajectory id; greedy clustering: a pose is a duplicate when its RMSD to an
already kept pose is below the threshold (1.0 A); RMSD is the plain
heavy-atom RMSD in atom order without superposition (the docking success
criterion of Section 2, "Model evaluation").
"""
import numpy as np

from . import fk as FK


def rmsd(xa, xb):
    xa = np.asarray(xa, np.float64)
    xb = np.asarray(xb, np.float64)
    return np.sqrt(np.mean(np.sum((xa - xb) ** 2, axis=-1), axis=-1))


def screen_score(E, n_tors, w_tor=0.01):
    return np.asarray(E, np.float64) / (1.0 + w_tor * n_tors)


def best_poses(topo, E_best, q_best, top_n=8, rmsd_cut=1.0, w_tor=0.01, margins=False):
    """Returns dict(idx, E, E_screen, q, xyz[, rmsd_margin])."""
    E_best = np.asarray(E_best, np.float64)
    T = len(E_best)
    order = sorted((i for i in range(T) if np.isfinite(E_best[i])), key=lambda i: (E_best[i], i))
    X = FK.fk(topo, q_best) if T else np.zeros((0, topo.n_atoms, 3))
    keep = []
    margin = np.inf
    for i in order:
        if len(keep) == top_n:
            break
        dup = False
        for k in keep:
            r = rmsd(X[i], X[k])
            margin = min(margin, abs(r - rmsd_cut))
            if r < rmsd_cut:
                dup = True
                break
        if not dup:
            keep.append(i)
    keep = np.array(keep, np.int64)
    out = dict(idx=keep, E=E_best[keep], E_screen=screen_score(E_best[keep], topo.n_tors, w_tor),
               q=np.asarray(q_best, np.float64)[keep], xyz=X[keep])
    if margins:
        out["rmsd_margin"] = margin
    return out


def screen_rank(scores, top_k):
    """Cross-ligand screening rank (Methods, E_screen): the top_k lowest
    scores in ascending order, equal scores by lower ligand index, NaN after
    +inf, -0.0 equal to +0.0; slots beyond the number of ligands get +inf and
    -1.  Returns (scores [top_k], ligand indices [top_k])."""
    v = np.asarray(scores, np.float64)
    n = len(v)
    # primary key: the score with NaN ordered last; secondary: the index
    nan = np.isnan(v)
    key = np.where(nan, 0.0, v)
    order = np.lexsort((np.arange(n), key, nan))
    k = min(top_k, n)
    out_s = np.full(top_k, np.inf)
    out_i = np.full(top_k, -1, np.int64)
    out_s[:k] = v[order[:k]]
    out_i[:k] = order[:k]
    return out_s, out_i
