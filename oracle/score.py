"""Energy and gradient of a pose, FP64 (oracle side).

E = E_inter + E_out + E_intra  (E_dock without the learned MDN term, which
needs trained network weights; Methods, E_dock).  The gradient is passed to
the ligand atom coordinates (Methods, after E_dock) and then to the DOFs by
the chain rule (fk.dof_gradient; Discussion item 3, manual derivatives).

E_inter (grid mode): sum_i trilerp(M[t_i], x_i).  Cell = floor((x - o)/h)
  clamped to [0, n-2]; a point on the upper face uses the lower cell with
  fraction 1.  The gradient is the analytic cell-local derivative.  A point
  outside the map box is interpolated at its clamped position and pays
  10 * |x - clamp(x)|_1 (E_out); clamped components get no interpolation
  gradient.
E_inter (direct mode): sum over receptor atoms inside the cutoffs, the
  paper's own pairwise form; used by invariance tests.
E_intra: sum over the intra-ligand pair list of sum_k w_k phi_k(r_ij).

Margins: `margin` is the smallest distance (A) from any decision threshold
the result depends on (cell faces, box faces, pair cutoffs, kinks of the
piecewise terms); `margin_E` only counts thresholds where the energy itself
jumps (hard pair cutoffs).  Two implementations that compute positions in
different precisions can legitimately disagree in the gradient only when
`margin` is below their position error, and in the energy only when
`margin_E` is.
"""
from dataclasses import dataclass
import numpy as np

from . import params as P
from . import terms
from . import fk as FK
from . import maps as MAPS


@dataclass
class Grid:
    origin: np.ndarray      # [3] float64
    spacing: float
    dims: tuple             # (nx, ny, nz)

    @property
    def lo(self):
        return np.asarray(self.origin, np.float64)

    @property
    def hi(self):
        return self.lo + self.spacing * (np.asarray(self.dims) - 1)


def grid_of(pocket):
    return Grid(np.asarray(pocket.origin, np.float64), float(pocket.spacing), tuple(pocket.dims))


def trilerp(M, grid, p):
    """Value, gradient, out-of-box penalty (+gradient) and face margin.

    M: [nz, ny, nx]; p: [n, 3].  Returns (v [n], g [n,3], eout [n],
    gout [n,3], margin [n], corners (cell [n,3] int, frac [n,3])).
    """
    p = np.asarray(p, np.float64)
    h = grid.spacing
    n = np.asarray(grid.dims)
    pc = np.clip(p, grid.lo, grid.hi)
    inside = (p >= grid.lo) & (p <= grid.hi)
    u = (pc - grid.lo) / h
    c = np.clip(np.floor(u).astype(np.int64), 0, n - 2)
    f = u - c
    fx, fy, fz = f[:, 0], f[:, 1], f[:, 2]
    cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
    C = {}
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                C[dx, dy, dz] = M[cz + dz, cy + dy, cx + dx]
    gx = ((1 - fy) * (1 - fz) * (C[1, 0, 0] - C[0, 0, 0]) + fy * (1 - fz) * (C[1, 1, 0] - C[0, 1, 0])
          + (1 - fy) * fz * (C[1, 0, 1] - C[0, 0, 1]) + fy * fz * (C[1, 1, 1] - C[0, 1, 1]))
    gy = ((1 - fx) * (1 - fz) * (C[0, 1, 0] - C[0, 0, 0]) + fx * (1 - fz) * (C[1, 1, 0] - C[1, 0, 0])
          + (1 - fx) * fz * (C[0, 1, 1] - C[0, 0, 1]) + fx * fz * (C[1, 1, 1] - C[1, 0, 1]))
    gz = ((1 - fx) * (1 - fy) * (C[0, 0, 1] - C[0, 0, 0]) + fx * (1 - fy) * (C[1, 0, 1] - C[1, 0, 0])
          + (1 - fx) * fy * (C[0, 1, 1] - C[0, 1, 0]) + fx * fy * (C[1, 1, 1] - C[1, 1, 0]))
    v = 0.0
    for (dx, dy, dz), cv in C.items():
        wx = fx if dx else 1 - fx
        wy = fy if dy else 1 - fy
        wz = fz if dz else 1 - fz
        v = v + wx * wy * wz * cv
    g = np.stack([gx, gy, gz], axis=1) / h * inside
    diff = p - pc
    eout = P.OUT_OF_GRID_K * np.abs(diff).sum(axis=1)
    gout = P.OUT_OF_GRID_K * np.sign(diff)
    ur = (p - grid.lo) / h
    m = np.clip(np.rint(ur), 0, n - 1)
    margin = (np.abs(ur - m) * h).min(axis=1)
    return v, g, eout, gout, margin, (c, f)


def cells(grid, p):
    """Cell index [n,3] (x, y, z) of each point, as trilerp chooses it."""
    p = np.asarray(p, np.float64)
    n = np.asarray(grid.dims)
    pc = np.clip(p, grid.lo, grid.hi)
    return np.clip(np.floor((pc - grid.lo) / grid.spacing).astype(np.int64), 0, n - 2)


def corner_weights(f):
    """Trilinear weights of the 8 cell corners, ordered (dx, dy, dz) loops."""
    fx, fy, fz = f[:, 0], f[:, 1], f[:, 2]
    out = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                out.append((dx, dy, dz, (fx if dx else 1 - fx) * (fy if dy else 1 - fy)
                            * (fz if dz else 1 - fz)))
    return out


def _jumps(preset, ti, tj):
    """Distances where a term of this type pair jumps in value (hard cutoffs
    of terms that are nonzero there; the clash cutoff is continuous)."""
    cuts = P.term_cutoffs(preset, ti, tj)
    if preset == P.PRESET_TRIDS:
        return [c for k, c in enumerate(cuts) if c is not None and k != 1]
    return [P.VINA_CUTOFF]


def _breakpoints(preset, ti, tj):
    """Distances where a term of this type pair jumps or kinks."""
    rs = P.radius(ti) + P.radius(tj)
    bps = [c for c in P.term_cutoffs(preset, ti, tj) if c is not None]
    if preset == P.PRESET_TRIDS:
        bps.append(P.CLASH_DMIN)
    else:
        if P.hydrophobic(ti) and P.hydrophobic(tj):
            bps += [rs + 0.5, rs + 1.5]
        if P.hbond_pair(ti, tj):
            bps += [rs - 0.7, rs]
    return bps


def intra(topo, preset, weights, x):
    """E_intra [P], gradient [P,N,3], per-pair |energy| sum [P], margin [P],
    value-jump margin [P]."""
    x = np.asarray(x, np.float64)
    Pn = x.shape[0]
    E = np.zeros(Pn)
    g = np.zeros_like(x)
    sabs = np.zeros(Pn)
    margin = np.full(Pn, np.inf)
    margin_e = np.full(Pn, np.inf)
    w = np.asarray(weights, np.float64)
    for i, j in topo.pairs:
        ti, tj = int(topo.types[i]), int(topo.types[j])
        r = x[:, i] - x[:, j]
        d = np.sqrt(np.sum(r * r, axis=1))
        within = terms.within_fp64(preset, d, ti, tj)
        vals, dvals = terms.pair_energy_terms(preset, d, ti, tj, within)
        e = w @ vals
        de = w @ dvals
        E += e
        sabs += np.abs(e)
        fij = (de / d)[:, None] * r
        g[:, i] += fij
        g[:, j] -= fij
        for b in _breakpoints(preset, ti, tj):
            margin = np.minimum(margin, np.abs(d - b))
        for b in _jumps(preset, ti, tj):
            margin_e = np.minimum(margin_e, np.abs(d - b))
    return E, g, sabs, margin, margin_e


class Scorer:
    """Grid-mode scorer for one pocket: combined maps + weights + preset."""

    def __init__(self, pocket, preset=P.PRESET_TRIDS, weights=None, G=None):
        self.preset = preset
        self.weights = np.asarray(P.default_weights(preset) if weights is None else weights,
                                  np.float64)
        self.grid = grid_of(pocket)
        self.pocket = pocket
        self.G = MAPS.build_maps(pocket, preset) if G is None else G
        self.M = MAPS.combine(self.G, self.weights)

    def inter(self, types, x):
        Pn, N, _ = x.shape
        e = np.zeros((Pn, N)); g = np.zeros((Pn, N, 3))
        eo = np.zeros((Pn, N)); go = np.zeros((Pn, N, 3))
        mg = np.zeros((Pn, N))
        for a in range(N):
            v, gg, eout, gout, m, _ = trilerp(self.M[int(types[a])], self.grid, x[:, a])
            e[:, a], g[:, a], eo[:, a], go[:, a], mg[:, a] = v, gg, eout, gout, m
        return e, g, eo, go, mg

    def score(self, topo, q, want_parts=False):
        """E [P], dE/dq [P, n_dof] and extras for poses q [P, n_dof]."""
        q = np.atleast_2d(np.asarray(q, np.float64))
        x = FK.fk(topo, q)
        e, g, eo, go, mg = self.inter(topo.types, x)
        Ei, gi, sabs_i, mi, mie = intra(topo, self.preset, self.weights, x)
        E = e.sum(1) + eo.sum(1) + Ei
        gat = g + go + gi
        dq = FK.dof_gradient(topo, q, x, gat)
        out = dict(E=E, dEdq=dq, x=x, g=gat,
                   S_abs=np.abs(e).sum(1) + eo.sum(1) + sabs_i,
                   margin=np.minimum(mg.min(1) if mg.size else np.inf, mi), margin_E=mie)
        if want_parts:
            out.update(E_inter=e.sum(1), E_out=eo.sum(1), E_intra=Ei)
        return out

    def energy(self, topo, q):
        return self.score(topo, q)["E"]


class _LazyMap:
    """Combined maps filled on demand: a node's value is computed (by the
    brute-force pair sum of maps.node_values) the first time it is read."""

    def __init__(self, pocket, preset, weights):
        self.pocket = pocket
        self.preset = preset
        self.w = np.asarray(weights, np.float64)
        nx, ny, nz = pocket.dims
        self.M = np.zeros((8, nz, ny, nx))
        self.done = np.zeros((nz, ny, nx), bool)

    def ensure(self, iz, iy, ix):
        nx, ny, nz = self.pocket.dims
        flat = np.unique((np.asarray(iz) * ny + np.asarray(iy)) * nx + np.asarray(ix))
        flat = flat[~self.done.reshape(-1)[flat]]
        if len(flat) == 0:
            return
        pts = MAPS.node_coords(self.pocket.origin, self.pocket.spacing, self.pocket.dims, flat)
        G = MAPS.node_values(self.pocket.xyz, self.pocket.type, pts, self.preset)   # [8, K, n]
        vals = np.einsum("k,tkn->tn", self.w, G)
        z, rem = np.divmod(flat, nx * ny)
        y, x = np.divmod(rem, nx)
        self.M[:, z, y, x] = vals
        self.done[z, y, x] = True


class LazyScorer(Scorer):
    """Grid-mode scorer whose map nodes are computed only where poses need them."""

    def __init__(self, pocket, preset=P.PRESET_TRIDS, weights=None):
        self.preset = preset
        self.weights = np.asarray(P.default_weights(preset) if weights is None else weights,
                                  np.float64)
        self.grid = grid_of(pocket)
        self.pocket = pocket
        self.lazy = _LazyMap(pocket, preset, self.weights)
        self.M = self.lazy.M

    def inter(self, types, x):
        c = cells(self.grid, x.reshape(-1, 3))
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    self.lazy.ensure(c[:, 2] + dz, c[:, 1] + dy, c[:, 0] + dx)
        return Scorer.inter(self, types, x)


class DirectScorer:
    """The paper's pairwise form: receptor-ligand pairs within the cutoffs.

    Same E_intra; E_inter summed directly over receptor atoms (FP64 cutoff
    decisions); no map box, so no E_out.  Gradient by the same chain rule.
    """

    def __init__(self, rec_xyz, rec_type, preset=P.PRESET_TRIDS, weights=None):
        self.rec = np.asarray(rec_xyz, np.float64)
        self.rtype = np.asarray(rec_type)
        self.preset = preset
        self.weights = np.asarray(P.default_weights(preset) if weights is None else weights,
                                  np.float64)

    def inter_atoms(self, types, x, extras=False):
        Pn, N, _ = x.shape
        e = np.zeros((Pn, N)); g = np.zeros((Pn, N, 3))
        eabs = np.zeros((Pn, N))
        margin = np.full(Pn, np.inf)
        margin_e = np.full(Pn, np.inf)
        for a in range(N):
            t = int(types[a])
            r = x[:, a, None, :] - self.rec[None]          # [P, R, 3]
            d = np.sqrt(np.sum(r * r, axis=2))
            for tr in range(P.N_TYPES):
                sel = self.rtype == tr
                if not np.any(sel):
                    continue
                dd = d[:, sel]
                within = terms.within_fp64(self.preset, dd, t, tr)
                vals, dvals = terms.pair_energy_terms(self.preset, dd, t, tr, within)
                ep = np.einsum("k,kpr->pr", self.weights, vals)
                e[:, a] += ep.sum(1)
                eabs[:, a] += np.abs(ep).sum(1)
                de = np.einsum("k,kpr->pr", self.weights, dvals)
                g[:, a] += np.einsum("pr,prc->pc", de / dd, r[:, sel])
                if extras:
                    for b in _breakpoints(self.preset, t, tr):
                        margin = np.minimum(margin, np.abs(dd - b).min(1))
                    for b in _jumps(self.preset, t, tr):
                        margin_e = np.minimum(margin_e, np.abs(dd - b).min(1))
        if extras:
            return e, g, eabs, margin, margin_e
        return e, g

    def score(self, topo, q, want_parts=False):
        q = np.atleast_2d(np.asarray(q, np.float64))
        x = FK.fk(topo, q)
        e, g, eabs, m1, m1e = self.inter_atoms(topo.types, x, extras=True)
        Ei, gi, sabs_i, mi, mie = intra(topo, self.preset, self.weights, x)
        gat = g + gi
        out = dict(E=e.sum(1) + Ei, dEdq=FK.dof_gradient(topo, q, x, gat), x=x, g=gat,
                   S_abs=eabs.sum(1) + sabs_i, margin=np.minimum(m1, mi),
                   margin_E=np.minimum(m1e, mie))
        if want_parts:
            out.update(E_inter=e.sum(1), E_intra=Ei)
        return out

    def energy(self, topo, q):
        return self.score(topo, q)["E"]
