"""Seeded synthetic pockets and ligands.

This module only draws inputs: receptor atom clouds with categorical types,
and ligand molecular graphs (elements, implicit hydrogen counts, bonds,
rotatable-bond flags, an input pose).  It holds none of the docking method's
arithmetic (no typing of ligand atoms, no torsion trees, no energies, no
boxes): both the FP64 oracle and the GPU library receive these arrays as
their inputs.  Every coordinate is rounded to float32 here, at the source, so
both sides see bit-identical inputs.

Workload shapes follow the synthetic stand-ins for the paper's benchmarks
(Time-split / PoseBusters per-complex docking, a TNF-alpha style
single-target screen and a DEKOIS-style multi-target screen): protein-like
atom density, 8 receptor atom types, drug-like ligands of 10-70 heavy atoms.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

# Receptor type indices (8 types).  The order is the one every consumer uses.
TYPE_NAMES = ("C_H", "C_P", "N_P", "N_D", "N_A", "O_A", "O_DA", "Cl_H")
RECEPTOR_TYPE_P = (0.35, 0.25, 0.05, 0.08, 0.05, 0.12, 0.07, 0.03)

# Ligand elements: 0=C, 1=N, 2=O, 3=Cl, with single-bond valences.
ELEMENT_NAMES = ("C", "N", "O", "Cl")
ELEMENT_P = (0.70, 0.12, 0.14, 0.04)
VALENCE = (4, 3, 2, 1)


@dataclass
class Pocket:
    xyz: np.ndarray          # [n, 3] float32, pocket centre at the origin
    type: np.ndarray         # [n] uint8, receptor type index
    origin: np.ndarray       # [3] float32, first grid node
    spacing: float           # grid spacing in Angstrom
    dims: tuple              # (nx, ny, nz)
    radius: float


@dataclass
class Ligands:
    atom_off: np.ndarray     # [n_lig+1] int32
    element: np.ndarray      # [sum N] uint8
    n_h: np.ndarray          # [sum N] uint8, implicit hydrogens
    xyz: np.ndarray          # [sum N, 3] float32, input pose
    bond_off: np.ndarray     # [n_lig+1] int32
    bonds: np.ndarray        # [sum B, 2] int32, ligand-local atom indices
    rotatable: np.ndarray    # [sum B] uint8
    pocket_index: np.ndarray = field(default=None)  # [n_lig] int32

    @property
    def n_ligands(self):
        return len(self.atom_off) - 1

    def ligand(self, i):
        a0, a1 = self.atom_off[i], self.atom_off[i + 1]
        b0, b1 = self.bond_off[i], self.bond_off[i + 1]
        return dict(element=self.element[a0:a1], n_h=self.n_h[a0:a1],
                    xyz=self.xyz[a0:a1], bonds=self.bonds[b0:b1],
                    rotatable=self.rotatable[b0:b1])

    def subset(self, idx):
        """A new Ligands holding the listed ligands, in that order."""
        parts = [self.ligand(int(i)) for i in idx]
        out = pack_ligands(parts)
        if self.pocket_index is not None:
            out.pocket_index = self.pocket_index[np.asarray(idx)].astype(np.int32)
        return out


def _rng(seed, *path):
    ss = np.random.SeedSequence([int(seed)] + [int(p) for p in path])
    return np.random.Generator(np.random.PCG64(ss))


def make_pocket(n_atoms=600, radius=None, grid=40, spacing=0.375, seed=0,
                min_spacing=2.2):
    """Receptor atoms uniform in a ball minus a central cavity of radius 0.4R.

    The radius keeps a protein-like density: R = 15 * (n/600)^(1/3).
    A hard-core minimum spacing is enforced by rejection.  The grid is a
    cube of `grid` nodes per side centred on the cavity (the origin).
    """
    if radius is None:
        radius = 15.0 * (n_atoms / 600.0) ** (1.0 / 3.0)
    rng = _rng(seed, 1)
    r_in = 0.4 * radius
    pts = np.zeros((0, 3))
    ms2 = min_spacing ** 2
    # Random sequential addition in batches; each candidate is checked
    # against accepted atoms and against earlier candidates of its batch.
    tries = 0
    while len(pts) < n_atoms:
        tries += 1
        if tries > 10000:
            raise RuntimeError("pocket generator could not place atoms")
        m = 4 * (n_atoms - len(pts)) + 16
        v = rng.normal(size=(m, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        u = rng.random(m)
        rr = (r_in ** 3 + u * (radius ** 3 - r_in ** 3)) ** (1.0 / 3.0)
        cand = v * rr[:, None]
        for c in cand:
            if len(pts) and np.min(np.sum((pts - c) ** 2, axis=1)) < ms2:
                continue
            pts = np.vstack([pts, c[None]])
            if len(pts) == n_atoms:
                break
    xyz = pts.astype(np.float32)
    types = rng.choice(8, size=n_atoms, p=np.array(RECEPTOR_TYPE_P)).astype(np.uint8)
    n = int(grid)
    o = np.float32(-(n - 1) * spacing / 2.0)
    return Pocket(xyz=xyz, type=types, origin=np.array([o, o, o], np.float32),
                  spacing=float(spacing), dims=(n, n, n), radius=float(radius))


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def make_ligand(n_atoms, n_tors, rng, center=(0.0, 0.0, 0.0), min_nonbonded=2.0):
    """One random tree-shaped molecule with single bonds.

    Atoms are grown one at a time onto a random existing atom that still has
    free valence; bond lengths are uniform in [1.3, 1.6] A and every
    non-bonded pair stays >= `min_nonbonded` apart.  `n_tors` bonds whose two
    ends are both non-terminal are flagged rotatable (clipped to how many
    such bonds exist).  Returns a dict of plain arrays.
    """
    for _attempt in range(200):
        ok = True
        elem = [0]  # start from a carbon
        pos = [np.zeros(3)]
        deg = [0]
        bonds = []
        for a in range(1, n_atoms):
            placed = False
            for _t in range(200):
                e = int(rng.choice(4, p=np.array(ELEMENT_P)))
                free = [i for i in range(len(elem)) if deg[i] < VALENCE[elem[i]]]
                # an atom being attached must itself keep a free valence
                # unless it is the last one (keeps the tree growable)
                if not free:
                    break
                p = free[int(rng.integers(len(free)))]
                if VALENCE[e] == 1 and a < n_atoms - 1 and len(free) <= 1:
                    continue
                d = rng.normal(size=3)
                d /= np.linalg.norm(d)
                L = 1.3 + 0.3 * rng.random()
                x = pos[p] + L * d
                P = np.array(pos)
                dist = np.sqrt(np.sum((P - x) ** 2, axis=1))
                dist[p] = 10.0
                if np.min(dist) < min_nonbonded:
                    continue
                elem.append(e)
                pos.append(x)
                deg.append(1)
                deg[p] += 1
                bonds.append((p, a))
                placed = True
                break
            if not placed:
                ok = False
                break
        if ok:
            break
    else:
        raise RuntimeError("ligand generator failed")
    elem = np.array(elem, np.uint8)
    deg = np.array(deg)
    n_h = np.array([VALENCE[e] for e in elem]) - deg
    bonds = np.array(bonds, np.int32).reshape(-1, 2)
    inner = [k for k, (i, j) in enumerate(bonds) if deg[i] >= 2 and deg[j] >= 2]
    n_rot = min(int(n_tors), len(inner))
    rot = np.zeros(len(bonds), np.uint8)
    if n_rot:
        rot[rng.choice(inner, size=n_rot, replace=False)] = 1
    P = np.array(pos)
    P = (P - P.mean(axis=0)) @ _random_rotation(rng).T + np.asarray(center)
    return dict(element=elem, n_h=n_h.astype(np.uint8), xyz=P.astype(np.float32),
                bonds=bonds, rotatable=rot)


def pack_ligands(parts):
    atom_off = np.zeros(len(parts) + 1, np.int32)
    bond_off = np.zeros(len(parts) + 1, np.int32)
    for i, p in enumerate(parts):
        atom_off[i + 1] = atom_off[i] + len(p["element"])
        bond_off[i + 1] = bond_off[i] + len(p["bonds"])
    cat = lambda k, dt, shape: (np.concatenate([p[k] for p in parts]).astype(dt)
                                if parts else np.zeros(shape, dt))
    return Ligands(atom_off=atom_off,
                   element=cat("element", np.uint8, (0,)),
                   n_h=cat("n_h", np.uint8, (0,)),
                   xyz=cat("xyz", np.float32, (0, 3)).reshape(-1, 3),
                   bond_off=bond_off,
                   bonds=cat("bonds", np.int32, (0, 2)).reshape(-1, 2),
                   rotatable=cat("rotatable", np.uint8, (0,)))


def _draw_ligand(i, n_atoms, n_tors, seed, center_jitter, stream):
    rng = _rng(seed, stream, i)
    na = n_atoms(rng) if callable(n_atoms) else int(n_atoms)
    nt = n_tors(rng) if callable(n_tors) else int(n_tors)
    c = rng.normal(size=3) * center_jitter
    return make_ligand(na, nt, rng, center=c)


def _draw_chunk(args):
    lo, hi, n_atoms, n_tors, seed, center_jitter, stream = args
    return [_draw_ligand(i, n_atoms, n_tors, seed, center_jitter, stream) for i in range(lo, hi)]


def make_ligands(n_ligands, n_atoms, n_tors, seed=0, center_jitter=1.0, stream=2, workers=1):
    """`n_atoms` / `n_tors`: ints, or callables rng -> int drawn per ligand.

    Ligand i is drawn from its own seeded generator, so the result does not
    depend on `workers` (> 1: processes of a spawn pool; the callables must
    then be module-level functions)."""
    if workers > 1 and n_ligands >= 256:
        import multiprocessing as mp
        step = (n_ligands + 4 * workers - 1) // (4 * workers)
        jobs = [(lo, min(n_ligands, lo + step), n_atoms, n_tors, seed, center_jitter, stream)
                for lo in range(0, n_ligands, step)]
        with mp.get_context("spawn").Pool(workers) as pool:
            parts = [p for chunk in pool.map(_draw_chunk, jobs) for p in chunk]
    else:
        parts = [_draw_ligand(i, n_atoms, n_tors, seed, center_jitter, stream) for i in range(n_ligands)]
    return pack_ligands(parts)


# per-ligand size distributions of the workloads (module-level so that pool
# workers can receive them)
def _atoms_10_60(r):
    return int(r.integers(10, 61))


def _tors_0_15(r):
    return int(r.integers(0, 16))


def _atoms_c4(r):
    # skewed toward 25-35 heavy atoms within 15-50
    return int(np.clip(np.rint(r.normal(30.0, 5.0)), 15, 50))


def _tors_0_12(r):
    return int(r.integers(0, 13))


def _atoms_10_70(r):
    return int(r.integers(10, 71))


def default_workers():
    """Processes for drawing large ligand sets: the host's cores, at most 16."""
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# ---------------------------------------------------------------------------
# The five workload shapes.
# ---------------------------------------------------------------------------

WORKLOADS = {
    # plain method, one pocket of 600 atoms, one 24-atom ligand, 4 torsions
    "C1": dict(n_rec=600, grid=40, n_lig=1, T=64, S=100),
    # screening shape: 2,000-atom pocket, 256 ligands of 10-60 atoms
    "C2": dict(n_rec=2000, grid=64, n_lig=256, T=128, S=200),
    # differentiation: C2's pocket, 64 ligands x 32 poses, Vina-form terms
    "C3": dict(n_rec=2000, grid=64, n_lig=64, T=32, S=0),
    # batching: 65,536 ligands of 15-50 atoms
    "C4": dict(n_rec=2000, grid=64, n_lig=65536, T=32, S=150),
    # mixed pockets: 16 pockets, 4,096 ligands each
    "C5": dict(n_rec=None, grid=None, n_lig=65536, T=64, S=200),
}


def workload(name, seed=0, n_lig=None, workers=1, ligand_ids=None):
    """(pockets, ligands, sampling dict) for one of the five workloads.

    `n_lig` truncates the ligand list (the first n ligands of the full
    workload, identical to the full draw's first n); `ligand_ids` instead
    draws just the listed ligands of the full workload (pocket_index kept).
    `workers` > 1 draws the ligands in a process pool (same result).
    """
    w = WORKLOADS[name]
    nl = w["n_lig"] if n_lig is None else int(n_lig)

    def ligands(n_atoms, n_tors, stream):
        if ligand_ids is None:
            return make_ligands(nl, n_atoms, n_tors, seed=seed, stream=stream, workers=workers)
        return pack_ligands([_draw_ligand(int(i), n_atoms, n_tors, seed, 1.0, stream) for i in ligand_ids])

    if name == "C1":
        pockets = [make_pocket(600, radius=15.0, grid=40, seed=seed)]
        ligs = ligands(24, 4, 2)
    elif name in ("C2", "C3"):
        pockets = [make_pocket(2000, grid=64, seed=seed)]
        sub = 0 if name == "C2" else 1
        ligs = ligands(_atoms_10_60, _tors_0_15, 2 + sub)
    elif name == "C4":
        pockets = [make_pocket(2000, grid=64, seed=seed)]
        ligs = ligands(_atoms_c4, _tors_0_12, 4)
    elif name == "C5":
        pockets = c5_pockets(seed)
        ligs = ligands(_atoms_10_70, _tors_0_15, 5)
        ids = np.arange(nl) if ligand_ids is None else np.asarray(ligand_ids)
        ligs.pocket_index = (ids % 16).astype(np.int32)
    else:
        raise KeyError(name)
    if ligs.pocket_index is None:
        ligs.pocket_index = np.zeros(nl, np.int32)
    return pockets, ligs, dict(T=w["T"], S=w["S"])


def c5_pockets(seed=0):
    """The 16 pockets of the mixed-pocket workload: 800-3,000 atoms, grid
    sides 48-96 nodes in steps of 8, at the same atom density."""
    rng = _rng(seed, 5)
    pockets = []
    for p in range(16):
        n_rec = int(rng.integers(800, 3001))
        side = int(rng.choice(np.arange(48, 97, 8)))
        pockets.append(make_pocket(n_rec, grid=side, seed=seed * 100 + p + 1))
    return pockets


def random_poses(n_dof, box_min, box_max, n, rng):
    """Uniform DOF vectors: translation in the box, angles in [-pi, pi).

    Only a draw of inputs; float32 at the source.
    """
    q = np.empty((n, n_dof), np.float64)
    q[:, 0:3] = box_min + (np.asarray(box_max) - np.asarray(box_min)) * rng.random((n, 3))
    q[:, 3:] = -np.pi + 2 * np.pi * rng.random((n, n_dof - 3))
    return q.astype(np.float32)


def vina_weights(rng, w0=(-0.0356, -0.00516, 0.840, -0.0351, -0.587)):
    """Per-term weights drawn around the Vina defaults, ~N(w0, 0.1|w0|)."""
    w0 = np.asarray(w0)
    return (w0 + 0.1 * np.abs(w0) * rng.normal(size=w0.shape)).astype(np.float32)


def make_residues(pocket, size=8, seed=0):
    """Residue index per receptor atom: seeded greedy groups of up to `size`
    mutually close atoms (a seed atom and its nearest unassigned neighbours
    within 6 A), numbered in order of creation."""
    rng = _rng(seed, 7)
    xyz = np.asarray(pocket.xyz, np.float64)
    n = len(xyz)
    res = np.full(n, -1, np.int32)
    nxt = 0
    for a in rng.permutation(n):
        if res[a] >= 0:
            continue
        free = np.flatnonzero(res < 0)
        d = np.linalg.norm(xyz[free] - xyz[a], axis=1)
        take = free[np.argsort(d, kind="stable")][:size]
        take = take[np.linalg.norm(xyz[take] - xyz[a], axis=1) < 6.0]
        res[take] = nxt
        nxt += 1
    return res


def make_mdn_params(n_ligand_atoms, n_res, K=4, seed=0):
    """Mixture parameters [n_ligand_atoms, n_res, K, 3] = (pi, mu, sigma):
    weights from a flat Dirichlet, means U[2.5, 5.5] A, widths U[0.3, 1.0] A."""
    rng = _rng(seed, 8)
    pi = rng.dirichlet(np.ones(K), size=(n_ligand_atoms, n_res))
    mu = rng.uniform(2.5, 5.5, size=(n_ligand_atoms, n_res, K))
    sig = rng.uniform(0.3, 1.0, size=(n_ligand_atoms, n_res, K))
    return np.stack([pi, mu, sig], axis=-1).astype(np.float32)
