"""Torsion tree, fragments and intra-ligand pair list (oracle side).

The sampling space is translation, rotation and the torsion angles of
rotatable bonds (Methods, "Conformation sampling"); N_tor counts the rotatable
bonds (E_screen).  The paper leaves the tree construction implicit; readings:

* Fragments are the connected components of the bond graph once rotatable
  bonds are removed; fragment ids follow the lowest atom index they contain.
  A rotatable bond must be a bridge (a rotatable ring bond is an error).
* Root = the fragment whose fragment-tree height is smallest (ties: lowest
  id).  Breadth-first order from the root, children in increasing id; the
  k-th non-root fragment in that order owns torsion k, whose axis runs from
  atom a_k (parent side) to atom b_k (child side).
* c0 = centroid of the root fragment's input coordinates (FP64): the point
  the translation DOF places and the rotation turns about.
* Intra-ligand pairs: i < j in different fragments and at least 4 bonds
  apart, sorted lexicographically.
* Translation box: axis-aligned bounds of the input pose unless given.
"""
from collections import deque
from dataclasses import dataclass
import numpy as np

from .atomtype import type_atoms

MAX_ATOMS = 128
MAX_TORS = 32


class TopologyError(ValueError):
    pass


class LimitError(ValueError):
    pass


@dataclass
class Topology:
    n_atoms: int
    types: np.ndarray        # [N] uint8
    atom_frag: np.ndarray    # [N] int32
    n_frags: int
    root: int
    frag_parent: np.ndarray  # [F] int32, -1 for the root
    frag_tors: np.ndarray    # [F] int32, torsion owned by the fragment, -1 root
    bfs: np.ndarray          # [F] fragment ids in BFS order
    tors_frag: np.ndarray    # [n_t] child fragment of torsion k
    tors_a: np.ndarray       # [n_t] axis atom on the parent side
    tors_b: np.ndarray       # [n_t] axis atom on the child side
    pairs: np.ndarray        # [P, 2] int32
    x0: np.ndarray           # [N, 3] float64 (values of the FP32 input)
    c0: np.ndarray           # [3] float64
    box_min: np.ndarray      # [3] float64
    box_max: np.ndarray      # [3] float64
    height: int

    @property
    def n_tors(self):
        return len(self.tors_frag)

    @property
    def n_dof(self):
        return 6 + self.n_tors

    def subtree_atoms(self, k):
        """Boolean mask of atoms moved by torsion k (its child's subtree)."""
        f0 = int(self.tors_frag[k])
        inside = np.zeros(self.n_frags, bool)
        for f in self.bfs:            # parents precede children in BFS
            if f == f0 or (self.frag_parent[f] >= 0 and inside[self.frag_parent[f]]):
                inside[f] = True
        return inside[self.atom_frag]


def _bfs_dist(adj, src, n):
    dist = np.full(n, -1, np.int64)
    dist[src] = 0
    dq = deque([src])
    while dq:
        u = dq.popleft()
        for v in adj[u]:
            if dist[v] < 0:
                dist[v] = dist[u] + 1
                dq.append(v)
    return dist


def build(element, n_h, xyz, bonds, rotatable, box_min=None, box_max=None):
    element = np.asarray(element)
    n = len(element)
    if n < 1:
        raise TopologyError("empty ligand")
    if n > MAX_ATOMS:
        raise LimitError("ligand has %d atoms > %d" % (n, MAX_ATOMS))
    xyz = np.asarray(xyz, np.float32).astype(np.float64).reshape(n, 3)
    if not np.all(np.isfinite(xyz)):
        raise TopologyError("non-finite coordinates")
    bonds = np.asarray(bonds, np.int64).reshape(-1, 2)
    rotatable = np.asarray(rotatable).astype(bool).reshape(-1)
    seen = set()
    adj = [[] for _ in range(n)]
    for i, j in bonds:
        if not (0 <= i < n and 0 <= j < n) or i == j:
            raise TopologyError("bad bond (%d, %d)" % (i, j))
        key = (min(i, j), max(i, j))
        if key in seen:
            raise TopologyError("duplicate bond (%d, %d)" % key)
        seen.add(key)
        adj[i].append(int(j))
        adj[j].append(int(i))
    if np.any(_bfs_dist(adj, 0, n) < 0):
        raise TopologyError("disconnected ligand")
    if int(rotatable.sum()) > MAX_TORS:
        raise LimitError("too many rotatable bonds")

    # fragments: components without rotatable bonds, ids by lowest atom
    rigid = [[] for _ in range(n)]
    for (i, j), r in zip(bonds, rotatable):
        if not r:
            rigid[i].append(int(j))
            rigid[j].append(int(i))
    frag = np.full(n, -1, np.int32)
    nf = 0
    for a in range(n):
        if frag[a] < 0:
            for b in np.nonzero(_bfs_dist(rigid, a, n) >= 0)[0]:
                frag[b] = nf
            nf += 1
    # fragment tree edges = rotatable bonds; must form a tree
    fadj = [[] for _ in range(nf)]
    redges = {}
    for (i, j), r in zip(bonds, rotatable):
        if not r:
            continue
        fi, fj = int(frag[i]), int(frag[j])
        if fi == fj or (min(fi, fj), max(fi, fj)) in redges:
            raise TopologyError("rotatable bond inside a ring")
        redges[(min(fi, fj), max(fi, fj))] = (int(i), int(j))
        fadj[fi].append(fj)
        fadj[fj].append(fi)
    if len(redges) != nf - 1:
        raise TopologyError("fragment graph is not a tree")
    for f in range(nf):
        fadj[f].sort()
    heights = [int(_bfs_dist(fadj, f, nf).max()) for f in range(nf)]
    root = int(np.argmin(heights))           # argmin keeps the lowest id on ties
    parent = np.full(nf, -1, np.int32)
    order = [root]
    dq = deque([root])
    visited = np.zeros(nf, bool)
    visited[root] = True
    while dq:
        u = dq.popleft()
        for v in fadj[u]:
            if not visited[v]:
                visited[v] = True
                parent[v] = u
                order.append(v)
                dq.append(v)
    frag_tors = np.full(nf, -1, np.int32)
    tf, ta, tb = [], [], []
    for f in order[1:]:
        p = int(parent[f])
        i, j = redges[(min(p, f), max(p, f))]
        a, b = (i, j) if frag[i] == p else (j, i)
        frag_tors[f] = len(tf)
        tf.append(f)
        ta.append(a)
        tb.append(b)

    # intra pairs: different fragments, >= 4 bonds apart
    pairs = []
    for i in range(n):
        di = _bfs_dist(adj, i, n)
        for j in range(i + 1, n):
            if frag[i] != frag[j] and di[j] >= 4:
                pairs.append((i, j))
    pairs = np.array(pairs, np.int32).reshape(-1, 2)

    c0 = xyz[frag == root].mean(axis=0)
    if box_min is None:
        box_min = xyz.min(axis=0)
    if box_max is None:
        box_max = xyz.max(axis=0)
    box_min = np.asarray(box_min, np.float32).astype(np.float64)
    box_max = np.asarray(box_max, np.float32).astype(np.float64)
    if np.any(box_min > box_max):
        raise TopologyError("box_min > box_max")
    return Topology(
        n_atoms=n, types=type_atoms(element, n_h, bonds), atom_frag=frag,
        n_frags=nf, root=root, frag_parent=parent, frag_tors=frag_tors,
        bfs=np.array(order, np.int32), tors_frag=np.array(tf, np.int32),
        tors_a=np.array(ta, np.int32), tors_b=np.array(tb, np.int32),
        pairs=pairs, x0=xyz, c0=c0, box_min=box_min, box_max=box_max,
        height=heights[root])


def from_ligands(ligs, i, **kw):
    d = ligs.ligand(i)
    return build(d["element"], d["n_h"], d["xyz"], d["bonds"], d["rotatable"], **kw)
