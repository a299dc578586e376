"""Ligand atom typing (oracle side).

Reading: the physics terms need a radius and donor / acceptor / hydrophobic
flags per atom (Methods, E_long / E_clash / E_Hbond).  From element,
implicit-H count and heavy neighbours:
  C  -> C_P if bonded to N or O, else C_H
  N  -> N_D if it carries H; else N_A if it has <= 2 heavy neighbours; else N_P
  O  -> O_DA if it carries H; else O_A
  Cl -> Cl_H
Elements: 0 C, 1 N, 2 O, 3 Cl.
"""
import numpy as np

C, N, O, CL = 0, 1, 2, 3
C_H, C_P, N_P, N_D, N_A, O_A, O_DA, CL_H = range(8)


def type_atoms(element, n_h, bonds):
    n = len(element)
    nbrs = [[] for _ in range(n)]
    for i, j in bonds:
        nbrs[int(i)].append(int(j))
        nbrs[int(j)].append(int(i))
    out = np.zeros(n, np.uint8)
    for a in range(n):
        e = int(element[a])
        if e == C:
            polar = any(int(element[b]) in (N, O) for b in nbrs[a])
            out[a] = C_P if polar else C_H
        elif e == N:
            if int(n_h[a]) >= 1:
                out[a] = N_D
            elif len(nbrs[a]) <= 2:
                out[a] = N_A
            else:
                out[a] = N_P
        elif e == O:
            out[a] = O_DA if int(n_h[a]) >= 1 else O_A
        elif e == CL:
            out[a] = CL_H
        else:
            raise ValueError("unknown element %d" % e)
    return out
