"""Forward kinematics of the torsion tree, FP64 (oracle side).

DOFs (Methods, "Conformation sampling"): q = (T, alpha, beta, gamma,
theta_0..theta_{n_t-1}); translation in [box_min, box_max], the three
rotation angles and every torsion in [-pi, pi).  Readings:
* rotation R = Rz(alpha) Ry(beta) Rx(gamma) (intrinsic Z-Y-X Euler angles),
  turning about c0, the root-fragment centroid; T is where c0 lands;
* torsions are deltas from the input pose, right-handed about a_k -> b_k.
Local frame: root (R, t) = (I, -c0); child fragment f of parent p with
torsion k:  R_f = R_p Rot(u_k, theta_k),
            t_f = R_p (x0_b - Rot(u_k, theta_k) x0_b) + t_p,
u_k = unit(x0_b - x0_a).  World: x = T + R (R_f x0 + t_f).
"""
import numpy as np


def rot_axis(u, theta):
    """Rotation matrices about unit axis u by angles theta [P] -> [P,3,3]."""
    c = np.cos(theta)[:, None, None]
    s = np.sin(theta)[:, None, None]
    ux = np.array([[0.0, -u[2], u[1]], [u[2], 0.0, -u[0]], [-u[1], u[0], 0.0]])
    uu = np.outer(u, u)
    return c * np.eye(3) + s * ux + (1.0 - c) * uu


def euler_zyx(a, b, g):
    """R = Rz(a) Ry(b) Rx(g), arrays [P] -> [P,3,3]."""
    ca, sa = np.cos(a), np.sin(a)
    cb, sb = np.cos(b), np.sin(b)
    cg, sg = np.cos(g), np.sin(g)
    P = len(a)
    Rz = np.zeros((P, 3, 3)); Ry = np.zeros((P, 3, 3)); Rx = np.zeros((P, 3, 3))
    Rz[:, 0, 0] = ca; Rz[:, 0, 1] = -sa; Rz[:, 1, 0] = sa; Rz[:, 1, 1] = ca; Rz[:, 2, 2] = 1
    Ry[:, 0, 0] = cb; Ry[:, 0, 2] = sb; Ry[:, 2, 0] = -sb; Ry[:, 2, 2] = cb; Ry[:, 1, 1] = 1
    Rx[:, 1, 1] = cg; Rx[:, 1, 2] = -sg; Rx[:, 2, 1] = sg; Rx[:, 2, 2] = cg; Rx[:, 0, 0] = 1
    return Rz @ Ry @ Rx, Rz, Ry


def fragment_frames(topo, q):
    """Local frames (R_f [P,F,3,3], t_f [P,F,3]) for every fragment."""
    q = np.atleast_2d(np.asarray(q, np.float64))
    P = q.shape[0]
    F = topo.n_frags
    Rf = np.zeros((P, F, 3, 3))
    tf = np.zeros((P, F, 3))
    r = topo.root
    Rf[:, r] = np.eye(3)
    tf[:, r] = -topo.c0
    for f in topo.bfs[1:]:
        p = topo.frag_parent[f]
        k = topo.frag_tors[f]
        xa = topo.x0[topo.tors_a[k]]
        xb = topo.x0[topo.tors_b[k]]
        u = (xb - xa) / np.linalg.norm(xb - xa)
        Rk = rot_axis(u, q[:, 6 + k])
        Rf[:, f] = Rf[:, p] @ Rk
        tf[:, f] = np.einsum("pij,pj->pi", Rf[:, p], xb - np.einsum("pij,j->pi", Rk, xb)) + tf[:, p]
    return Rf, tf


def fk(topo, q):
    """World coordinates x [P, N, 3] for poses q [P, n_dof]."""
    q = np.atleast_2d(np.asarray(q, np.float64))
    Rf, tf = fragment_frames(topo, q)
    R, _, _ = euler_zyx(q[:, 3], q[:, 4], q[:, 5])
    fa = topo.atom_frag
    local = np.einsum("pnij,nj->pni", Rf[:, fa], topo.x0) + tf[:, fa]
    return q[:, None, 0:3] + np.einsum("pij,pnj->pni", R, local)


def dof_gradient(topo, q, x, g):
    """Chain rule from atom gradients g = dE/dx [P,N,3] to dE/dq [P,n_dof].

    dE/dT = sum_i g_i;  tau = sum_i (x_i - T) x g_i;
    dE/d(alpha, beta, gamma) = tau . (e_z, Rz e_y, Rz Ry e_x);
    dE/dtheta_k = u_k^world . sum_{i in subtree(k)} (x_i - x_{b_k}) x g_i.
    """
    q = np.atleast_2d(np.asarray(q, np.float64))
    P = q.shape[0]
    out = np.zeros((P, topo.n_dof))
    out[:, 0:3] = g.sum(axis=1)
    r = x - q[:, None, 0:3]
    tau = np.cross(r, g).sum(axis=1)
    _, Rz, Ry = euler_zyx(q[:, 3], q[:, 4], q[:, 5])
    ez = np.array([0.0, 0.0, 1.0])
    ey = np.einsum("pij,j->pi", Rz, np.array([0.0, 1.0, 0.0]))
    ex = np.einsum("pij,j->pi", Rz @ Ry, np.array([1.0, 0.0, 0.0]))
    out[:, 3] = tau @ ez
    out[:, 4] = np.einsum("pi,pi->p", tau, ey)
    out[:, 5] = np.einsum("pi,pi->p", tau, ex)
    for k in range(topo.n_tors):
        m = topo.subtree_atoms(k)
        a, b = topo.tors_a[k], topo.tors_b[k]
        u = x[:, b] - x[:, a]
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        t = np.cross(x[:, m] - x[:, b][:, None], g[:, m]).sum(axis=1)
        out[:, 6 + k] = np.einsum("pi,pi->p", u, t)
    return out
