"""torch.autograd.Function around the differentiable form of the score.

    E = dock_score(pockets, L, pose_lig, w, G_list, q=q)      # or xyz=...
    E.sum().backward()    # -> G.grad, w.grad, q.grad (or xyz.grad)

Forward: dock_score_terms.  Backward: dock_score_adjoint, which recomputes
the forward kinematics from the saved DOFs (no per-pose coordinates are
stored) and scatters dL/dG, dL/dw, dL/dq, dL/dx in one kernel.
"""
import torch

from . import binding as B


class DockScoreFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pockets, L, pose_lig, q, xyz, w, *G):
        G = list(G)
        Gin = [g.detach().contiguous() for g in G]
        wd = w.detach().contiguous()
        qd = None if q is None else q.detach().contiguous()
        xd = None if xyz is None else xyz.detach().contiguous()
        E = B.dock_score_terms(pockets, L, pose_lig, wd, q=qd, xyz=xd, G=Gin)
        ctx.pockets, ctx.L = pockets, L
        ctx.has_q, ctx.has_x = q is not None, xyz is not None
        ctx.save_for_backward(pose_lig, wd, *([qd] if qd is not None else []),
                              *([xd] if xd is not None else []), *Gin)
        return E

    @staticmethod
    def backward(ctx, dLdE):
        saved = list(ctx.saved_tensors)
        pose_lig, w = saved[0], saved[1]
        i = 2
        q = xyz = None
        if ctx.has_q:
            q = saved[i]; i += 1
        if ctx.has_x:
            xyz = saved[i]; i += 1
        G = saved[i:]
        need = ctx.needs_input_grad
        dLdq = torch.zeros_like(q) if (q is not None and need[3]) else None
        dLdx = torch.zeros_like(xyz) if (xyz is not None and need[4]) else None
        dLdw = torch.zeros_like(w) if need[5] else None
        dLdG = [torch.zeros_like(g) if need[6 + k] else None for k, g in enumerate(G)]
        B.dock_score_adjoint(ctx.pockets, ctx.L, pose_lig, w, dLdE.contiguous().float(), q=q, xyz=xyz,
                             G=list(G), dLdG=dLdG, dLdw=dLdw, dLdq=dLdq, dLdx=dLdx)
        return (None, None, None, dLdq, dLdx, dLdw, *dLdG)


def dock_score(pockets, L, pose_lig, w, G, q=None, xyz=None):
    """Differentiable scores.  pockets: Pocket or list; w: [n_pockets, K];
    G: per-term map tensor or list of them [8, K, nz, ny, nx]; exactly one of
    q [P, q_stride] / xyz [P, max_atoms, 3]."""
    if isinstance(pockets, B.Pocket):
        pockets = [pockets]
    if torch.is_tensor(G):
        G = [G]
    return DockScoreFn.apply(pockets, L, pose_lig, q, xyz, w, *G)
