"""Metropolis Monte Carlo with local refinement, FP64 (oracle side).

Methods, "Conformation sampling" and Fig. 2: each copy starts from random
DOFs; every loop perturbs one variable, refines the pose by gradient
descent, and accepts the move iff rand(0,1) < exp(-beta * dE), beta = 0.069
(acceptance 0.5 at dE = 10).  Readings:
* "one variable" = one scalar DOF, chosen uniformly and resampled uniformly
  over its full range (box for translation, [-pi, pi) for angles);
* dE = E(refined proposal) - E(current);
* the best pose is the lowest refined energy seen (a proposal below the best
  is always accepted, since the best never exceeds the current energy);
* random numbers from Philox (philox.py): initial DOF d from purpose 0,
  block d // 4, word d % 4; step s from purpose 1: word 0 -> DOF index
  floor(x * n_dof / 2^32), word 1 -> new value, word 2 -> acceptance u.

State (q_cur, E_cur, q_best, E_best, step) fully describes a trajectory, so
a run can stop after any step and resume with identical results.
"""
from dataclasses import dataclass
import numpy as np

from . import params as P
from . import philox as PX
from . import optim


LOCAL_ADAM = optim.ADAM
LOCAL_LINESEARCH = optim.LINESEARCH
LOCAL_SGD = optim.SGD
LOCAL_RMSPROP = optim.RMSPROP
LOCAL_ADAGRAD = optim.ADAGRAD
LOCAL_ADAMW = optim.ADAMW


@dataclass
class SamplerParams:
    n_traj: int = 64
    n_steps: int = 100
    n_local: int = 10
    local_opt: int = LOCAL_ADAM
    lr: float = P.ADAM_LR
    beta1: float = P.ADAM_B1
    beta2: float = P.ADAM_B2
    eps: float = P.ADAM_EPS
    mc_beta: float = P.MC_BETA
    seed: int = 0


@dataclass
class State:
    q_cur: np.ndarray
    E_cur: np.ndarray
    q_best: np.ndarray
    E_best: np.ndarray
    step: int


def dof_range(topo):
    n = topo.n_dof
    lo = np.full(n, -np.pi)
    hi = np.full(n, np.pi)
    lo[0:3] = topo.box_min
    hi[0:3] = topo.box_max
    return lo, hi


def initial_q(topo, lig_id, seed, traj):
    """Random initial DOFs for trajectories `traj` (array)."""
    traj = np.asarray(traj)
    n = topo.n_dof
    lo, hi = dof_range(topo)
    q = np.zeros((len(traj), n))
    for blk in range((n + 3) // 4):
        w = PX.draw(lig_id, seed, traj, 0, PX.PURPOSE_INIT, blk)
        for r in range(4):
            d = 4 * blk + r
            if d < n:
                q[:, d] = lo[d] + (hi[d] - lo[d]) * PX.to_unit(w[r])
    return q


class EvalLog:
    """Every evaluation of every trajectory, in the order the trajectory makes
    them: rows[p] is a list of (q, E, dE/dq, S_abs, margin_E, margin) with the
    scale and margins of score.Scorer.  A record only: the sampler's
    arithmetic does not depend on it."""

    def __init__(self, n_traj):
        self.rows = [[] for _ in range(n_traj)]

    def add(self, q, r, live=None):
        for p in range(len(q)):
            if live is None or live[p]:
                self.rows[p].append((q[p].copy(), float(r["E"][p]), r["dEdq"][p].copy(),
                                     float(r["S_abs"][p]), float(r["margin_E"][p]),
                                     float(r["margin"][p])))


def init_state(scorer, topo, lig_id, prm, traj=None, evlog=None):
    traj = np.arange(prm.n_traj) if traj is None else np.asarray(traj)
    q = initial_q(topo, lig_id, prm.seed, traj)
    r = scorer.score(topo, q)
    if evlog is not None:
        evlog.add(q, r)
    E = r["E"]
    return State(q_cur=q, E_cur=E, q_best=q.copy(), E_best=E.copy(), step=0)


def run_steps(scorer, topo, lig_id, prm, state, n_steps, traj=None, trace=None,
              n_evals=None, evlog=None):
    """Advance every trajectory by n_steps MC steps (in place; returns state).
    evlog (an EvalLog) records every evaluation when given."""
    traj = np.arange(len(state.E_cur)) if traj is None else np.asarray(traj)
    lo, hi = dof_range(topo)
    n = topo.n_dof
    last = {}

    def score_fn(q):
        r = scorer.score(topo, q)
        last["r"] = r
        if evlog is not None and prm.local_opt != LOCAL_LINESEARCH:
            evlog.add(q, r)
        return r["E"], r["dEdq"]

    def ls_log(q, E, g, live):
        if evlog is not None:
            evlog.add(q, last["r"], live)

    for _ in range(n_steps):
        s = state.step + 1
        w = PX.draw(lig_id, prm.seed, traj, s, PX.PURPOSE_STEP, 0)
        j = PX.mulhi_index(w[0], n)
        q = state.q_cur.copy()
        rows = np.arange(len(traj))
        q[rows, j] = lo[j] + (hi[j] - lo[j]) * PX.to_unit(w[1])
        if prm.local_opt == LOCAL_ADAM:
            q, E = optim.adam_refine(score_fn, q, prm.n_local, topo.box_min, topo.box_max,
                                     prm.lr, prm.beta1, prm.beta2, prm.eps)
        elif prm.local_opt == LOCAL_LINESEARCH:
            q, E = optim.linesearch_refine(score_fn, q, prm.n_local, topo.box_min,
                                           topo.box_max, n_evals=n_evals, log=ls_log)
        else:
            q, E = optim.first_order_refine(prm.local_opt, score_fn, q, prm.n_local, topo.box_min,
                                            topo.box_max, prm.lr, prm.beta1, prm.beta2, prm.eps)
        u = PX.to_unit(w[2])
        dE = E - state.E_cur
        with np.errstate(over="ignore"):
            acc = u < np.exp(-prm.mc_beta * dE)
        if trace is not None:
            trace.append(dict(step=s, j=j.copy(), E_prop=E.copy(), E_cur=state.E_cur.copy(),
                              u=u.copy(), accept=acc.copy(),
                              margin=np.abs(np.log(np.maximum(u, 1e-300)) + prm.mc_beta * dE)))
        state.q_cur[acc] = q[acc]
        state.E_cur[acc] = E[acc]
        better = E < state.E_best
        state.q_best[better] = q[better]
        state.E_best[better] = E[better]
        state.step = s
    return state


def sample(scorer, topo, lig_id, prm, traj=None, trace=None, evlog=None):
    st = init_state(scorer, topo, lig_id, prm, traj, evlog=evlog)
    return run_steps(scorer, topo, lig_id, prm, st, prm.n_steps, traj, trace, evlog=evlog)
