"""Local refinement steps, FP64 (oracle side).

ADAM (Methods, "Conformation sampling": Adam with learning rate 0.1; Table
S5 keeps Adam over AdamW / RMSprop / AdaGrad / SGD).  Readings: the
published default beta1 = 0.9, beta2 = 0.999, eps = 1e-8 with bias
correction; L steps per MC step; moments restart at every MC step.
  m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2
  q <- q - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
LINESEARCH (the alternative local rule): steepest descent along the unit
direction d = -g/|g|, alpha = 2^-j for j = 0..10, the first alpha with
  E(q + alpha d) <= E(q) + 1e-4 * alpha * (g . d)
is taken; if none is, the pose stays and its refinement ends.  After every
update the angles are wrapped to [-pi, pi) and the translation is clamped to
the box.

Optimiser variants compared in Table S5 (AdamW, RMSprop, AdaGrad, SGD), each
with the same learning rate, moments reset per MC step, and the PyTorch
default hyper-parameters as reading (RMSprop alpha 0.99, AdamW weight decay
0.01, eps as Adam's):
  SGD      q <- q - lr g
  RMSprop  v <- a v + (1-a) g^2;  q <- q - lr g / (sqrt(v) + eps)
  AdaGrad  s <- s + g^2;          q <- q - lr g / (sqrt(s) + eps)
  AdamW    q <- q (1 - lr wd), then the Adam step
"""
import numpy as np

from . import params as P

ARMIJO_C = 1e-4
LS_MAX_HALVINGS = 10

ADAM, LINESEARCH, SGD, RMSPROP, ADAGRAD, ADAMW = range(6)
RMS_ALPHA = 0.99
WEIGHT_DECAY = 0.01


def wrap_clamp(q, box_min, box_max):
    q = np.array(q, np.float64, copy=True)
    q[:, 0:3] = np.clip(q[:, 0:3], box_min, box_max)
    q[:, 3:] = q[:, 3:] - P.TWO_PI * np.floor((q[:, 3:] + np.pi) / P.TWO_PI)
    return q


def adam_refine(score_fn, q, n_local, box_min, box_max, lr=P.ADAM_LR, b1=P.ADAM_B1,
                b2=P.ADAM_B2, eps=P.ADAM_EPS, trace=None):
    """n_local Adam steps from q [P, n_dof]; returns (q, E at the final q).

    score_fn(q) -> (E, dEdq).  Evaluations: n_local gradient evaluations plus
    one final energy: n_local + 1 per call.
    """
    q = np.array(q, np.float64, copy=True)
    m = np.zeros_like(q)
    v = np.zeros_like(q)
    for t in range(1, n_local + 1):
        E, g = score_fn(q)
        if trace is not None:
            trace.append((q.copy(), E.copy(), g.copy()))
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        q = wrap_clamp(q - lr * mh / (np.sqrt(vh) + eps), box_min, box_max)
    E, g = score_fn(q)
    if trace is not None:
        trace.append((q.copy(), E.copy(), g.copy()))
    return q, E


def first_order_refine(kind, score_fn, q, n_local, box_min, box_max, lr=P.ADAM_LR, b1=P.ADAM_B1,
                       b2=P.ADAM_B2, eps=P.ADAM_EPS, alpha=RMS_ALPHA, wd=WEIGHT_DECAY):
    """n_local steps of SGD / RMSprop / AdaGrad / AdamW; returns (q, E)."""
    if kind == ADAM:
        return adam_refine(score_fn, q, n_local, box_min, box_max, lr, b1, b2, eps)
    q = np.array(q, np.float64, copy=True)
    m = np.zeros_like(q)
    v = np.zeros_like(q)
    for t in range(1, n_local + 1):
        E, g = score_fn(q)
        if kind == SGD:
            step = lr * g
        elif kind == RMSPROP:
            v = alpha * v + (1 - alpha) * g * g
            step = lr * g / (np.sqrt(v) + eps)
        elif kind == ADAGRAD:
            v = v + g * g
            step = lr * g / (np.sqrt(v) + eps)
        elif kind == ADAMW:
            q = q * (1 - lr * wd)
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            step = lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        else:
            raise ValueError(kind)
        q = wrap_clamp(q - step, box_min, box_max)
    E, g = score_fn(q)
    return q, E


def linesearch_refine(score_fn, q, n_local, box_min, box_max, n_evals=None, log=None):
    """n_local Armijo steps; returns (q, E).  n_evals[p] counts evaluations.

    A search that finds no acceptable alpha ends the pose's refinement.
    log(q, E, g, live), when given, receives every evaluation together with
    the mask of poses whose search it belongs to (a record, no arithmetic).
    """
    q = np.array(q, np.float64, copy=True)
    E, g = score_fn(q)
    if log is not None:
        log(q, E, g, np.ones(len(q), bool))
    if n_evals is not None:
        n_evals += 1
    stopped = np.zeros(len(q), bool)
    for _ in range(n_local):
        gn = np.linalg.norm(g, axis=1)
        stopped |= ~(gn > 0)
        d = np.where(stopped[:, None], 0.0, -g / np.where(stopped, 1.0, gn)[:, None])
        slope = np.einsum("pi,pi->p", g, d)
        done = stopped.copy()
        newq, newE, newg = q.copy(), E.copy(), g.copy()
        alpha = 1.0
        for _j in range(LS_MAX_HALVINGS + 1):
            if np.all(done):
                break
            cand = wrap_clamp(q + alpha * d, box_min, box_max)
            Ec, gc = score_fn(cand)
            if log is not None:
                log(cand, Ec, gc, ~done)
            if n_evals is not None:
                n_evals += ~done
            ok = (~done) & (Ec <= E + ARMIJO_C * alpha * slope)
            newq[ok], newE[ok], newg[ok] = cand[ok], Ec[ok], gc[ok]
            done |= ok
            alpha *= 0.5
        stopped |= ~done
        q, E, g = newq, newE, newg
    return q, E
