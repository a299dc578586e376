"""Coupled-trajectory comparison of a sampler's evaluation log with the
oracle's own run (used by the GPU sampler tests).

Both sides draw every random number from the same Philox stream (key =
(ligand, seed), counter = (trajectory, step, purpose, block)), so a GPU
trajectory and the oracle's trajectory of the same index visit the same poses
until a decision taken on floating-point values comes out differently.  The
oracle never sees a GPU value: it runs its own sampler in FP64 and logs every
evaluation (oracle.sampler.EvalLog); the GPU logs its own (record_trace).  The
two logs are compared row by row:

  q      |q_gpu - q_oracle| <= Q_PART = 2e-3 (angles modulo 2 pi)
  E      |E_gpu - E_oracle - (g_gpu + g_oracle) . dq / 2|
             <= 1e-5 max(|E|, S_abs) (1 + (|dq| / 1e-3)^2)
  dE/dq  |g_gpu - g_oracle| <= 1e-4 |g| + 1e-4 while |dq| <= 1e-6, else
         cosine >= 0.99 (the change of the gradient along a drift needs the
         Hessian)

An FP32 trajectory drifts slowly away from the FP64 one (rounding of the
poses and of each update); the energy test integrates the gradient along
that drift by the trapezoid rule, whose error is third order in |dq|.  A
parting is the first row that fails.  A pose that crosses Q_PART by gradual
growth (no jump of more than JUMP times from the previous row) is reported as
drift.  A jump, or a different evaluation count, is legitimate only if a
decision just before it lies within the tolerance band, measured on the
oracle's values:

  Metropolis  |ln u + beta dE|             <= MC_BAND
  Armijo      |E_trial - (E + c a slope)|  <= ARMIJO_BAND * max(|E|, S_abs)
  Adam/SGD..  min_j |m_hat_j| / |g|        <= SIGN_BAND (a step direction that
              an FP32 gradient error can turn)
  cutoff      the oracle's margin_E / margin (a pair, a cell face or a kink
              within 3e-5 A plus LEVER * |dq| of a decision, LEVER = 15 A
              bounding how far a drift of the DOFs moves an atom)

Rows whose oracle margin lies within that band are not compared (the energy
or gradient may jump between the two poses), but the comparison goes on.

Rows are compared until the first such explained parting; an unexplained one
fails the test.
"""
import numpy as np

Q_PART = 2e-3
JUMP = 20.0
MC_BAND = 2e-3
ARMIJO_BAND = 1e-4
SIGN_BAND = 2e-3
MARGIN = 3e-5
LEVER = 15.0
ARMIJO_C = 1e-4
ARMIJO_TRIALS = 11


def _dq(qg, qo):
    d = np.abs(qg - qo)
    d[3:] = np.abs(np.angle(np.exp(1j * (qg[3:] - qo[3:]))))
    return d


def decision_margins(rows, kind, n_local, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Per row of one oracle trajectory, the smallest relative margin of the
    decisions taken right after that row (inf if none), and the row indices
    where each MC step ends.  rows: EvalLog rows of one trajectory."""
    n = len(rows)
    m_arm = np.full(n, np.inf)
    m_sign = np.full(n, np.inf)
    step_end = []
    if kind == "linesearch":
        # rows: [init] then per MC step: base eval, then searches of trials
        k = 1
        while k < n:
            base = k
            E, g = rows[base][1], rows[base][2]
            scale = max(abs(E), rows[base][3], 1.0)
            k += 1
            steps_done = 0
            ended = False
            while steps_done < n_local and not ended:
                gn = np.linalg.norm(g)
                if not gn > 0:
                    ended = True
                    break
                slope = -gn
                alpha, accepted = 1.0, False
                for _ in range(11):
                    if k >= n:
                        ended = True
                        break
                    Et = rows[k][1]
                    thr = E + ARMIJO_C * alpha * slope
                    m_arm[k] = abs(Et - thr) / scale
                    k += 1
                    if Et <= thr:
                        E, g = Et, rows[k - 1][2]
                        accepted = True
                        break
                    alpha *= 0.5
                if not accepted:
                    ended = True
                steps_done += 1
            step_end.append(k - 1)
    else:
        per = n_local + 1
        k = 1
        while k + per - 1 < n:
            m = None
            v = None
            for t in range(n_local):
                g = rows[k + t][2]
                if m is None:
                    m = np.zeros_like(g)
                    v = np.zeros_like(g)
                m = b1 * m + (1 - b1) * g
                v = b2 * v + (1 - b2) * g * g
                gn = max(np.linalg.norm(g), 1e-30)
                if kind in ("adam", "adamw"):
                    mh = m / (1 - b1 ** (t + 1))
                    m_sign[k + t] = np.min(np.abs(mh)) / gn
                elif kind in ("rmsprop", "adagrad"):
                    m_sign[k + t] = np.min(np.abs(g)) / gn
            step_end.append(k + per - 1)
            k += per
    return m_arm, m_sign, np.asarray(step_end, np.int64)


def compare(gpu_rows, gpu_n, orc_rows, mc_margin, kind, n_local, lr, n_dof):
    """Compares one trajectory.  gpu_rows [cap, 2*qs+1] (q, g, E); gpu_n its
    evaluation count; orc_rows the oracle's EvalLog rows; mc_margin [S] the
    oracle's Metropolis margins per step.  Returns (rows_agreeing, parted,
    explained, reason); a parting by gradual drift (no jump) is explained as
    "drift"."""
    qs = (gpu_rows.shape[1] - 1) // 2
    n_cmp = min(gpu_n, len(orc_rows))
    m_arm, m_sign, step_end = decision_margins(orc_rows, kind, n_local, lr)
    first_bad, why_bad, dq_prev, jump = None, "", 0.0, False
    cut_band = MARGIN
    for k in range(n_cmp):
        q_o, E_o, g_o, S_o, mE_o, m_o = orc_rows[k]
        q_g = gpu_rows[k, :n_dof].astype(np.float64)
        g_g = gpu_rows[k, qs:qs + n_dof].astype(np.float64)
        E_g = float(gpu_rows[k, 2 * qs])
        dq = _dq(q_g, q_o)
        dqm = float(dq.max())
        sd = q_g - q_o
        sd[3:] = np.angle(np.exp(1j * sd[3:]))
        gn = float(np.linalg.norm(g_o))
        scale = max(abs(E_o), S_o)
        if dqm > Q_PART:
            first_bad, why_bad = k, "pose %.2g" % dqm
            jump = dqm > JUMP * max(dq_prev, 1e-5)
            break
        # a decision (cell face, cutoff, kink) within the oracle position error
        # plus the atoms' displacement by the drift (lever arm <= LEVER)
        band = MARGIN + LEVER * dqm
        if m_o > band:
            trap = abs(E_g - E_o - 0.5 * float((g_g + g_o) @ sd))
            if not trap <= 1e-5 * scale * (1.0 + (dqm / 1e-3) ** 2) + 1e-6:
                first_bad, why_bad = k, "energy %.3g vs %.3g (trapezoid residual %.2g of scale %.3g)" % (
                    E_g, E_o, trap, scale)
                break
        elif mE_o > band:
            if not abs(E_g - E_o) <= 1e-5 * scale + 2.0 * gn * float(np.linalg.norm(sd)) + 1e-6:
                first_bad, why_bad = k, "energy %.3g vs %.3g near a kink" % (E_g, E_o)
                break
        if m_o > band and gn > 0:
            if dqm <= 1e-6:
                bad = np.linalg.norm(g_g - g_o) > 1e-4 * gn + 1e-4
            else:
                bad = float(g_g @ g_o) < 0.99 * gn * np.linalg.norm(g_g)
            if bad:
                first_bad, why_bad = k, "gradient |dg| %.3g of |g| %.3g at drift %.2g" % (
                    np.linalg.norm(g_g - g_o), gn, dqm)
                break
        dq_prev = dqm
        cut_band = max(cut_band, band)
    if first_bad is None and gpu_n == len(orc_rows):
        return n_cmp, False, True, ""
    k = n_cmp if first_bad is None else first_bad
    if first_bad is not None and why_bad.startswith("pose") and not jump:
        return k, True, True, "drift; row %d %s" % (k, why_bad)
    # decisions that could have parted them: every decision from the start of
    # the MC step holding row k - 1 up to row k - 1, and the Metropolis test
    # closing the previous step
    prev_end = step_end[step_end < k - 1]
    lo = int(prev_end[-1]) if len(prev_end) else 0
    reasons = []
    arm = m_arm[lo:k].min(initial=np.inf)
    sign = m_sign[lo:k].min(initial=np.inf)
    s_idx = int(np.searchsorted(step_end, k - 1))     # steps that ended before row k
    mc = np.inf
    if len(mc_margin):
        mcs = [mc_margin[i] for i in (s_idx - 1, s_idx) if 0 <= i < len(mc_margin)]
        mc = min(mcs) if mcs else np.inf
    hi = min(k + 1, len(orc_rows))
    cut = min([orc_rows[j][4] for j in range(lo, hi)] + [orc_rows[j][5] for j in range(lo, hi)] + [np.inf])
    if arm <= ARMIJO_BAND:
        reasons.append("armijo %.2g" % arm)
    if sign <= SIGN_BAND:
        reasons.append("step sign %.2g" % sign)
    if mc <= MC_BAND:
        reasons.append("metropolis %.2g" % mc)
    if cut <= max(cut_band, MARGIN + LEVER * dq_prev):
        reasons.append("cutoff %.2g" % cut)
    detail = "row %d of %d/%d: %s (armijo %.2g sign %.2g metropolis %.2g cutoff %.2g)" % (
        k, gpu_n, len(orc_rows), why_bad or "evaluation count", arm, sign, mc, cut)
    # only a jump of the pose or a different evaluation count can come from a
    # decision; an energy or gradient mismatch at agreeing poses cannot
    if first_bad is not None and not why_bad.startswith("pose"):
        reasons = [r for r in reasons if r.startswith("cutoff")]
    return k, True, bool(reasons), (", ".join(reasons) + "; " if reasons else "") + detail


def compare_run(gpu_trace, gpu_nev, evlog, mc_trace, kind, n_local, lr, n_dof):
    """All trajectories of one ligand.  gpu_trace [T, cap, 2*qs+1]; gpu_nev
    [T]; evlog the oracle's EvalLog; mc_trace the oracle sampler's per-step
    trace (list of dicts with 'margin').  Returns a summary dict."""
    T = len(gpu_nev)
    mcm = np.stack([t["margin"] for t in mc_trace], axis=0) if mc_trace else np.zeros((0, T))
    out = dict(T=T, whole=0, parted=0, explained=0, unexplained=[], rows=0, first_part=[])
    for t in range(T):
        rows, parted, expl, why = compare(gpu_trace[t], int(gpu_nev[t]), evlog.rows[t], mcm[:, t], kind,
                                          n_local, lr, n_dof)
        out["rows"] += rows
        if not parted:
            out["whole"] += 1
        else:
            out["parted"] += 1
            out["first_part"].append(rows)
            if expl:
                out["explained"] += 1
            else:
                out["unexplained"].append((t, why))
    return out


def summary(res):
    """One line for the test log."""
    fp = res["first_part"]
    return "%d/%d trajectories whole, %d parted (%d explained, first parting row median %s), %d rows agree" % (
        res["whole"], res["T"], res["parted"], res["explained"], int(np.median(fp)) if fp else "-", res["rows"])


def check_linesearch_log(rows, n_rows, n_dof, n_local, box_min, box_max):
    """Replays the Armijo line search on one trajectory's log (rows [cap,
    2*qs+1] of (q, g, E)): every trial pose is the search's base pose moved by
    alpha = 2^-j along d = -g/|g| (then wrapped and clamped); the decision read
    off the next row (a halved trial from the same base means a rejection)
    follows E_trial <= E + 1e-4 alpha (g . d) unless the two sides lie within
    FP32 resolution of each other; each search ends at its first accepted
    trial; n_local accepted steps or a failed search end an MC step's
    refinement.  Returns (trials, accepted, within resolution)."""
    qs = (rows.shape[1] - 1) // 2
    n = n_dof
    R = np.asarray(rows[:n_rows], np.float64)

    def moved(q, d, alpha):
        x = q + alpha * d
        x[:3] = np.clip(x[:3], box_min, box_max)
        x[3:] = x[3:] - 2 * np.pi * np.floor((x[3:] + np.pi) / (2 * np.pi))
        return x

    def near(a, b):
        d = np.abs(a - b)
        d[3:] = np.abs(np.angle(np.exp(1j * (a[3:] - b[3:]))))
        return d.max() < 2e-5 * (1 + np.abs(b).max())

    n_trials = n_acc = n_band = 0
    k = 1
    while k < n_rows:
        # a base row (the perturbed pose of an MC step), then the searches
        qb, Eb, gb = R[k, :n], R[k, 2 * qs], R[k, qs:qs + n]
        k += 1
        for _ in range(n_local):
            gn = np.linalg.norm(gb)
            if not gn > 0 or k >= n_rows:
                break
            d = -gb / gn
            alpha, acc = 1.0, False
            for j in range(ARMIJO_TRIALS):
                if k >= n_rows:
                    break
                qt, Et = R[k, :n], R[k, 2 * qs]
                assert near(qt, moved(qb, d, alpha)), ("trial pose", k)
                n_trials += 1
                thr = Eb + ARMIJO_C * alpha * (-gn)
                k += 1
                rejected = j < ARMIJO_TRIALS - 1 and k < n_rows and near(R[k, :n], moved(qb, d, alpha / 2))
                band = 4e-7 * max(1.0, abs(Eb), abs(Et))
                if abs(Et - thr) <= band:
                    n_band += 1
                elif j < ARMIJO_TRIALS - 1:
                    assert rejected == (Et > thr), ("armijo decision", k - 1, Et, thr)
                if not rejected:
                    acc = Et <= thr + band
                    if acc:
                        n_acc += 1
                        qb, Eb, gb = qt, Et, R[k - 1, qs:qs + n]
                    break
                alpha *= 0.5
            if not acc:
                break
    return n_trials, n_acc, n_band


class _Log:
    def __init__(self, rows):
        self.rows = rows


def oracle_run(args):
    """Pool worker: the oracle's own run of the listed trajectories of one
    ligand (a lazily filled grid scorer on its pocket) with its evaluation
    log.  args = (pocket, preset, weights, ligands, index in `ligands`,
    ligand id (the Philox key), SamplerParams fields, trajectories).
    Returns (rows per trajectory, per-step Metropolis margins)."""
    pocket, preset, weights, ligs, i, lig_id, prm_kw, traj = args
    from oracle import topology, score as SC, sampler as SM
    topo = topology.from_ligands(ligs, i)
    sc = SC.LazyScorer(pocket, preset, weights=np.asarray(weights, np.float64))
    evlog, mct = SM.EvalLog(len(traj)), []
    SM.sample(sc, topo, int(lig_id), SM.SamplerParams(**prm_kw), traj=np.asarray(traj), trace=mct, evlog=evlog)
    return evlog.rows, [t["margin"] for t in mct]


def compare_prefix(gpu_trace, gpu_nev, rows, margins, kind, n_local, lr, n_dof):
    """compare_run over the oracle's (shorter) run: each GPU log is cut to
    the oracle's row count when it holds at least as many rows."""
    nev = np.asarray([min(int(g), len(r)) for g, r in zip(gpu_nev, rows)])
    return compare_run(gpu_trace, nev, _Log(rows), [dict(margin=m) for m in margins], kind, n_local, lr, n_dof)
