"""E_MDN from supplied mixture parameters, FP64 (oracle side).

Test infrastructure only: the GPU library never imports it.

Methods, "Scoring functions" (the mixture density network term): for a
receptor residue i and a ligand atom j, d_ij is the smallest distance between
the atom and any atom of the residue.  With the mixture parameters
(pi_k, mu_k, sigma_k) of that pair,

    P(d) = sum_k pi_k exp(-(d - mu_k)^2 / (2 sigma_k^2))

(the printed exponent lacks its minus sign; read as a decaying Gaussian, as
for E_long and E_Hbond) and

    E_MDN = - sum_{i, j : d_ij < 5} P(d_ij).

E_dock adds w_MDN * E_MDN with w_MDN = 1.  The network that predicts the
parameters from the two molecules is out of scope: the caller supplies them.
The gradient with respect to x_j goes through d_ij at the residue's nearest
atom.  Readings: the cutoff is decided on the FP64 distance here; ties for the
nearest atom take the lowest receptor index.
"""
import numpy as np

CUTOFF = 5.0
W_MDN = 1.0


def residue_lists(residue):
    """residue index per receptor atom -> list of atom index arrays."""
    residue = np.asarray(residue, np.int64)
    n_res = int(residue.max()) + 1 if len(residue) else 0
    return [np.flatnonzero(residue == i) for i in range(n_res)]


def mixture(d, params):
    """P(d) and dP/dd for d [...] and params [..., K, 3] = (pi, mu, sigma)."""
    pi, mu, sig = params[..., 0], params[..., 1], params[..., 2]
    x = d[..., None] - mu
    g = pi * np.exp(-x * x / (2.0 * sig * sig))
    return g.sum(-1), (-g * x / (sig * sig)).sum(-1)


def mdn_energy(x, rec_xyz, residue, params):
    """E_MDN [P], dE/dx [P, N, 3] and two margins [P] for poses x [P, N, 3].

    params [N, n_res, K, 3] for the ligand's atoms (caller atom order).
    margin_E: smallest |d_ij - 5| (the energy jumps at the cutoff);
    margin: also the smallest gap between a residue's nearest and second
    nearest atom (the gradient switches atoms there).
    """
    x = np.asarray(x, np.float64)
    rec = np.asarray(rec_xyz, np.float64)
    res = residue_lists(residue)
    P_, N = x.shape[:2]
    E = np.zeros(P_)
    g = np.zeros_like(x)
    margin_E = np.full(P_, np.inf)
    margin = np.full(P_, np.inf)
    for i, atoms in enumerate(res):
        r = rec[atoms]                                           # [A, 3]
        diff = x[:, :, None, :] - r[None, None]                  # [P, N, A, 3]
        dist = np.sqrt(np.sum(diff * diff, axis=-1))             # [P, N, A]
        a = np.argmin(dist, axis=-1)                             # lowest index on ties
        d = np.take_along_axis(dist, a[..., None], -1)[..., 0]   # [P, N]
        inside = d < CUTOFF
        p, dp = mixture(d, params[:, i])
        E -= np.where(inside, p, 0.0).sum(-1)
        unit = np.take_along_axis(diff, a[..., None, None].repeat(3, -1), 2)[:, :, 0] / \
            np.where(d > 0, d, 1.0)[..., None]
        g -= np.where(inside[..., None], dp[..., None] * unit, 0.0)
        margin_E = np.minimum(margin_E, np.abs(d - CUTOFF).min(-1))
        if len(atoms) > 1:
            srt = np.sort(dist, axis=-1)
            gap = np.where(inside, srt[..., 1] - srt[..., 0], np.inf)
            margin = np.minimum(margin, gap.min(-1))
    margin = np.minimum(margin, margin_E)
    return W_MDN * E, W_MDN * g, margin_E, margin
