"""Pins of the oracle's pair functions and closed forms (CPU).

Values fixed by the paper's definitions (Methods, "Scoring functions" and
"Conformation sampling") or by the mathematics of each term; derivatives
pinned by central finite differences.
"""
import math
import numpy as np
import pytest

from oracle import params as P, terms, best

C_H, C_P, N_P, N_D, N_A, O_A, O_DA, CL_H = range(8)


def test_hbond_peak_is_minus_one_at_2p88():
    # E_Hbond: Gaussian with mu = 2.88, sigma = 0.3 -> -1 at d = mu.
    v, dv = terms.trids_hbond(np.array([2.88]))
    assert v[0] == -1.0 and dv[0] == 0.0


def test_hbond_one_sigma():
    v, _ = terms.trids_hbond(np.array([2.88 + 0.3, 2.88 - 0.3]))
    np.testing.assert_allclose(v, -math.exp(-0.5), rtol=1e-14)


def test_long_minimum_at_surface_distance_3():
    rsum = 3.6
    d = np.linspace(3.6, 9.9, 6301)
    v, _ = terms.trids_long(d, rsum)
    assert abs(d[np.argmin(v)] - (rsum + 3.0)) < 1.5e-3
    assert terms.trids_long(np.array([rsum + 3.0]), rsum)[0][0] == -1.0
    # width 2 A (Vina's second Gaussian): -exp(-1) two Angstrom off the peak
    np.testing.assert_allclose(terms.trids_long(np.array([rsum + 1.0, rsum + 5.0]), rsum)[0],
                               -math.exp(-1.0), rtol=1e-14)


def test_clash_zero_at_dclash_and_log2_at_half():
    for dc in (2.6, 3.4, 3.8):
        assert terms.trids_clash(np.array([dc]), dc)[0][0] == 0.0
        np.testing.assert_allclose(terms.trids_clash(np.array([dc / 2]), dc)[0], math.log(2.0),
                                   rtol=1e-14)
    # floor at 0.1 A keeps the log finite
    assert np.isfinite(terms.trids_clash(np.array([0.0]), 3.0)[0][0])


def test_dclash_is_2p6_for_donor_acceptor_pairs():
    assert P.term_cutoffs(P.PRESET_TRIDS, N_D, O_A)[1] == 2.6
    assert P.term_cutoffs(P.PRESET_TRIDS, O_A, O_DA)[1] == 2.6
    assert P.term_cutoffs(P.PRESET_TRIDS, C_H, C_P)[1] == pytest.approx(3.8)
    # hbond term only for donor/acceptor pairs, cutoff 3.4
    assert P.term_cutoffs(P.PRESET_TRIDS, C_H, O_A)[2] is None
    assert P.term_cutoffs(P.PRESET_TRIDS, N_D, N_A)[2] == 3.4
    assert P.term_cutoffs(P.PRESET_TRIDS, C_H, C_H)[0] == 10.0


def test_paper_weights():
    assert P.TRIDS_WEIGHTS == (0.2, 10.0, 0.6)
    assert P.W_TOR == 0.01 and P.MC_BETA == 0.069 and P.ADAM_LR == 0.1


def test_vina_special_values():
    assert terms.vina_gauss1(np.array([0.0]))[0][0] == 1.0
    assert terms.vina_gauss2(np.array([3.0]))[0][0] == 1.0
    assert terms.vina_repulsion(np.array([-1.0]))[0][0] == 1.0
    assert terms.vina_repulsion(np.array([0.5]))[0][0] == 0.0
    assert terms.vina_hydrophobic(np.array([1.0]))[0][0] == 0.5
    assert terms.vina_hydrophobic(np.array([0.2]))[0][0] == 1.0
    assert terms.vina_hydrophobic(np.array([1.6]))[0][0] == 0.0
    np.testing.assert_allclose(terms.vina_hbond(np.array([-0.35]))[0], 0.5, rtol=1e-14)
    assert terms.vina_hbond(np.array([-1.0]))[0][0] == 1.0


@pytest.mark.parametrize("preset,K", [(P.PRESET_TRIDS, 3), (P.PRESET_VINA, 5)])
def test_term_derivatives_by_central_difference(preset, K):
    rng = np.random.default_rng(0)
    h = 1e-6
    for ti in range(8):
        for tj in range(8):
            d = rng.uniform(0.3, 9.5, 200)
            bps = [c for c in P.term_cutoffs(preset, ti, tj) if c is not None]
            rs = P.radius(ti) + P.radius(tj)
            bps += [0.1, rs + 0.5, rs + 1.5, rs - 0.7, rs]
            d = d[np.min(np.abs(d[:, None] - np.array(bps)[None]), axis=1) > 1e-3]
            for k in range(K):
                if P.term_cutoffs(preset, ti, tj)[k] is None:
                    continue
                v, dv = terms.phi(preset, k, d, ti, tj)
                fd = (terms.phi(preset, k, d + h, ti, tj)[0] - terms.phi(preset, k, d - h, ti, tj)[0]) / (2 * h)
                np.testing.assert_allclose(dv, fd, rtol=1e-6, atol=1e-7)


def test_screen_score_closed_form():
    # E_screen = E_dock / (1 + w_tor * N_tor)
    np.testing.assert_allclose(best.screen_score(-10.0, 5), -10.0 / 1.05, rtol=1e-15)
    assert best.screen_score(-7.0, 0) == -7.0


def test_metropolis_half_acceptance_at_delta_10():
    # beta = 0.069 is chosen so that exp(-beta * 10) is (about) 0.5
    p = math.exp(-P.MC_BETA * 10.0)
    assert abs(p - 0.5) < 2e-3
    np.testing.assert_allclose(p, 0.5 * math.exp(math.log(2.0) - 0.69), rtol=1e-14)


def test_fp32_cutoff_decision_matches_numpy_float32():
    # d2 computed in FP32 with a fixed order; the decision compares with
    # fl32(c)^2 in FP32.  Check against an explicit float32 evaluation.
    rng = np.random.default_rng(1)
    a = rng.uniform(-20, 20, (1000, 3)).astype(np.float32)
    b = rng.uniform(-20, 20, (1000, 3)).astype(np.float32)
    d2 = terms.d2_fp32(a, b)
    for i in range(0, 1000, 97):
        dx, dy, dz = (np.float32(a[i, c] - b[i, c]) for c in range(3))
        ref = np.float32(np.float32(np.float32(dx * dx) + np.float32(dy * dy)) + np.float32(dz * dz))
        assert d2[i] == ref
