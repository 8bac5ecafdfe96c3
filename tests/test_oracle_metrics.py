"""Pins of the oracle's reconstruction metrics, its stochastic-rounding key schedule and
its Lipschitz estimate: hand-computed values and an eigen-decomposition of the
explicitly assembled operator."""
import math

import numpy as np
import pytest

import synthetic as syn


def test_rmse_and_relative_error_hand_values(orc):
    xt = np.array([3.0, 4.0])
    # x = 0: every entry is missed entirely
    assert orc.relative_error(np.zeros(2), xt) == 1.0
    assert orc.rmse(np.zeros(2), xt) == pytest.approx(3.5355339059327378, rel=1e-15)   # sqrt(25 / 2)
    # an error of a tenth of x_true in every entry
    assert orc.relative_error(np.array([3.3, 4.4]), xt) == pytest.approx(0.1, rel=1e-14)
    # one wrong voxel of eight, by 1: sqrt(1/8), over the whole 3-D array
    x3, t3 = np.zeros((2, 2, 2)), np.zeros((2, 2, 2))
    t3[1, 0, 1] = 1.0
    assert orc.rmse(x3, t3) == pytest.approx(0.3535533905932738, rel=1e-15)
    assert orc.relative_error(x3, t3) == 1.0
    # symmetric in the sign of the error, zero at the truth
    assert orc.rmse(xt, xt) == 0.0 and orc.relative_error(xt, xt) == 0.0
    assert orc.rmse(xt + 0.5, xt) == orc.rmse(xt - 0.5, xt) == 0.5


def test_psnr_hand_values_and_peak(orc):
    # peak = max x_true = 2, RMSE = 0.2: 20 log10(10) = 20 dB.  A peak taken from x (2.2)
    # or from the range of x_true (1) would give 20.83 dB or 13.98 dB.
    xt = np.array([2.0, 1.5, 1.25, 1.0])
    x = xt + np.array([0.2, -0.2, 0.2, -0.2])
    assert orc.psnr(x, xt) == pytest.approx(20.0, abs=1e-12)
    # a tenfold smaller error adds exactly 20 dB
    assert orc.psnr(xt + np.array([0.02, -0.02, 0.02, -0.02]), xt) == pytest.approx(40.0, abs=1e-12)


def test_trial_key_hand_values(orc):
    from paper_2605_12085_amd.driver import sr_key
    cases = [((0, 0, 0), 0),
             ((1, 2, 3), 4294967427),                 # 2^32 + 2*64 + 3
             ((2024, 359, 5), 8693013830085),         # 2024*2^32 + 359*64 + 5
             ((2 ** 32 + 1, 0, 0), 4294967296),       # wraps modulo 2^64
             ((0, 1, 63), 127)]                       # trial 63 stays below the next iteration
    for (s, k, j), want in cases:
        assert orc.trial_key(s, k, j) == want
        # the GPU driver's key schedule (written independently) gives the same keys
        assert sr_key(s, k, j) == want


def test_power_iteration_matches_eigenvalues_of_explicit_operator(orc):
    # L_N = n_theta/|N| lambda_max(A_N^T A_N) from the explicit 4^3 matrix
    g = syn.tiny_geometry(n=4, det=12, views=16, du=0.8)
    views = np.array([1, 4, 8, 13])
    A = orc.assemble_matrix(g, views)
    lam = np.linalg.eigvalsh(A.T @ A)
    L_exact = g.n_views / len(views) * lam[-1]
    L = orc.power_iteration_L(g, views, iters=300)
    # the Rayleigh quotient never exceeds the top eigenvalue; power iteration converges
    # from below at the rate (lambda_2/lambda_1)^iters
    assert L <= L_exact * (1 + 1e-12)
    assert L == pytest.approx(L_exact, rel=1e-9)
    # a single view and a different batch size scale as n_theta/|N|
    A1 = orc.assemble_matrix(g, [5])
    L1 = orc.power_iteration_L(g, [5], iters=300)
    assert L1 == pytest.approx(g.n_views * np.linalg.eigvalsh(A1.T @ A1)[-1], rel=1e-9)
