"""Pins of the PSRF oracle (Section 2.4.2, eqs. winco, btwco, psrf with M = 1).

* A hand-worked case: three chains of four states at mu_p +- sigma (so every
  chain mean and within-chain variance is exact), whose B, W and R are worked
  out on paper below.
* Identical chains: no between-chain spread, R = (n - 1)/n.
* Stopping errors (Section 3.3): a covariance scaled by 1 + eps, a mean off by
  a 3-4-5 vector.
* Independent draws from one Gaussian: sqrt(R) - 1 is O(1/n) (Gelman and
  Rubin's statistic tends to 1); chains offset by a known shift fail it.
"""
import numpy as np
import pytest

from oracle import psrf as op


def test_hand_worked_three_chains():
    # chain p: mu_p + (sigma, -sigma, sigma, -sigma) with mu = (0, 1, 2), sigma = 1
    # m^p = mu_p, C^p = 1;  m^glob = 1
    # B = n/(P-1) sum (mu_p - 1)^2 = 4/2 * 2 = 4
    # W = n/((n-1) P) sum C^p = 4/(3*3) * 3 = 4/3
    # R = (n-1)/n + (P+1)/(P n) * B/W = 3/4 + (4/12) * 3 = 7/4
    mu = np.array([0.0, 1.0, 2.0])
    pm = np.array([1.0, -1.0, 1.0, -1.0])
    chains = (mu[:, None] + pm[None, :])[:, :, None]          # (P=3, n=4, d=1)
    B, W, R = op.psrf_terms(chains)
    assert B[0] == pytest.approx(4.0, rel=1e-15)
    assert W[0] == pytest.approx(4.0 / 3.0, rel=1e-15)
    assert R[0] == pytest.approx(1.75, rel=1e-15)
    assert op.psrf(chains)[0] == pytest.approx(np.sqrt(1.75), rel=1e-15)


def test_identical_chains_have_no_between_spread():
    rng = np.random.default_rng(3)
    one = rng.standard_normal((50, 6))
    chains = np.stack([one] * 5)
    B, W, R = op.psrf_terms(chains)
    assert np.all(B < 1e-25 * W)          # only the rounding of the mean of equal means
    np.testing.assert_allclose(R, 49 / 50, rtol=1e-13)


def test_independent_draws_converge_and_offsets_are_detected():
    rng = np.random.default_rng(11)
    P, n, d = 8, 20000, 5
    chains = rng.standard_normal((P, n, d)) * np.array([1.0, 2.0, 0.5, 3.0, 1e-3])
    r = op.psrf(chains) - 1.0
    assert np.all(np.abs(r) < 2e-3), r
    shifted = chains.copy()
    shifted[0, :, :] += 0.5 * np.array([1.0, 2.0, 0.5, 3.0, 1e-3])   # half a standard deviation
    assert np.all(op.psrf(shifted) - 1.0 > 0.01)


def test_rejects_degenerate_sizes():
    with pytest.raises(ValueError):
        op.psrf(np.zeros((1, 10, 2)))
    with pytest.raises(ValueError):
        op.psrf(np.zeros((3, 1, 2)))


def test_stopping_errors_on_known_perturbations():
    # C = (1 + eps) Sigma exactly gives a relative Frobenius error of eps;
    # a mean off by (3, 4, 0, ...) is 5 away in the Euclidean norm
    rng = np.random.default_rng(4)
    G = rng.standard_normal((6, 6))
    Sigma = G @ G.T + 6 * np.eye(6)
    mu = rng.standard_normal(6)
    eps = 0.125
    S = (1 + eps) * Sigma + np.outer(mu, mu)
    assert op.cov_rel_error(S, mu, Sigma) == pytest.approx(eps, rel=1e-13)
    assert op.cov_rel_error(Sigma + np.outer(mu, mu), mu, Sigma) < 1e-15
    off = mu + np.array([3.0, 4.0, 0, 0, 0, 0])
    assert op.mean_abs_error(off, mu) == pytest.approx(5.0, rel=1e-15)
