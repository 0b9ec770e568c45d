"""Pins of the oracle's other proposal families (Section 2.3): random walk
(eq. rw), pCN (eq. pcn) and adaptive Metropolis (RW with the adapted factor).

* Hand-worked one-dimensional steps: RW accepts with log pi(x') - log pi(x);
  pCN on a target equal to its prior N(0, 1) accepts every proposal.
* pCN's log alpha is the likelihood ratio alone: for pi_1 = N(0, (B + I)^-1)
  with the prior N(0, I), log alpha = -1/2 x'^T B x' + 1/2 x^T B x, with B
  obtained by inverting the covariance (LAPACK), not from the oracle.
* The fixed families keep their factor and pivot at an update (beta still
  adapts); AM refactorises like DIAM.
* Each family reproduces a Gaussian's mean and second moments within 4 MC
  standard errors; a random walk that contracts toward 0 like pCN but keeps
  the symmetric acceptance (a planted mistake) fails the same check.
"""
import math

import numpy as np
import pytest

from oracle import diam as od
from oracle import ess as oe
from oracle import targets as ot
from paper_1506_05741_amd import synth


def std_normal_1d(X):
    return -0.5 * X[0] ** 2


@pytest.mark.parametrize("prop", ["rw", "am"])
def test_walk_step_hand_worked(prop):
    # x = 0.4, A = I, beta = 0.5, W = 1: x' = 0.9,
    # log alpha = -0.81/2 + 0.16/2 = -0.325
    o = od.DiamOracle(std_normal_1d, 1, 1, 5, 0.5, X=np.array([[0.4]]), proposal=prop)
    acc, la = o.step(np.array([[1.0]]), np.array([0.5]))
    assert la[0] == pytest.approx(-0.325, abs=1e-15)
    assert acc[0] == (math.log(0.5) < -0.325)
    assert o.X[0, 0] == pytest.approx(0.9 if acc[0] else 0.4, abs=1e-15)


def test_pcn_on_its_own_prior_accepts_everything():
    # pi = N(0, 1) = the prior: the pCN proposal leaves it invariant, log alpha = 0
    o = od.DiamOracle(std_normal_1d, 1, 3, 5, 0.5, X=np.array([[0.4, -1.3, 2.2]]), proposal="pcn")
    W = np.array([[1.0, -0.7, 0.3]])
    acc, la = o.step(W, np.array([1 - 1e-15] * 3))
    np.testing.assert_allclose(la, 0.0, atol=1e-14)
    assert acc.all()
    np.testing.assert_allclose(o.X[0], math.sqrt(0.75) * np.array([0.4, -1.3, 2.2]) + 0.5 * W[0], rtol=1e-15)


def test_pcn_log_alpha_is_the_likelihood_ratio():
    d, P = 12, 5
    t = synth.paper_gaussian("pi1", d, 4)
    B = np.linalg.inv(t.Sigma) - np.eye(d)               # likelihood precision of pi_1 = N(0, (B + I)^-1)
    X = synth.gaussian_exact_draws(t, P, 5)
    o = od.DiamOracle(lambda Y: ot.gaussian_logpdf(t.R, t.mu, Y), d, P, 10, 0.6, X=X, proposal="pcn")
    W = np.random.default_rng(6).standard_normal((d, P))
    Xp = math.sqrt(1 - 0.36) * X + 0.6 * W
    _, la = o.step(W, np.full(P, 0.5))
    ref = -0.5 * np.einsum("ip,ij,jp->p", Xp, B, Xp) + 0.5 * np.einsum("ip,ij,jp->p", X, B, X)
    np.testing.assert_allclose(la, ref, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("prop", ["diam", "am", "pcn", "rw"])
def test_update_refactors_only_the_adaptive_families(prop):
    d, P, n_lag = 6, 4, 8
    t = synth.gaussian_target(d, 1)
    o = od.DiamOracle(lambda Y: ot.gaussian_logpdf(t.R, t.mu, Y), d, P, n_lag, 0.3, X=synth.gaussian_exact_draws(t, P, 2),
                      proposal=prop, adapt=(0.3, 0.5, 1.5, 1.0))
    rng = np.random.default_rng(3)
    for k in range(n_lag):
        o.step(rng.standard_normal((d, P)), np.full(P, 1e-300))   # u tiny: every finite log alpha accepts
    o.merge_moments()
    assert o.update_proposal() == od.OK
    assert o.beta == pytest.approx(0.45)                           # all accepted: beta * 1.5
    if prop in ("pcn", "rw"):
        assert np.array_equal(o.A, np.eye(d)) and np.all(o.x_ref == 0)
    else:
        assert not np.array_equal(o.A, np.eye(d))
        np.testing.assert_allclose(o.x_ref, o.m_glob)


def _moments_within_4se(o, t, windows, seed):
    rng = np.random.default_rng(seed)
    ends = []
    for w in range(windows):
        o.run_window(rng.standard_normal((o.n_lag, o.P, o.d)), synth.draw_uniforms(o.P, o.n_lag, 500 + w + 97 * seed))
        ends.append(o.X.copy())
    Xs = np.stack(ends)                                   # windows x d x P
    worst = 0.0
    for v, lam in ((t.v_max, t.lam[0]), (t.v_min, t.lam[-1])):
        f1 = np.einsum("i,wip->wp", v, Xs)
        f2 = (f1 - v @ t.mu) ** 2
        for f, truth in ((f1, v @ t.mu), (f2, lam)):
            ess = oe.ess_chains(f)
            worst = max(worst, abs(f.mean() - truth) / (f.std() / math.sqrt(ess)))
    return worst


def _family_run(prop, t, beta, band):
    d, P, n_lag = t.d, 16, 25
    o = od.DiamOracle(lambda Y: ot.gaussian_logpdf(t.R, t.mu, Y), d, P, n_lag, beta,
                      X=synth.gaussian_exact_draws(t, P, 11), proposal=prop, adapt=band + (1.2, 1.0))
    if prop == "am":
        S0, m0 = synth.gaussian_warm_moments(t)
        assert o.seed_moments(S0, m0, 10 * P * n_lag) == od.OK
    return o


@pytest.mark.parametrize("prop,band", [("am", (0.1, 0.3)), ("pcn", (0.3, 0.5)), ("rw", (0.1, 0.3))])
def test_family_reproduces_gaussian_moments(prop, band):
    t = synth.gaussian_target(4, 7)                       # cond 16, mean ~ N(0, I)
    o = _family_run(prop, t, od.initial_beta(4), band)
    worst = _moments_within_4se(o, t, 160, 1)
    assert worst < 4.0, worst


def test_contracting_walk_with_symmetric_acceptance_fails(monkeypatch):
    # planted mistake: the pCN contraction toward 0 with the random walk's
    # acceptance; the chains then target a distribution pulled toward 0
    def wrong(X, A, W, beta, alpha=1.0):
        return math.sqrt(1.0 - beta * beta) * X + beta * alpha * (A @ W)
    monkeypatch.setattr(od, "rw_proposal", wrong)
    t = synth.gaussian_target(4, 7)
    o = _family_run("rw", t, od.initial_beta(4), (0.1, 0.3))
    assert _moments_within_4se(o, t, 160, 1) > 4.0
