"""Pins of the oracle's local-global logistics (Section 2.4.1 with M > 1).

* Two-pass definitions: between global merges, chain p's covariance
  C^{p,glob} and pivot m^{p,glob} (eqs. mom2pg, mom1pg, cov2pg) equal the
  1/n covariance and mean, computed from scratch, of every state merged
  globally so far pooled with chain p's own states of the current batch; the
  global moments after M intervals equal those of every state of every chain.
* Each chain then proposes with its own factor and pivot: x' = x_ref_p +
  rho (x - x_ref_p) + beta L_p W, with L_p L_p^T = C^{p,glob}.
* Chain by chain, the proposal keeps the chain's own reference Gaussian
  N(x_ref_p, L_p L_p^T) invariant: with that Gaussian as the target, the
  chain's log alpha is 0; accepting with the shared pair's whitening while
  proposing with the per-chain pairs (a planted mistake) breaks it.
* The sampler with M = 4 reproduces a Gaussian's moments within 4 MC
  standard errors.
"""
import math

import numpy as np
import pytest

from oracle import diam as od
from oracle import ess as oe
from oracle import targets as ot
from paper_1506_05741_amd import synth


def pooled(states):
    X = np.concatenate(states, axis=1)
    m = X.mean(axis=1)
    return ((X - m[:, None]) @ (X - m[:, None]).T) / X.shape[1], m


def test_local_global_moments_are_the_pooled_two_pass_ones():
    d, P, n_lag, M = 5, 3, 8, 3
    t = synth.gaussian_target(d, 2)
    o = od.DiamOracle(lambda X: ot.gaussian_logpdf(t.R, t.mu, X), d, P, n_lag, 0.4,
                      X=synth.gaussian_exact_draws(t, P, 3), M=M)
    rng = np.random.default_rng(4)
    merged = []                                   # every state merged globally
    batch = [[] for _ in range(P)]                # chain p's states of the current batch
    for k in range(2 * M + 1):
        for _ in range(n_lag):
            o.step(rng.standard_normal((d, P)), np.full(P, 1e-300))   # every finite log alpha accepts
            for p in range(P):
                batch[p].append(o.X[:, p:p + 1].copy())
        o.merge_moments()
        if (k + 1) % M == 0:
            for p in range(P):
                merged += batch[p]
                batch[p] = []
            assert o.m_int == 0
            C, m = pooled(merged)
            np.testing.assert_allclose(od.sample_covariance(o.S_glob, o.m_glob), C, rtol=1e-10, atol=1e-12)
            np.testing.assert_allclose(o.m_glob, m, rtol=1e-10, atol=1e-12)
        assert o.update_proposal() == od.OK
        if o.m_int > 0:
            for p in range(P):
                C, m = pooled(merged + batch[p])
                np.testing.assert_allclose(o.Ap[p] @ o.Ap[p].T, C, rtol=1e-9, atol=1e-12)
                np.testing.assert_allclose(o.xrp[:, p], m, rtol=1e-10, atol=1e-12)
        else:
            assert o.Ap is None
            C, m = pooled(merged)
            np.testing.assert_allclose(o.A @ o.A.T, C, rtol=1e-9, atol=1e-12)


def test_each_chain_proposes_with_its_own_factor():
    d, P, n_lag = 4, 3, 6
    t = synth.gaussian_target(d, 5)
    o = od.DiamOracle(lambda X: ot.gaussian_logpdf(t.R, t.mu, X), d, P, n_lag, 0.6,
                      X=synth.gaussian_exact_draws(t, P, 6), M=2)
    S0, m0 = synth.gaussian_warm_moments(t)
    assert o.seed_moments(S0, m0, 12) == od.OK              # few pseudo-samples: chains differ
    rng = np.random.default_rng(8)
    for _ in range(n_lag):
        o.step(rng.standard_normal((d, P)), np.full(P, 1e-300))
    o.merge_moments()
    assert o.update_proposal() == od.OK and o.Ap is not None
    assert not np.allclose(o.Ap[0], o.Ap[1])
    X0 = o.X.copy()
    W = rng.standard_normal((d, P))
    o.step(W, np.full(P, 1e-300))
    rho = math.sqrt(1 - 0.36)
    for p in range(P):
        C = o.Ap[p] @ o.Ap[p].T
        L = np.linalg.cholesky(C)                            # LAPACK, from the covariance
        expect = o.xrp[:, p] + rho * (X0[:, p] - o.xrp[:, p]) + 0.6 * L @ W[:, p]
        np.testing.assert_allclose(o.X[:, p], expect, rtol=1e-10, atol=1e-12)


def _local_global_run(t, M, windows, seed):
    d, P, n_lag = t.d, 8, 25
    o = od.DiamOracle(lambda X: ot.gaussian_logpdf(t.R, t.mu, X), d, P, n_lag, 0.5,
                      X=synth.gaussian_exact_draws(t, P, 11), M=M)
    S0, m0 = synth.gaussian_warm_moments(t)
    assert o.seed_moments(S0, m0, P * n_lag) == od.OK       # one window's weight: the local moments matter
    rng = np.random.default_rng(seed)
    ends = []
    for w in range(windows):
        o.run_window(rng.standard_normal((n_lag, P, d)), synth.draw_uniforms(P, n_lag, 900 + w + 31 * seed))
        ends.append(o.X.copy())
    Xs = np.stack(ends)
    worst = 0.0
    for v, lam in ((t.v_max, t.lam[0]), (t.v_min, t.lam[-1])):
        f1 = np.einsum("i,wip->wp", v, Xs)
        for f, truth in ((f1, v @ t.mu), ((f1 - v @ t.mu) ** 2, lam)):
            ess = oe.ess_chains(f)
            worst = max(worst, abs(f.mean() - truth) / (f.std() / math.sqrt(ess)))
    return worst


def test_local_global_sampler_reproduces_gaussian_moments():
    t = synth.gaussian_target(4, 13)
    assert _local_global_run(t, 4, 200, 1) < 4.0


def _local_state():
    """An oracle after one local update whose chains hold distinct factors."""
    d, P, n_lag = 4, 3, 6
    t = synth.gaussian_target(d, 5)
    o = od.DiamOracle(lambda X: ot.gaussian_logpdf(t.R, t.mu, X), d, P, n_lag, 0.6,
                      X=synth.gaussian_exact_draws(t, P, 6), M=2)
    S0, m0 = synth.gaussian_warm_moments(t)
    assert o.seed_moments(S0, m0, 12) == od.OK
    rng = np.random.default_rng(8)
    for _ in range(n_lag):
        o.step(rng.standard_normal((d, P)), np.full(P, 1e-300))
    o.merge_moments()
    assert o.update_proposal() == od.OK and o.Ap is not None
    return o


def _la_at_own_reference(o, q):
    """log alpha of one step when the target is chain q's reference Gaussian
    N(x_ref_q, A_q A_q^T) (its log density through a LAPACK solve)."""
    Aq, xq = o.Ap[q].copy(), o.xrp[:, q].copy()

    def logpi(X):
        Y = np.linalg.solve(Aq @ Aq.T, X - xq[:, None])
        return -0.5 * np.sum((X - xq[:, None]) * Y, axis=0)
    o.logpi = logpi
    o.lp = logpi(o.X)
    _, la = o.step(np.random.default_rng(20 + q).standard_normal((o.d, o.P)), np.full(o.P, 0.5))
    return la


def test_each_chain_leaves_its_own_reference_gaussian_invariant():
    # eq. diam keeps N(x_ref, A A^T) invariant; with per-chain pairs this holds
    # chain by chain: log alpha = 0 exactly for the chain whose pair defines the target
    for q in range(3):
        la = _la_at_own_reference(_local_state(), q)
        assert abs(la[q]) < 1e-10, (q, la)
        assert np.all(np.abs(np.delete(la, q)) > 1e-6)


def test_shared_whitening_with_per_chain_proposals_fails(monkeypatch):
    # planted mistake: chains propose with their own (L_p, x_ref_p) but the
    # acceptance whitens with the shared pair
    real, held = od.whiten, []
    monkeypatch.setattr(od, "whiten", lambda A, x_ref, X: real(held[0].A, held[0].x_ref, X) if held
                        else real(A, x_ref, X))
    o = _local_state()
    held.append(o)
    la = _la_at_own_reference(o, 0)
    assert abs(la[0]) > 1e-3
