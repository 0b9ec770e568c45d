"""Twisted Gaussian targets (Section 3.1's pi_5 / pi_6) on the GPU.

* FP64 path against the oracle on pi_6 (b = 2) with an inflated proposal
  (alpha = 1.3): log pi at the start, then decision parity (the oracle
  following the GPU through near-ties), log alpha, states, merged moments and
  factor over several windows.
* FP32 and mixed paths: log pi at the start against the FP64 definition, with
  a twist weight on every odd row so that every tile (and, in the mixed form,
  both split-target tile shapes) applies the pairing.
* pi_5 (b = 0.3, d = 100 as in the paper) in the mixed form: the posterior
  mean and variance of u = V^T x within 4 Monte Carlo standard errors of the
  paper's closed forms.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import diam as od
from oracle import ess as oe
from oracle import targets as ot
from paper_1506_05741_amd import diam, synth
from tests.gpu_parity import assert_few_forced, oracle_follow


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def exact_moments(t):
    mu_u, var_u = ot.twisted_u_moments(t.sig2, t.b)
    m = t.V @ mu_u
    return t.V @ np.diag(var_u) @ t.V.T + np.outer(m, m), m, mu_u, var_u


@pytest.mark.parametrize("d", [40, 130])
def test_fp64_twisted_decision_parity(d):
    P, n_lag, alpha = 8, 10, 1.3
    t = synth.twisted_target(d, 11, 2.0)
    x0 = synth.twisted_exact_draws(t, P, 12)
    cfg = diam.make_config(d, P, n_lag, "fp64", beta=0.4, alpha=alpha, seed=5)
    s = diam.Sampler(cfg, dev(t.mu), dev(t.R), dev(x0.T), twist=dev(t.c))
    o = od.DiamOracle(lambda X: ot.twisted_logpdf(t.R, t.mu, t.c, X), d, P, n_lag, 0.4, alpha=alpha, X=x0)
    S0, m0, _, _ = exact_moments(t)
    assert s.seed_moments(dev(S0), dev(m0), 10 * P * n_lag)[0] == diam.OK
    assert o.seed_moments(S0, m0, 10 * P * n_lag) == od.OK
    lp = host(s.get_f64(diam.F_LOGP, (P,)))
    np.testing.assert_allclose(lp, o.lp, rtol=1e-12, atol=1e-12)
    o.A = host(s.get_f64(diam.F_L, (d, d))).T.copy()       # the GPU's factor (independent FP64 roundings)
    o.Z = od.whiten(o.A, o.x_ref, o.X)
    rng = np.random.default_rng(3)
    total = forced = 0
    for w in range(3):
        W = rng.standard_normal((n_lag, P, d))
        U = synth.draw_uniforms(P, n_lag, 40 + w)
        s.step_batch(n_lag, dev(W), dev(U))
        acc_g = host(s.get(diam.F_ACC)).reshape(n_lag, P).astype(bool)
        la_g = host(s.get_f64(diam.F_LA, (n_lag, P)))
        a, f = oracle_follow(o, W, U, acc_g, la_g, 1e-9, where=f"twisted d={d} window {w}")
        total, forced = total + a, forced + f
        X = host(s.get_f64(diam.F_X, (P, d))).T
        assert np.linalg.norm(X - o.X) <= 1e-12 * np.linalg.norm(o.X)
        s.merge_moments()
        o.merge_moments()
        assert s.update_proposal()[0] == diam.OK
        assert o.update_proposal() == od.OK
        o.A = host(s.get_f64(diam.F_L, (d, d))).T.copy()   # adopt the GPU's factor (independent FP64 roundings)
        o.Z = od.whiten(o.A, o.x_ref, o.X)
    print(f"\n[fp64 twisted d={d}] compared 3 windows decision-for-decision, each merged and refactorised: "
          f"{total} accepted of {3 * n_lag * P}, {forced} forced near-ties", flush=True)
    assert_few_forced(forced, 3 * n_lag * P)
    assert total > 0


@pytest.mark.parametrize("prec,d,P", [("fp32", 130, 16), ("mixed", 128, 64), ("mixed", 256, 128)])
def test_twisted_log_density_against_fp64(prec, d, P):
    # every odd row twisted, weights of either sign, on a dense Gaussian of the benchmark family
    t = synth.gaussian_target(d, 4)
    c = np.zeros(d)
    c[1::2] = np.random.default_rng(6).uniform(-0.4, 0.4, d // 2)
    x0 = synth.gaussian_exact_draws(t, P, 5)
    cfg = diam.make_config(d, P, 8, prec, seed=5)
    s = diam.Sampler(cfg, dev(t.mu), dev(t.R, torch.float32), dev(x0.T), twist=dev(c))
    lp = host(s.get_f64(diam.F_LOGP, (P,)))
    ref = ot.twisted_logpdf(t.R, t.mu, c, x0)
    err = np.max(np.abs(lp - ref) / (1 + np.abs(ref)))
    print(f"\n[{prec} d={d} P={P}] twisted log pi vs FP64: max rel error {err:.2e}", flush=True)
    assert err < 1e-4


def test_mixed_pi5_moments_within_4se():
    # beta = 0.3 keeps the acceptance inside Section 3.2's band (about 0.47 here).
    # With beta = 0.5 (acceptance about 0.24) and half the windows, the FP64
    # oracle itself under-estimates the twisted variances by up to 4.5 SE on
    # some seeds: the heavy tail is visited too rarely in so short a run
    d, P, n_lag, alpha, beta, windows = 100, 64, 50, 1.2, 0.3, 120
    t = synth.twisted_target(d, 21, 0.3)
    x0 = synth.twisted_exact_draws(t, P, 22)
    cfg = diam.make_config(d, P, n_lag, "mixed", beta=beta, alpha=alpha, seed=8)
    s = diam.Sampler(cfg, dev(t.mu), dev(t.R, torch.float32), dev(x0.T), twist=dev(t.c))
    S0, m0, mu_u, var_u = exact_moments(t)
    assert s.seed_moments(dev(S0), dev(m0), 10 * P * n_lag)[0] == diam.OK
    ends = []
    for _ in range(windows):
        s.step_batch(n_lag)
        s.merge_moments()
        assert s.update_proposal()[0] == diam.OK
        ends.append(t.V.T @ host(s.get_f64(diam.F_X, (P, d))).T)
    U = np.stack(ends)
    worst = 0.0
    zs = []
    for k in list(range(0, 10)) + [d - 1]:
        for f, truth in ((U[:, k, :], mu_u[k]), ((U[:, k, :] - mu_u[k]) ** 2, var_u[k])):
            ess = oe.ess_chains(f)
            z = (f.mean() - truth) / (f.std() / math.sqrt(ess))
            zs.append(round(float(z), 2))
            worst = max(worst, abs(z))
    acc = host(s.get(diam.F_NACC).view(torch.int32)).sum() / (P * n_lag * windows)
    print(f"\n[mixed pi_5 d=100] worst |z| {worst:.2f} over the twisted and some untwisted coordinates, "
          f"acceptance {acc:.3f}; z (mean, variance) per coordinate: {zs}", flush=True)
    assert worst < 4.0
