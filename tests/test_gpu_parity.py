"""FP64 HIP path vs the FP64 oracle on the same pre-drawn W and U.

Bar (FP64): accept decisions identical away from near-ties (at a near-tie
the oracle takes the GPU's decision and the comparison goes on, see
tests/gpu_parity.py), log alpha within the near-tie threshold, states within 1e-12 relative, merged moments,
factor and pivot within a bound set by the conditioning of the covariance.
The near-tie threshold is |log alpha - log u| < max(1e-9, 10 kappa(C) u d)
and the state tolerance max(1e-12, kappa(C) u): two correct FP64 Cholesky
factorisations of C differ by about kappa(C) u relative, and |z|^2 ~ d
carries that into log alpha, so at d = 1024 (kappa ~ 1e6) two exact
implementations legitimately disagree at the 1e-7 level in log alpha and
1e-12..1e-10 in the states.  At d = 32 both bars are the fixed 1e-9 and
1e-12, and a shared-factor run at d = 1024 (the oracle adopts the GPU's
factor after each update) holds them too.  Sizes span several 64-row tiles with
ragged tails, a degenerate d = 1 chain and the d = 32 / P = 4 / n_lag = 50
configuration from a literal cold start.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import diam as od
from oracle import targets as ot
from paper_1506_05741_amd import diam, synth
from tests.gpu_parity import assert_few_forced, oracle_follow
from tests.philox_ref import gpu_normals_f64, gpu_uniforms

NEAR_TIE = 1e-9


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


class Pair:
    """A GPU sampler and an oracle sampler on the same target and start.

    share_factor: after every factorisation the oracle adopts the GPU's factor
    (and recomputes its z), which takes the legitimate rounding differences
    between two FP64 Cholesky implementations out of the step comparison."""

    def __init__(self, d, P, n_lag, tseed, prec="fp64", warm=False, beta=0.3, seed=1234, x0=None, N0=None,
                 share_factor=False):
        self.share = share_factor
        self.t = t = synth.gaussian_target(d, tseed)
        self.d, self.P, self.n_lag = d, P, n_lag
        if x0 is None:
            x0 = synth.gaussian_exact_draws(t, P, tseed + 50) if warm else np.zeros((d, P))
        self.o = od.DiamOracle(lambda X: ot.gaussian_logpdf(t.R, t.mu, X), d, P, n_lag, beta, X=x0)
        cfg = diam.make_config(d, P, n_lag, prec, beta=beta, seed=seed)
        rdt = torch.float64 if prec == "fp64" else torch.float32
        self.s = diam.Sampler(cfg, dev(t.mu), dev(t.R, rdt), dev(x0.T))
        if warm:
            S, m = synth.gaussian_warm_moments(t)
            n0 = N0 if N0 is not None else 10 * P * n_lag
            st, j = self.s.seed_moments(dev(S), dev(m), n0)
            assert st == diam.OK
            assert self.o.seed_moments(S, m, n0) == od.OK
            assert j == self.o.last_jitter
            self.adopt()

    def adopt(self):
        if self.share:
            d = self.d
            self.o.A = host(self.s.get_f64(diam.F_L, (d, d))).T.copy()
            self.o.Z = od.whiten(self.o.A, self.o.x_ref, self.o.X)

    def gx(self):
        return host(self.s.get_f64(diam.F_X, (self.P, self.d))).T


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def tie_threshold(pr):
    if pr.share:
        return NEAR_TIE
    kappa = np.linalg.cond(pr.o.A) ** 2
    return max(NEAR_TIE, 10.0 * kappa * np.finfo(float).eps * pr.d)


def state_tolerance(pr):
    """1e-12 relative; where the factors are computed independently and C is
    ill-conditioned, kappa(C) u (the agreement two FP64 factorisations allow)."""
    if pr.share:
        return 1e-12
    kappa = np.linalg.cond(pr.o.A) ** 2
    return max(1e-12, kappa * np.finfo(float).eps)


def run_window(pr, W, U, split=None):
    """One window on both sides, the oracle following the GPU through
    near-ties (tests/gpu_parity.py); returns the number of forced decisions."""
    P, n = pr.P, W.shape[0]
    las, accs = [], []
    t0 = 0
    for k in split or [n]:
        pr.s.step_batch(k, dev(W[t0:t0 + k]), dev(U[t0:t0 + k]))
        las.append(host(pr.s.get_f64(diam.F_LA, (k, P))))
        accs.append(host(pr.s.get(diam.F_ACC)).reshape(k, P))
        t0 += k
    la_g = np.concatenate(las)
    acc_g = np.concatenate(accs).astype(bool)
    _, forced = oracle_follow(pr.o, W, U, acc_g, la_g, tie_threshold(pr), where=f"d={pr.d}")
    return forced


def check_states(pr):
    tol = state_tolerance(pr)
    Xg = pr.gx()
    for p in range(pr.P):
        assert rel(Xg[:, p], pr.o.X[:, p]) <= tol, (p, rel(Xg[:, p], pr.o.X[:, p]))
    # the cached log density is the target's value at the state the GPU holds
    lp = host(pr.s.get_f64(diam.F_LOGP, (pr.P,)))
    lp_ref = ot.gaussian_logpdf(pr.t.R, pr.t.mu, Xg)
    assert np.allclose(lp, lp_ref, rtol=1e-10, atol=1e-10)
    if tol <= 1e-12:
        assert np.allclose(lp, pr.o.lp, rtol=1e-10, atol=1e-10)


def check_merge_update(pr, cond_tol=True):
    d = pr.d
    pr.s.merge_moments()
    pr.o.merge_moments()
    S = host(pr.s.get_f64(diam.F_S, (d, d))).T
    m = host(pr.s.get_f64(diam.F_M, (d,)))
    assert rel(S, pr.o.S_glob) <= 1e-12, rel(S, pr.o.S_glob)
    assert rel(m, pr.o.m_glob) <= 1e-12, rel(m, pr.o.m_glob)
    st, j = pr.s.update_proposal()
    assert pr.o.update_proposal() == (od.OK if st == diam.OK else od.E_NOT_PD)
    assert j == pr.o.last_jitter
    L = host(pr.s.get_f64(diam.F_L, (d, d))).T
    C = od.sample_covariance(pr.o.S_glob, pr.o.m_glob)
    kappa = np.linalg.cond(C) if np.all(np.isfinite(C)) else 1.0
    tol = max(1e-12, 100 * kappa * np.finfo(float).eps)
    assert rel(L, pr.o.A) <= tol, (rel(L, pr.o.A), tol)
    assert np.allclose(np.triu(L, 1), 0.0)
    xr = host(pr.s.get_f64(diam.F_XREF, (d,)))
    assert rel(xr, pr.o.x_ref) <= 1e-12
    Z = host(pr.s.get_f64(diam.F_Z, (pr.P, d))).T
    assert rel(Z, pr.o.Z) <= max(1e-10, tol * 10), rel(Z, pr.o.Z)
    pr.adopt()
    return kappa


@pytest.mark.parametrize("case", [
    # d, P, n_lag, target seed, warm, windows, split
    (32, 4, 50, 0, False, 8, None),      # literal cold start of the d = 32 configuration
    (200, 70, 20, 3, True, 3, None),     # 4 row tiles (ragged 8), 2 column tiles (ragged 6)
    (130, 3, 7, 5, True, 3, [3, 4]),     # several calls per window
    (1, 1, 5, 6, False, 4, None),        # degenerate d = 1, one chain
    (1024, 64, 10, 1, True, 2, None),    # the d = 1024, P = 64 configuration, short windows
    (1024, 64, 10, 1, True, 2, "share"), # same, oracle adopts the GPU factor: the strict bar
])
def test_fp64_decision_parity(case):
    d, P, n_lag, tseed, warm, windows, split = case
    share = split == "share"
    split = None if share else split
    log(f"parity d={d} P={P} n_lag={n_lag} warm={warm} windows={windows} shared factor={share}")
    pr = Pair(d, P, n_lag, tseed, warm=warm, share_factor=share)
    lp0 = host(pr.s.get_f64(diam.F_LOGP, (P,)))
    assert np.allclose(lp0, pr.o.lp, rtol=1e-12, atol=1e-12)
    W = synth.draw_normals(d, P, windows * n_lag, 100 + d)
    U = synth.draw_uniforms(P, windows * n_lag, 200 + d)
    forced = 0
    for k in range(windows):
        sl = slice(k * n_lag, (k + 1) * n_lag)
        forced += run_window(pr, W[sl], U[sl], split)
        check_states(pr)
        kappa = check_merge_update(pr)
        log(f"  window {k}: accepted so far {int(pr.o.n_accepted.sum())}, forced near-ties {forced}, "
            f"cond(C) {kappa:.3g}")
    nacc = host(pr.s.get(diam.F_NACC).view(torch.int32))
    assert np.array_equal(nacc, pr.o.n_accepted)
    log(f"  compared: {windows} windows of {n_lag} steps x {P} chains, each merged and refactorised; "
        f"{forced} forced near-ties")
    assert_few_forced(forced, windows * n_lag * P)


def test_philox_draws_match_published_definition():
    d, P, n = 70, 5, 3
    seed = 0x1234_5678_9ABC_DEF0
    t = synth.gaussian_target(d, 0)
    cfg = diam.make_config(d, P, 8, "fp64", seed=seed)
    s = diam.Sampler(cfg, dev(t.mu), dev(t.R), dev(np.zeros((P, d))))
    for s0 in (0, n):
        s.step_batch(n)
        U = host(s.get_f64(diam.F_U, (n, P)))
        assert np.array_equal(U, gpu_uniforms(seed, s0, n, P))
        W = host(s.get_f64(diam.F_W, (n, P, d)))
        ref = gpu_normals_f64(seed, s0, n, d, P)
        assert np.allclose(W, ref, rtol=1e-13, atol=1e-13)
    assert abs(W.mean()) < 0.2 and abs(W.std() - 1) < 0.1


def test_jitter_and_not_pd_follow_the_oracle():
    d, P = 16, 3
    pr = Pair(d, P, 4, 2)
    m = np.linspace(-1, 1, d)
    # S = m m^T gives C = 0 exactly: every pivot fails, jitter level 0 succeeds
    st, j = pr.s.seed_moments(dev(np.outer(m, m)), dev(m), 10.0)
    assert pr.o.seed_moments(np.outer(m, m), m, 10.0) == od.OK
    assert st == diam.OK and j == 0 == pr.o.last_jitter
    L = host(pr.s.get_f64(diam.F_L, (d, d))).T
    assert np.allclose(L, pr.o.A, rtol=1e-12, atol=1e-15)
    # negative definite: every level fails, the factor and pivot are kept
    st, j = pr.s.seed_moments(dev(-np.eye(d)), dev(np.zeros(d)), 10.0)
    assert st == diam.E_NOT_PD and j == 13
    L2 = host(pr.s.get_f64(diam.F_L, (d, d))).T
    assert np.array_equal(L, L2)
    assert np.allclose(host(pr.s.get_f64(diam.F_XREF, (d,))), m)


def test_call_order_is_enforced():
    d, P, n_lag = 8, 2, 4
    pr = Pair(d, P, n_lag, 1)
    with pytest.raises(diam.DiamError) as e:
        pr.s.merge_moments()
    assert e.value.status == diam.E_STATE
    pr.s.step_batch(3)
    with pytest.raises(diam.DiamError) as e:
        pr.s.step_batch(2)
    assert e.value.status == diam.E_STATE
    with pytest.raises(diam.DiamError) as e:
        pr.s.update_proposal()
    assert e.value.status == diam.E_STATE
    pr.s.step_batch(1)
    pr.s.merge_moments()
    assert pr.s.update_proposal()[0] == diam.OK
    st = pr.s.stats()
    assert st["steps"] == 4 and st["windows"] == 1 and st["steps_in_window"] == 0
    assert st["n_samples"] == 4 * P


def test_nan_state_is_always_rejected():
    d, P = 8, 2
    x0 = np.zeros((d, P))
    x0[3, 1] = np.nan
    pr = Pair(d, P, 6, 1, x0=x0)
    W = synth.draw_normals(d, P, 6, 1)
    U = synth.draw_uniforms(P, 6, 2)
    pr.s.step_batch(6, dev(W), dev(U))
    acc = host(pr.s.get(diam.F_ACC)).reshape(6, P).astype(bool)
    assert not acc[:, 1].any()
    for t in range(6):
        a, _ = pr.o.step(W[t].T, U[t])
        assert a[1] == acc[t, 1] and a[0] == acc[t, 0]


def test_runs_are_bitwise_reproducible():
    d, P, n_lag = 96, 8, 16
    outs = []
    for _ in range(2):
        pr = Pair(d, P, n_lag, 4, warm=True, seed=77)
        for _ in range(3):
            pr.s.step_batch(n_lag)
            pr.s.merge_moments()
            pr.s.update_proposal()
        outs.append((host(pr.s.get(diam.F_X)), host(pr.s.get(diam.F_S)), host(pr.s.get(diam.F_L))))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_trace_records_log_density_and_projections():
    d, P, n_lag = 40, 6, 12
    pr = Pair(d, P, n_lag, 2, warm=True)
    proj = np.stack([pr.t.v_max, pr.t.v_min])           # (2, d) == d x 2 column-major
    trace = torch.zeros((2 * n_lag, 3, P), dtype=torch.float64, device="cuda")
    pr.s.set_trace(dev(proj), trace)
    W = synth.draw_normals(d, P, 2 * n_lag, 5)
    U = synth.draw_uniforms(P, 2 * n_lag, 6)
    for k in range(2):
        sl = slice(k * n_lag, (k + 1) * n_lag)
        pr.s.step_batch(n_lag, dev(W[sl]), dev(U[sl]))
        for t in range(k * n_lag, (k + 1) * n_lag):
            pr.o.step(W[t].T, U[t])
            tr = host(trace[t])
            assert np.allclose(tr[0], pr.o.lp, rtol=1e-10, atol=1e-9)
            assert np.allclose(tr[1:], proj @ pr.o.X, rtol=1e-10, atol=1e-10)
        pr.s.merge_moments()
        pr.s.update_proposal()
        pr.o.merge_moments()
        pr.o.update_proposal()


def test_beta_adaptation_follows_the_oracle():
    """Step-size adaptation of Algorithm 1 on both sides: decisions equal step
    for step, beta after every update bitwise equal.  The exact warm start
    with a small beta (every proposal accepted) drives beta up; moments seeded
    with a 9x over-dispersed covariance (proposals far too wide) drive it
    down."""
    d, P, n_lag = 24, 8, 12
    adapt = (0.3, 0.5, 1.25, 0.9)
    for warm, beta0 in ((True, 0.05), (False, 0.6)):
        t = synth.gaussian_target(d, 9)
        pr = Pair(d, P, n_lag, 9, warm=warm, beta=beta0, share_factor=True,
                  x0=synth.gaussian_exact_draws(t, P, 59))
        if not warm:
            S9 = 9.0 * t.Sigma + np.outer(t.mu, t.mu)
            assert pr.s.seed_moments(dev(S9), dev(t.mu), 1e12)[0] == diam.OK
            assert pr.o.seed_moments(S9, t.mu, 1e12) == od.OK
            pr.adopt()
        pr.o.adapt = adapt
        pr.s.set_beta_adaptation(True, *adapt)
        betas = []
        rng = np.random.default_rng(21 if warm else 22)
        for w in range(6):
            W = rng.standard_normal((n_lag, P, d))
            U = synth.draw_uniforms(P, n_lag, 100 + w)
            forced = run_window(pr, W, U)
            assert_few_forced(forced, n_lag * P)
            check_merge_update(pr)
            b = pr.s.stats()["beta"]
            assert b == pr.o.beta, (w, b, pr.o.beta)
            betas.append(b)
        log(f"{'exact' if warm else 'over-dispersed'} start, beta0 {beta0}: beta after each update {betas}")
        assert len(set(betas)) > 1                        # the rule moved beta
    with pytest.raises(diam.DiamError):
        pr.s.set_beta_adaptation(True, 0.5, 0.3, 1.25, 0.9)
    with pytest.raises(diam.DiamError):
        pr.s.set_beta_adaptation(True, 0.3, 0.5, 1.0, 0.9)
    with pytest.raises(diam.DiamError):
        pr.s.set_beta_adaptation(True, 0.3, 0.5, 1.25, 1.5)
    b = pr.s.stats()["beta"]
    pr.s.set_beta_adaptation(False)
    pr.s.step_batch(n_lag)
    pr.s.merge_moments()
    assert pr.s.update_proposal()[0] == diam.OK
    assert pr.s.stats()["beta"] == b                     # off: beta stays
