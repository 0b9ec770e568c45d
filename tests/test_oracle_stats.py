"""Statistical and closed-form pins of the oracle sampler, the ESS estimator,
the MLP surrogate and delayed acceptance.

* IACT of an AR(1) with coefficient rho is (1 + rho)/(1 - rho) (Section 2.2,
  eq. mse, with Theta = rho/(1 - rho)); at the exact covariance every DIAM
  proposal is accepted and each whitened coordinate is such an AR(1) with
  rho = sqrt(1 - beta^2), so IACT(v^T x) = 42.42 and, for the log-density
  (a sum of squared AR(1) terms), IACT = (1 + rho^2)/(1 - rho^2) = 21.22.
* Gaussian posterior moments within 4 Monte Carlo standard errors.
* A d = 2 twisted target (the paper's phi, Section 3.1) against bin masses
  from Gauss-Legendre quadrature; chi-square with per-bin variances taken
  from the spread across independent chains.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import roots_legendre

from oracle import diam as od
from oracle import ess as oe
from oracle import mlp as om
from oracle import targets as ot
from paper_1506_05741_amd import synth

BETA = 0.3
RHO = math.sqrt(1 - BETA ** 2)


def _ar1(n, rho, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(n) * math.sqrt(1 - rho * rho)
    x = np.empty(n)
    x[0] = rng.standard_normal()
    for i in range(1, n):
        x[i] = rho * x[i - 1] + e[i]
    return x


@pytest.mark.parametrize("rho", [0.0, 0.5, RHO])
def test_iact_estimator_on_ar1(rho):
    taus = [oe.iact(_ar1(100000, rho, s)) for s in range(4)]
    exact = (1 + rho) / (1 - rho)
    assert abs(np.mean(taus) / exact - 1) < 0.08, (np.mean(taus), exact)


def _warm_gauss(d, P, n_lag, seed=0, N0=None, beta=BETA, alpha=1.0):
    t = synth.gaussian_target(d, seed)
    o = od.DiamOracle(lambda X: ot.gaussian_logpdf(t.R, t.mu, X), d, P, n_lag, beta, alpha=alpha,
                      X=synth.gaussian_exact_draws(t, P, seed + 100))
    S, m = synth.gaussian_warm_moments(t)
    o.seed_moments(S, m, N0 if N0 is not None else 10 * P * n_lag)
    return t, o


def _run(o, n_windows, seed, collect):
    W = synth.draw_normals(o.d, o.P, n_windows * o.n_lag, seed)
    U = synth.draw_uniforms(o.P, n_windows * o.n_lag, seed + 1)
    out = []
    for k in range(n_windows):
        for s in range(o.n_lag):
            i = k * o.n_lag + s
            o.step(W[i].T, U[i])
            out.append(collect(o))
        o.merge_moments()
        o.update_proposal()
    return np.array(out)


def test_iact_closed_form_at_exact_covariance():
    d, P = 8, 8
    t, o = _warm_gauss(d, P, 100, seed=3, N0=1e15)
    v = t.v_max
    tr = _run(o, 150, 21, lambda o: np.concatenate([v @ o.X, o.lp]))
    assert o.n_accepted.min() == 150 * 100         # every proposal accepted
    lin = np.mean([oe.iact(tr[:, p]) for p in range(P)])
    quad = np.mean([oe.iact(tr[:, P + p]) for p in range(P)])
    assert abs(lin / ((1 + RHO) / (1 - RHO)) - 1) < 0.10, lin
    assert abs(quad / ((1 + RHO ** 2) / (1 - RHO ** 2)) - 1) < 0.10, quad


def _moment_check(t, traces_x, k_sigma=4.0):
    """traces_x: n x d x P states.  Checks means and second central moments
    of v^T x for unit vectors v (coordinates, extreme eigenvectors, random)."""
    n, d, P = traces_x.shape
    V = np.concatenate([np.eye(d), t.Q[:, [0, -1]], synth.unit_vectors(d, 16, 77)], axis=1)
    worst = 0.0
    for j in range(V.shape[1]):
        v = V[:, j]
        f = np.einsum("i,nip->np", v, traces_x)        # n x P
        for g, truth in ((f, v @ t.mu), ((f - v @ t.mu) ** 2, v @ t.Sigma @ v)):
            ess = oe.ess_chains(g)
            se = g.std() / math.sqrt(ess)
            z = abs(g.mean() - truth) / se
            worst = max(worst, z)
    assert worst < k_sigma, worst
    return worst


def test_gaussian_moments_within_4se_d8():
    t, o = _warm_gauss(8, 4, 50, seed=5)
    X = _run(o, 160, 31, lambda o: o.X.copy())
    _moment_check(t, X)


@pytest.mark.slow
def test_gaussian_moments_within_4se_config_d32():
    """d = 32, P = 4, n_lag = 50, 2e4 samples per chain, warm protocol."""
    t, o = _warm_gauss(32, 4, 50, seed=0)
    X = _run(o, 400, 41, lambda o: o.X.copy())
    _moment_check(t, X)


def test_moment_check_has_teeth():
    """Samples from a covariance inflated by 10 % must fail the 4-SE check."""
    t = synth.gaussian_target(8, 5)
    Y = synth.gaussian_exact_draws(t, 4 * 4000, 9)
    Y = t.mu[:, None] + 1.1 * (Y - t.mu[:, None])
    with pytest.raises(AssertionError):
        _moment_check(t, Y.reshape(8, 4000, 4).transpose(1, 0, 2))


# ---------------------------------------------------------------------------
# d = 2 twisted target against quadrature
# ---------------------------------------------------------------------------
B_TWIST = 0.5
VAR2 = np.array([1.0, 0.25])
X1_EDGES = np.linspace(-4.0, 4.0, 21)
X2_EDGES = np.linspace(-16.0 * B_TWIST - 2.0, 2.0, 21)


def _bin_masses(b):
    """Mass of every histogram bin by 16 x 16 Gauss-Legendre quadrature."""
    xg, wg = roots_legendre(16)
    n1, n2 = len(X1_EDGES) - 1, len(X2_EDGES) - 1
    masses = np.empty((n1, n2))
    for i in range(n1):
        a1, c1 = X1_EDGES[i], X1_EDGES[i + 1]
        x1 = 0.5 * (c1 - a1) * xg + 0.5 * (c1 + a1)
        w1 = 0.5 * (c1 - a1) * wg
        for j in range(n2):
            a2, c2 = X2_EDGES[j], X2_EDGES[j + 1]
            x2 = 0.5 * (c2 - a2) * xg + 0.5 * (c2 + a2)
            w2 = 0.5 * (c2 - a2) * wg
            G1, G2 = np.meshgrid(x1, x2, indexing="ij")
            pts = np.stack([G1.ravel(), G2.ravel()])
            dens = np.exp(ot.twisted2d_logpdf(pts, b, VAR2)).reshape(16, 16)
            masses[i, j] = w1 @ dens @ w2
    return masses


def _twisted_chains(P=64, n_lag=50, n_windows=400, seed=0):
    lp = lambda X: ot.twisted2d_logpdf(X, B_TWIST, VAR2)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((2, P)) * np.sqrt(VAR2)[:, None]
    x0 = np.stack([y[0], y[1] - B_TWIST * y[0] ** 2])
    o = od.DiamOracle(lp, 2, P, n_lag, BETA, X=x0)
    m = np.array([0.0, -B_TWIST])
    C = np.diag([VAR2[0], VAR2[1] + 2 * B_TWIST ** 2])
    o.seed_moments(C + np.outer(m, m), m, 1000)
    return _run(o, n_windows, seed + 7, lambda o: o.X.copy())


def _chi2_pvalue(X, masses, min_expected=2000):
    """Chi-square of pooled bin frequencies against the quadrature masses.

    The P chains are independent, so each bin's Monte Carlo variance is
    estimated from the spread of the per-chain frequencies; this absorbs the
    autocorrelation of every bin indicator without estimating its IACT."""
    n_steps, _, P = X.shape
    H = np.stack([np.histogram2d(X[:, 0, p], X[:, 1, p], bins=[X1_EDGES, X2_EDGES])[0].ravel()
                  for p in range(P)]) / n_steps
    pb = masses.ravel()
    keep = pb * n_steps * P >= min_expected
    mean = H[:, keep].mean(axis=0)
    var = H[:, keep].var(axis=0, ddof=1) / P
    # each term is approximately F(1, P-1); rescale its mean to 1
    stat = np.sum((mean - pb[keep]) ** 2 / var) * (P - 3) / (P - 1)
    return stats.chi2.sf(stat, int(keep.sum())), int(keep.sum())


def test_twisted_d2_histogram_matches_quadrature():
    masses = _bin_masses(B_TWIST)
    assert abs(masses.sum() - 1.0) < 1e-4
    X = _twisted_chains()
    p, dof = _chi2_pvalue(X, masses)
    assert dof >= 40
    assert p > 1e-3, p
    # a planted mistake in the density (twist off by 10 %) is detected
    p_bad, _ = _chi2_pvalue(X, _bin_masses(1.1 * B_TWIST))
    assert p_bad < 1e-6, p_bad


# ---------------------------------------------------------------------------
# MLP surrogate
# ---------------------------------------------------------------------------
def test_gelu_matches_normal_cdf():
    a = np.linspace(-6, 6, 101)
    assert np.allclose(om.gelu(a), a * stats.norm.cdf(a), rtol=1e-13, atol=1e-15)
    h = 1e-6
    fd = (om.gelu(a + h) - om.gelu(a - h)) / (2 * h)
    assert np.allclose(om.gelu_grad(a), fd, rtol=1e-7, atol=1e-8)


def test_mlp_gradients_match_finite_differences():
    layers = (7, 5, 4, 1)
    params = om.he_init(3, layers)
    rng = np.random.default_rng(4)
    params = [p + 0.1 * rng.standard_normal(p.shape) for p in params]
    Xs = rng.standard_normal((7, 11))
    t = rng.standard_normal(11)
    _, grads = om.loss_and_grad(params, Xs, t)
    h = 1e-6
    for k, p in enumerate(params):
        fd = np.empty_like(p)
        for idx in np.ndindex(p.shape):
            pp = [q.copy() for q in params]
            pp[k][idx] += h
            lp_, _ = om.loss_and_grad(pp, Xs, t)
            pp[k][idx] -= 2 * h
            lm_, _ = om.loss_and_grad(pp, Xs, t)
            fd[idx] = (lp_ - lm_) / (2 * h)
        assert np.allclose(grads[k], fd, rtol=1e-6, atol=1e-9), k


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    p = [rng.standard_normal((3, 2))]
    g = [rng.standard_normal((3, 2))]
    z = [np.zeros((3, 2))]
    out, m, v = om.adam_step(p, g, z, z, 1, lr=1e-3)
    # bias-corrected m/sqrt(v) = g/|g| on the first step
    assert np.allclose(out[0], p[0] - 1e-3 * g[0] / (np.abs(g[0]) + 1e-8), rtol=0, atol=1e-15)


def test_round_bf16():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.14159])
    r = om.round_bf16(vals)
    assert r[0] == 1.0 and r[1] == 1.0            # tie rounds to even
    assert r[2] == 1.0 + 2 ** -7                  # above the half-way point
    assert r[3] == -2.5
    assert abs(r[4] - 3.14159) <= 2 ** -8 * 3.14159


# ---------------------------------------------------------------------------
# Delayed acceptance
# ---------------------------------------------------------------------------
def test_delayed_acceptance_with_exact_surrogate_reduces_to_plain():
    d, P, n = 8, 5, 60
    t, o1 = _warm_gauss(d, P, n, seed=2, N0=200)
    _, o2 = _warm_gauss(d, P, n, seed=2, N0=200)
    W = synth.draw_normals(d, P, n, 3)
    U = synth.draw_uniforms(P, n, 4, stages=2)
    s_cur = o2.lp.copy()
    lp = o2.logpi
    for i in range(n):
        a1, _ = o1.step(W[i].T, U[i, 0])
        a2, pass1, s_cur = o2.step_delayed(W[i].T, U[i, 0], U[i, 1], lp, s_cur)
        assert np.array_equal(a1, a2) and np.array_equal(a1, pass1)
    assert np.array_equal(o1.X, o2.X)


def test_delayed_acceptance_biased_surrogate_is_exact():
    d, P, n_lag = 6, 4, 50
    t, o = _warm_gauss(d, P, n_lag, seed=6, beta=0.6)
    v = t.Q[:, 0]
    bad = lambda X: o.logpi(X) + 0.4 * (v @ (X - t.mu[:, None])) ** 2 + 0.3
    s_cur = bad(o.X)
    n_w = 120
    W = synth.draw_normals(d, P, n_w * n_lag, 12)
    U = synth.draw_uniforms(P, n_w * n_lag, 13, stages=2)
    X = []
    passed = 0
    for k in range(n_w):
        for s in range(n_lag):
            i = k * n_lag + s
            acc, pass1, s_cur = o.step_delayed(W[i].T, U[i, 0], U[i, 1], bad, s_cur)
            passed += pass1.sum()
            X.append(o.X.copy())
        o.merge_moments()
        o.update_proposal()
        s_cur = bad(o.X)
    X = np.array(X)
    # the biased first stage does reject, and the second stage repairs it
    assert o.n_accepted.sum() < passed < n_w * n_lag * P
    _moment_check(t, X)


def test_he_init_scales_by_fan_in():
    """He-normal initialisation (He et al. 2015): weights of the layer from
    fan_in to fan_out inputs are N(0, 2 / fan_in), stored fan_out x fan_in,
    and biases start at zero.  Layers with fan_in != fan_out make a fan-out
    scale (or a transposed shape) fail; each variance is tested against a
    chi-square band of 5 standard deviations, each mean at 5 standard errors."""
    layers = (512, 256, 64, 1)
    params = om.he_init(11, layers)
    assert len(params) == 2 * (len(layers) - 1)
    for k, (fi, fo) in enumerate(zip(layers[:-1], layers[1:])):
        W, b = params[2 * k], params[2 * k + 1]
        assert W.shape == (fo, fi) and b.shape == (fo,)
        assert np.array_equal(b, np.zeros(fo))
        n = W.size
        var = 2.0 / fi
        s2 = float(np.mean(W * W))                     # the mean is known to be 0
        assert abs(s2 / var - 1.0) <= 5.0 * math.sqrt(2.0 / n), (k, s2, var)
        assert abs(W.mean()) <= 5.0 * math.sqrt(var / n), (k, W.mean())
    # the default network is the 512-256-256-1 surrogate
    assert [p.shape for p in om.he_init(0)] == [(256, 512), (256,), (256, 256), (256,), (1, 256), (1,)]
    # reproducible from the seed, different across seeds
    assert all(np.array_equal(a, b) for a, b in zip(om.he_init(5, layers), om.he_init(5, layers)))
    assert not np.array_equal(om.he_init(5, layers)[0], om.he_init(6, layers)[0])
