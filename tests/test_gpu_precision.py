"""Precision forms (FP32, mixed BF16/FP32) against the FP64 oracle.

Per-stage errors are measured at identical inputs so that each stage's own
rounding is isolated:
  * Xi = beta alpha A W          vs the oracle's product with the FP64 factor
  * log pi at the start           vs the oracle's FP64 target
  * merged S, m of one window     vs FP64 moments of the GPU's own visited states
  * factor A after the update     vs numpy's Cholesky of the GPU's own FP64 moments
The sampler as a whole must reproduce the Gaussian posterior moments within 4
Monte Carlo standard errors in every precision.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import diam as od
from oracle import ess as oe
from oracle import targets as ot
from paper_1506_05741_amd import diam, synth


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make(d, P, n_lag, prec, tseed=3, seed=99, N0=None):
    t = synth.gaussian_target(d, tseed)
    x0 = synth.gaussian_exact_draws(t, P, tseed + 7)
    cfg = diam.make_config(d, P, n_lag, prec, seed=seed)
    rdt = torch.float64 if prec == "fp64" else torch.float32
    s = diam.Sampler(cfg, dev(t.mu), dev(t.R, rdt), dev(x0.T))
    S, m = synth.gaussian_warm_moments(t)
    st, _ = s.seed_moments(dev(S), dev(m), N0 if N0 is not None else 10 * P * n_lag)
    assert st == diam.OK
    return t, x0, s


# bounds: fp32 contractions ~ 1e-7 relative; the mixed factor and normals are
# bf16 hi + lo pairs (~2^-17 relative per entry) with fp32 accumulation
XI_TOL = {"fp32": 1e-5, "mixed": 1e-4}
LP_TOL = {"fp32": 1e-4, "mixed": 1e-4}
S_TOL = {"fp32": 1e-5, "mixed": 5e-3}


@pytest.mark.parametrize("prec,P,d,tseed", [("fp32", 32, 256, 3), ("mixed", 32, 256, 3), ("mixed", 64, 256, 3),
                                            ("mixed", 128, 256, 3), ("fp32", 64, 1024, 1), ("mixed", 64, 1024, 1)])
def test_per_stage_error_against_fp64(prec, P, d, tseed):
    # P = 64 and 128 take the mixed form's two-part half target contraction (64 and
    # 128 tiles); d = 1024, seed 1, P = 64 is the d = 1024 configuration's target
    n_lag = 16
    t, x0, s = make(d, P, n_lag, prec, tseed=tseed)
    o = od.DiamOracle(lambda X: ot.gaussian_logpdf(t.R, t.mu, X), d, P, n_lag, 0.3, X=x0)
    S0, m0 = synth.gaussian_warm_moments(t)
    o.seed_moments(S0, m0, 10 * P * n_lag)
    # (b) log density at the start
    lp = host(s.get_f64(diam.F_LOGP, (P,)))
    e_lp = float(np.max(np.abs(lp - o.lp) / (1 + np.abs(o.lp))))
    # (a) proposal contraction on the same W
    W = synth.draw_normals(d, P, n_lag, 1)
    U = synth.draw_uniforms(P, n_lag, 2)
    states = []
    for k in range(n_lag):                                   # one step per call: read every state
        s.step_batch(1, dev(W[k:k + 1]), dev(U[k:k + 1]))
        if k == 0:
            xi = host(s.get(diam.F_XI).view(torch.float32)).reshape(P, d).T.astype(np.float64)
            xi_ref = 0.3 * (o.A @ W[0].T)
            e_xi = rel(xi, xi_ref)
        states.append(host(s.get_f64(diam.F_X, (P, d))).T)
    # (d) merge of the GPU's own visited states vs FP64 moments of those states
    Xw = np.concatenate(states, axis=1)
    N = 10 * P * n_lag
    S_ref = (N * S0 + Xw @ Xw.T) / (N + Xw.shape[1])
    m_ref = (N * m0 + Xw.sum(axis=1)) / (N + Xw.shape[1])
    s.merge_moments()
    S = host(s.get_f64(diam.F_S, (d, d))).T
    m = host(s.get_f64(diam.F_M, (d,)))
    C_ref = S_ref - np.outer(m_ref, m_ref)
    C = S - np.outer(m, m)
    e_S = rel(S, S_ref)
    e_C = rel(C, C_ref)
    e_m = rel(m, m_ref)
    # (e) factor: FP64 Cholesky of the GPU's own moments, then rounding
    st, j = s.update_proposal()
    assert st == diam.OK
    L = host(s.get_f64(diam.F_L, (d, d))).T
    L_ref = np.linalg.cholesky(C)
    e_L = rel(L, L_ref)
    print(f"\n[{prec}] per-stage relative error vs FP64: Xi {e_xi:.3e}  logpi {e_lp:.3e}  "
          f"S {e_S:.3e}  C {e_C:.3e}  m {e_m:.3e}  L {e_L:.3e} (jitter {j})", flush=True)
    assert e_xi < XI_TOL[prec]
    assert e_lp < LP_TOL[prec]
    assert e_S < S_TOL[prec] and e_m < S_TOL[prec]
    assert e_L < (1e-5 if prec == "fp32" else 1e-4)


def _moments_ok(t, X, k_sigma=4.0):
    """X: n x d x P states (window ends).  Means and second central moments of
    v^T x for coordinates, extreme eigenvectors and random unit vectors."""
    n, d, P = X.shape
    V = np.concatenate([np.eye(d)[:, : min(d, 32)], t.Q[:, [0, -1]], synth.unit_vectors(d, 16, 5)], axis=1)
    worst = 0.0
    for j in range(V.shape[1]):
        v = V[:, j]
        f = np.einsum("i,nip->np", v, X)
        for g, truth in ((f, v @ t.mu), ((f - v @ t.mu) ** 2, v @ t.Sigma @ v)):
            ess = oe.ess_chains(g)
            z = abs(g.mean() - truth) / (g.std() / math.sqrt(ess))
            worst = max(worst, z)
    return worst


@pytest.mark.parametrize("prec,d,P", [("fp64", 32, 256), ("fp32", 32, 256), ("mixed", 32, 256), ("mixed", 128, 64)])
def test_posterior_moments_within_4se(prec, d, P):
    # (mixed, 128, 64) runs the two-part half target contraction
    n_lag, windows = 50, 40
    t, x0, s = make(d, P, n_lag, prec, tseed=0, seed=7)
    ends = []
    for _ in range(windows):
        s.step_batch(n_lag)
        s.merge_moments()
        assert s.update_proposal()[0] == diam.OK
        ends.append(host(s.get_f64(diam.F_X, (P, d))).T)
    X = np.stack(ends)
    worst = _moments_ok(t, X)
    acc = host(s.get(diam.F_NACC).view(torch.int32)).sum() / (P * n_lag * windows)
    print(f"\n[{prec}] worst |z| over means and variances: {worst:.2f}, acceptance {acc:.3f}", flush=True)
    assert worst < 4.0
    assert acc > 0.5


def test_mixed_target_reports_a_proposal_outside_the_half_range():
    """The mixed form's Gaussian target takes x - mu in half precision after
    a power-of-two scale per coordinate, chosen at each update from the
    states' spread and the proposal scale with a factor of 1024 of headroom.
    A proposal far beyond that (chains exactly at the mean, a seeded pivot
    100 away with a proposal scale of 1e-4: the contraction toward the pivot
    moves every coordinate by about 4.6) must be reported by the next update
    as an error instead of being rejected silently."""
    d, P, n_lag = 128, 64, 4
    t = synth.gaussian_target(d, 3)
    x0 = np.repeat(t.mu[:, None], P, axis=1)     # d x P, every chain at the mean
    cfg = diam.make_config(d, P, n_lag, "mixed", seed=5)
    s = diam.Sampler(cfg, dev(t.mu), dev(t.R, torch.float32), dev(x0.T))
    m0 = t.mu + 100.0
    S0 = 1e-8 * np.eye(d) + np.outer(m0, m0)
    st, _ = s.seed_moments(dev(S0), dev(m0), 1000.0)
    assert st == diam.OK
    s.step_batch(n_lag)
    s.merge_moments()
    with pytest.raises(diam.DiamError, match="range of the mixed-form target"):
        s.update_proposal()
    s.close()


def test_mixed_target_over_coordinate_scales_from_1e_minus6_to_1e6():
    """The mixed form brings x - mu and R into the half range with power-of-two
    scales per coordinate (from the states' spread and the factor's row norms,
    chosen again at every update) and per row of R.  On a Gaussian whose
    coordinate scales span twelve decades, log pi of the states must match
    FP64 at FP32 level at the start, after the warm-start update and after a
    window of steps evaluated at the new scales."""
    d, P, n_lag = 256, 64, 16
    rng = np.random.default_rng(11)
    sk = 10.0 ** rng.uniform(-6.0, 6.0, d)
    Q = np.linalg.qr(rng.standard_normal((d, d)))[0]
    lam = rng.uniform(0.5, 2.0, d)
    R = (Q / np.sqrt(lam)).T / sk                     # diag(lam)^-1/2 Q^T diag(sk)^-1
    R32 = R.astype(np.float32).astype(np.float64)     # the library reads R in FP32
    mu = sk * rng.standard_normal(d)
    B = (sk[:, None] * Q) * np.sqrt(lam)              # x = mu + B w, w ~ N(0, I)
    Sigma = B @ B.T
    x0 = mu[:, None] + B @ rng.standard_normal((d, P))
    cfg = diam.make_config(d, P, n_lag, "mixed", seed=21)
    s = diam.Sampler(cfg, dev(mu), dev(R, torch.float32), dev(x0.T))

    def check(where):
        X = host(s.get_f64(diam.F_X, (P, d))).T
        y = R32 @ (X - mu[:, None])
        lp_ref = -0.5 * np.sum(y * y, axis=0)
        lp = host(s.get_f64(diam.F_LOGP, (P,)))
        err = float(np.max(np.abs(lp - lp_ref) / (1.0 + np.abs(lp_ref))))
        print(f"\n[{where}] log pi relative error {err:.2e}, log pi mean {lp_ref.mean():.1f}", flush=True)
        # FP32 level: sqrt(d) u32 relative on sums of O(1) terms
        assert err < 4 * math.sqrt(d) * 2.0 ** -24, (where, err)

    check("start")
    S0 = Sigma + np.outer(mu, mu)
    st, _ = s.seed_moments(dev(S0), dev(mu), 10.0 * P * n_lag)
    assert st == diam.OK
    check("after the update")
    nacc = np.zeros(P, dtype=np.int32)
    n = dev(nacc, torch.int32)
    s.step_batch(n_lag, n_accepted=n)
    assert host(n).sum() > 0.5 * P * n_lag            # the states moved: log pi came from the half path
    check("after a window")
    s.merge_moments()
    st, _ = s.update_proposal()
    assert st == diam.OK
    s.step_batch(n_lag)
    check("after a second window")
    s.close()


def test_mixed_step_traces_log_density_and_projections():
    """The mixed form's single-launch step at d = 256 (the target's K-split
    reduction, the decision and the update in one kernel) records per step the
    log density of the current states and their projections: checked against
    the FP64 log density (of the FP32-rounded R the target was given) and the
    FP64 projections of the sampler's own states, after each of three
    single-step calls and after a call of the window's remaining steps."""
    d, P, n_lag = 256, 64, 6
    t, x0, s = make(d, P, n_lag, "mixed", tseed=3)
    proj = np.stack([t.v_max, t.v_min])
    trace = torch.zeros((n_lag, 3, P), dtype=torch.float64, device="cuda")
    s.set_trace(dev(proj), trace)
    R32 = t.R.astype(np.float32).astype(np.float64)

    def check(row, where):
        X = host(s.get_f64(diam.F_X, (P, d))).T
        y = R32 @ (X - t.mu[:, None])
        lp_ref = -0.5 * np.sum(y * y, axis=0)
        tr = host(trace[row])
        err = float(np.max(np.abs(tr[0] - lp_ref) / (1.0 + np.abs(lp_ref))))
        assert err < 4 * math.sqrt(d) * 2.0 ** -24, (where, err)
        assert np.allclose(tr[1:], proj @ X, rtol=1e-12, atol=1e-12), where
        return X

    X = host(s.get_f64(diam.F_X, (P, d))).T
    moved = 0
    for k in range(3):
        s.step_batch(1)
        Xn = check(k, f"single step {k}")
        moved += int(np.any(Xn != X, axis=0).sum())
        X = Xn
    s.step_batch(n_lag - 3)  # the window holds n_lag steps
    check(n_lag - 1, "end of a call of the remaining steps")
    assert moved > P, moved  # most chains accepted at least once in three steps
    s.close()
