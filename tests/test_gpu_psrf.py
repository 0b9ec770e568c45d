"""PSRF on the GPU (Section 2.4.2, M = 1) against the oracle.

The library folds each merged window's stored states into per-chain FP64
accumulators; the states it folds are the window's pivot plus the stored
shift, rounded to the store's precision (FP64, FP32, or bf16 of the FP32
value in the mixed form).  The test reads every visited state after each
step, applies the same rounding to the shift from that window's pivot, and
compares sqrt(R_i) of every coordinate with the oracle's definition-level
computation on those states.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import psrf as op
from paper_1506_05741_amd import diam, synth


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def stored(x, xr, prec):
    """The state the window store represents: pivot + shift in the store's precision."""
    sh = torch.as_tensor(x - xr[None, :])
    if prec == "fp32":
        sh = sh.float().double()
    elif prec == "mixed":
        sh = sh.float().bfloat16().double()
    return xr[None, :] + sh.numpy()


def run(prec, d, P, n_lag, windows, tseed=2, enable_after=0):
    t = synth.gaussian_target(d, tseed)
    x0 = synth.gaussian_exact_draws(t, P, tseed + 5)
    cfg = diam.make_config(d, P, n_lag, prec, seed=17)
    rdt = torch.float64 if prec == "fp64" else torch.float32
    s = diam.Sampler(cfg, dev(t.mu), dev(t.R, rdt), dev(x0.T))
    S0, m0 = synth.gaussian_warm_moments(t)
    assert s.seed_moments(dev(S0), dev(m0), 10 * P * n_lag)[0] == diam.OK
    chains = []
    for w in range(windows):
        if w == enable_after:
            s.psrf_enable(True)
            chains = []
        xr = host(s.get_f64(diam.F_XREF, (d,)))
        for _ in range(n_lag):
            s.step_batch(1)
            chains.append(stored(host(s.get_f64(diam.F_X, (P, d))), xr, prec))
        s.merge_moments()
        assert s.update_proposal()[0] == diam.OK
    return s, np.stack(chains, axis=1)          # (P, n, d)


@pytest.mark.parametrize("prec,d", [("fp64", 40), ("fp32", 40), ("mixed", 40), ("mixed", 42)])
def test_psrf_matches_oracle(prec, d):
    # d = 40: four coordinates per thread; d = 42: one
    P, n_lag = 6, 10
    s, chains = run(prec, d, P, n_lag, windows=4, enable_after=1)
    out, worst = s.psrf()
    ref = op.psrf(chains)
    got = host(out)
    err = np.max(np.abs(got - ref))
    print(f"\n[{prec}] sqrt(R): max |GPU - oracle| {err:.2e} over {d} coordinates, "
          f"n = {chains.shape[1]} states per chain, worst sqrt(R) - 1 = {worst:.3e}", flush=True)
    assert err < 1e-11
    assert worst == pytest.approx(float(np.max(ref - 1.0)), abs=1e-11)


def test_psrf_state_errors_and_restart():
    d, P, n_lag = 16, 4, 6
    t = synth.gaussian_target(d, 1)
    x0 = synth.gaussian_exact_draws(t, P, 2)
    s = diam.Sampler(diam.make_config(d, P, n_lag, "fp64", seed=3), dev(t.mu), dev(t.R), dev(x0.T))
    S0, m0 = synth.gaussian_warm_moments(t)
    assert s.seed_moments(dev(S0), dev(m0), 10 * P * n_lag)[0] == diam.OK
    with pytest.raises(diam.DiamError):
        s.psrf()                                  # not enabled
    s.psrf_enable(True)
    with pytest.raises(diam.DiamError):
        s.psrf()                                  # nothing folded yet
    s.step_batch(n_lag)
    s.merge_moments()
    assert s.update_proposal()[0] == diam.OK
    out1, w1 = s.psrf()
    assert math.isfinite(w1)
    s.psrf_enable(True)                           # restart: the next window alone
    s.step_batch(n_lag)
    s.merge_moments()
    out2, w2 = s.psrf()
    assert not torch.equal(out1, out2)
    s.psrf_enable(False)
    with pytest.raises(diam.DiamError):
        s.psrf()
    one = diam.Sampler(diam.make_config(d, 1, n_lag, "fp64", seed=3), dev(t.mu), dev(t.R), dev(x0[:, :1].T))
    one.psrf_enable(True)
    one.step_batch(n_lag)
    one.merge_moments()
    with pytest.raises(diam.DiamError):
        one.psrf()                                # one chain: no between-chain variance


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_moment_error_matches_oracle(prec):
    """Stopping errors of Section 3.3 on the GPU's merged moments against the
    oracle's evaluation of the same moments."""
    d, P, n_lag = 48, 8, 12
    t = synth.gaussian_target(d, 6)
    x0 = synth.gaussian_exact_draws(t, P, 7)
    rdt = torch.float64 if prec == "fp64" else torch.float32
    s = diam.Sampler(diam.make_config(d, P, n_lag, prec, seed=2), dev(t.mu), dev(t.R, rdt), dev(x0.T))
    S0, m0 = synth.gaussian_warm_moments(t)
    assert s.seed_moments(dev(S0), dev(m0), 2 * P * n_lag)[0] == diam.OK
    for _ in range(3):
        s.step_batch(n_lag)
        s.merge_moments()
        assert s.update_proposal()[0] == diam.OK
    S = host(s.get_f64(diam.F_S, (d, d))).T
    m = host(s.get_f64(diam.F_M, (d,)))
    cov, mean = s.moment_error(dev(t.Sigma), dev(t.mu))
    cov_ref, mean_ref = op.cov_rel_error(S, m, t.Sigma), op.mean_abs_error(m, t.mu)
    print(f"\n[{prec}] covariance rel. Frobenius error {cov:.4e} (oracle {cov_ref:.4e}), "
          f"mean error {mean:.4e} (oracle {mean_ref:.4e})", flush=True)
    assert cov == pytest.approx(cov_ref, rel=1e-10)
    assert mean == pytest.approx(mean_ref, rel=1e-10)
    cov2, mean2 = s.moment_error(dev(t.Sigma))
    assert cov2 == cov and math.isnan(mean2)
