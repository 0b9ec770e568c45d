"""Closed-form integrated autocorrelation times on the GPU path (the d = 32
configuration's target, FP64).

With the proposal factor at chol(Sigma) and the pivot at mu (a warm start
whose pseudo-count dwarfs the run, so the merged moments stay exact), every
log alpha is 0 and the whitened coordinates follow z' = rho z + beta W: an
AR(1) with rho = sqrt(1 - beta^2).  Then IACT(v^T x) = (1 + rho)/(1 - rho)
= 42.42 at beta = 0.3, and log pi = -1/2 |z|^2 (a sum of squared AR(1) terms)
has IACT (1 + rho^2)/(1 - rho^2) = 21.22.  The estimates come from the
library's per-step traces (Geyer's initial monotone sequence, averaged over
the chains).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ess as oe
from paper_1506_05741_amd import diam, synth


def test_closed_form_iact_at_the_exact_covariance():
    d, P, n_lag, windows, beta = 32, 64, 50, 200, 0.3
    rho = math.sqrt(1 - beta * beta)
    t = synth.gaussian_target(d, 0)
    x0 = synth.gaussian_exact_draws(t, P, 1)
    dev = torch.device("cuda")
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    s = diam.Sampler(diam.make_config(d, P, n_lag, "fp64", beta=beta, seed=11), T(t.mu), T(t.R), T(x0.T))
    S0, m0 = synth.gaussian_warm_moments(t)
    assert s.seed_moments(T(S0), T(m0), 1e12)[0] == diam.OK
    trace = torch.zeros((windows * n_lag, 2, P), dtype=torch.float64, device=dev)
    s.set_trace(T(t.v_max[None, :]), trace)
    for _ in range(windows):
        s.step_batch(n_lag)
        s.merge_moments()
        assert s.update_proposal()[0] == diam.OK
    tr = trace.cpu().numpy()
    acc = s.get(diam.F_NACC).view(torch.int32).sum().item() / (P * n_lag * windows)
    tau_lp = np.mean([oe.iact(tr[:, 0, p]) for p in range(P)])
    tau_v = np.mean([oe.iact(tr[:, 1, p]) for p in range(P)])
    exact_v, exact_lp = (1 + rho) / (1 - rho), (1 + rho * rho) / (1 - rho * rho)
    print(f"\n[d=32 exact covariance] acceptance {acc:.4f}; IACT(v_max^T x) {tau_v:.2f} (closed form {exact_v:.2f}), "
          f"IACT(log pi) {tau_lp:.2f} (closed form {exact_lp:.2f})", flush=True)
    assert acc > 0.999
    assert abs(tau_v / exact_v - 1) < 0.1
    assert abs(tau_lp / exact_lp - 1) < 0.1
