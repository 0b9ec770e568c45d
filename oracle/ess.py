"""Integrated autocorrelation time and effective sample size.

Test infrastructure only (see ``oracle/__init__.py``).

Section 2.2 (eq. mse) defines the IACT 1 + 2 Theta, Theta = sum_{n>=1} rho_n,
and N_eff = N / IACT.  For a geometric ACF rho_n = rho^n this is
(1 + rho)/(1 - rho); the paper's printed simplification Theta = 1/(1-rho)
drops the n = 0 term and is not used here.  The paper gives no estimator;
this module uses Geyer's initial monotone sequence estimator (Geyer 1992,
"Practical Markov chain Monte Carlo"): sums of adjacent autocovariance pairs
Gamma_m = gamma_{2m} + gamma_{2m+1} are truncated at the first non-positive
pair and made monotone non-increasing.
"""
from __future__ import annotations

import numpy as np


def autocovariance(x: np.ndarray) -> np.ndarray:
    """Biased (1/n) autocovariance of a 1-D series at all lags, via FFT."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    y = x - x.mean()
    m = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(y, m)
    ac = np.fft.irfft(f * np.conj(f), m)[:n]
    return ac / n


def iact(x: np.ndarray) -> float:
    """Integrated autocorrelation time 1 + 2 sum_{n>=1} rho_n (Geyer IMS)."""
    g = autocovariance(x)
    n = g.size
    if g[0] <= 0.0:
        return float("nan")
    npairs = n // 2
    G = g[0:2 * npairs:2] + g[1:2 * npairs:2]
    tot = 0.0
    prev = np.inf
    for m in range(npairs):
        gm = G[m]
        if gm <= 0.0:
            break
        if gm > prev:
            gm = prev
        tot += gm
        prev = gm
    tau = (2.0 * tot - g[0]) / g[0]
    return float(max(tau, 1.0 / n))


def ess_chains(traces: np.ndarray) -> float:
    """Total ESS of P independent chains: sum_p n / tau_p.  traces is n x P."""
    traces = np.asarray(traces, dtype=np.float64)
    n, P = traces.shape
    return float(sum(n / iact(traces[:, p]) for p in range(P)))
