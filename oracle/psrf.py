"""Potential scale reduction factor of P concurrent chains.

Test infrastructure only (see ``oracle/__init__.py``).

Section 2.4.2 defines, from the chain-local moments accumulated over K
batches of M intervals of n_lag steps (eq. winco), the between-chain
quantity B_i and the within-chain quantity W_i of every coordinate i
(eq. btwco) and R_i (eq. psrf); the diagnostic in direction i is sqrt(R_i).
With M = 1 (every chain merges after each interval), chain p's local moments
after K windows are the plain averages over its n = K n_lag visited states:

    m^p = (1/n) sum_t x_t^p,   C^p_ii = (1/n) sum_t (x_t^p)_i^2 - (m^p_i)^2,

and the global mean is the average of the P chain means (equal counts).
Then

    B_i = n/(P-1) sum_p (m^p - m^glob)_i^2,
    W_i = n/((n-1) P) sum_p C^p_ii,
    R_i = (n-1)/n + (P+1)/(P n) B_i / W_i.

The definitions are evaluated directly from all samples, in FP64, with the
second moments taken about each chain's mean (same value as S - m m^T,
without its cancellation).
"""
from __future__ import annotations

import numpy as np


def chain_moments(chains: np.ndarray):
    """chains: (P, n, d) visited states.  Per-chain means (P, d) and
    1/n variances C^p_ii (P, d)."""
    X = np.asarray(chains, dtype=np.float64)
    m = X.mean(axis=1)
    c = ((X - m[:, None, :]) ** 2).mean(axis=1)
    return m, c


def psrf_terms(chains: np.ndarray):
    """B (d,), W (d,), R (d,) of eqs. btwco and psrf for chains (P, n, d)."""
    X = np.asarray(chains, dtype=np.float64)
    P, n, _ = X.shape
    if P < 2 or n < 2:
        raise ValueError("the diagnostic needs at least two chains of at least two states")
    m, c = chain_moments(X)
    mg = m.mean(axis=0)
    B = n / (P - 1) * ((m - mg) ** 2).sum(axis=0)
    W = n / ((n - 1) * P) * c.sum(axis=0)
    R = (n - 1) / n + (P + 1) / (P * n) * B / W
    return B, W, R


def psrf(chains: np.ndarray) -> np.ndarray:
    """sqrt(R_i) for every coordinate i."""
    return np.sqrt(psrf_terms(chains)[2])


# ---- stopping rules of the experiments -----------------------------------------
# Section 3.3 stops a run when the sample covariance is within a relative
# Frobenius-norm TOL of the true covariance (TOL = 1e-3), or, when n_lag is
# tuned, when the sample mean is within a Euclidean-norm TOL of the true mean
# (TOL = 0.01).  The sample moments are the merged raw second moment S and
# mean m: C = S - m m^T (eq. sampcov).

def cov_rel_error(S: np.ndarray, m: np.ndarray, Sigma: np.ndarray) -> float:
    """|S - m m^T - Sigma|_F / |Sigma|_F."""
    C = np.asarray(S, dtype=np.float64) - np.outer(m, m)
    return float(np.linalg.norm(C - Sigma) / np.linalg.norm(Sigma))


def mean_abs_error(m: np.ndarray, mu: np.ndarray) -> float:
    """|m - mu|_2."""
    return float(np.linalg.norm(np.asarray(m, dtype=np.float64) - mu))
