"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module only *draws* inputs: target parameters, initial states and the
random numbers a sampler consumes.  It holds none of the sampler's
arithmetic (no proposal, acceptance, moment merge or factorisation), so the
CPU oracle and the GPU library can both be fed from it without sharing any
part of the method.

Target recipes
--------------
* Gaussian targets N(mu, Sigma) with Sigma = Q diag(lambda) Q^T,
  lambda_i = i^-2 and Q the sign-fixed orthogonal factor of a seeded
  Gaussian matrix.  The random targets of the paper's numerical section
  (Section 3.1) are dense Gaussians whose density costs one dense
  matrix-vector product; this family keeps that cost and makes the
  conditioning explicit (cond(Sigma) = d^2).  Draw order: the d x d matrix
  G first, then mu, from ``numpy.random.default_rng(seed)``.
  The density is carried by its whitening matrix R = diag(lambda^-1/2) Q^T,
  so that log pi(x) = -1/2 ||R (x - mu)||^2 + const.
* The paper's Gaussian test targets (Section 3.1), mean 0: with A a seeded
  standard normal d x r matrix and B = A A^T, pi_1 = N(0, (B + I)^-1)
  (r = d), pi_2 = N(0, (B/d + I)^-1), pi_3 = pi_1 with r = d/10, and pi_4 =
  N(0, V diag[(sigma^-2 n^-4 + 1)^-1] V^T) with V the eigenvectors of pi_1's
  covariance, smallest variance first, n = 1 .. d (``paper_gaussian``).
* Bayesian logistic regression: design A (n x d, FP32, entries N(0, 1/d)),
  true weights w ~ N(0, I), labels y ~ Bernoulli(sigmoid(A w)), prior
  N(0, prior_var I); draws in that order from ``default_rng(seed)``.
* The batch of many small Gaussians: d_t log-uniform in [128, 3072] drawn
  from ``default_rng(999)``, target t built with seed 1000 + t.

Random numbers of the sampler
-----------------------------
Normals W are stored step-major: ``W[t]`` is a P x d C-ordered block, which
is the d x P column-major matrix the library expects (chain p = column p).
Uniforms lie strictly inside (0, 1): u = (k + 0.5) / 2^52 with k an integer
in [0, 2^52), every value exact in FP64, so log u is always finite and < 0.
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np

__all__ = [
    "GaussianTarget",
    "gaussian_target",
    "gaussian_exact_draws",
    "gaussian_warm_moments",
    "paper_gaussian",
    "twisted_target",
    "twisted_exact_draws",
    "twisted_warm_moments",
    "LogRegData",
    "logreg_data",
    "batch_dims",
    "draw_normals",
    "draw_uniforms",
    "unit_vectors",
]


@dataclass
class GaussianTarget:
    d: int
    mu: np.ndarray      # (d,)    float64
    Q: np.ndarray       # (d, d)  float64, orthogonal, column i <-> lambda_i
    lam: np.ndarray     # (d,)    float64, lambda_i = i^-2
    R: np.ndarray       # (d, d)  float64, R = diag(lambda^-1/2) Q^T
    Sigma: np.ndarray   # (d, d)  float64, Q diag(lambda) Q^T

    @property
    def v_min(self) -> np.ndarray:
        """Eigenvector of the smallest eigenvalue of Sigma."""
        return self.Q[:, -1].copy()

    @property
    def v_max(self) -> np.ndarray:
        """Eigenvector of the largest eigenvalue of Sigma."""
        return self.Q[:, 0].copy()


def gaussian_target(d: int, seed: int) -> GaussianTarget:
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((d, d))
    mu = rng.standard_normal(d)
    Q, Rq = np.linalg.qr(G)
    s = np.sign(np.diag(Rq))
    s[s == 0] = 1.0
    Q = Q * s[None, :]
    i = np.arange(1, d + 1, dtype=np.float64)
    lam = i ** -2.0
    R = i[:, None] * Q.T
    Sigma = (Q * lam[None, :]) @ Q.T
    Sigma = 0.5 * (Sigma + Sigma.T)
    return GaussianTarget(d=d, mu=mu, Q=Q, lam=lam, R=np.ascontiguousarray(R), Sigma=Sigma)


def gaussian_exact_draws(t: GaussianTarget, n: int, seed: int) -> np.ndarray:
    """n exact draws from N(mu, Sigma) as a d x n array (column = draw)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((t.d, n))
    return t.mu[:, None] + t.Q @ (np.sqrt(t.lam)[:, None] * g)


def gaussian_warm_moments(t: GaussianTarget):
    """Exact raw moments (S, m) = (Sigma + mu mu^T, mu) of the target, used to
    seed the global moment accumulators for the warm-start protocol."""
    return t.Sigma + np.outer(t.mu, t.mu), t.mu.copy()


def paper_gaussian(name: str, d: int, seed: int, sigma2: float = None) -> GaussianTarget:
    """pi_1 .. pi_4 of Section 3.1 as a GaussianTarget (mu = 0; Q, lam in
    descending order of variance).  sigma2 is pi_4's data variance (default
    1/d, cond O(d); 1/d^2 gives cond O(d^2))."""
    rng = np.random.default_rng(seed)
    r = d // 10 if name == "pi3" else d
    if r < 1:
        raise ValueError("pi_3 needs d >= 10")
    A = rng.standard_normal((d, r))
    lamB, U = np.linalg.eigh(A @ A.T)          # ascending: U[:, j] has the j-th largest variance of C
    if name in ("pi1", "pi3"):
        lam = 1.0 / (lamB + 1.0)
    elif name == "pi2":
        lam = 1.0 / (lamB / d + 1.0)
    elif name == "pi4":
        s2 = 1.0 / d if sigma2 is None else float(sigma2)
        n = np.arange(d, 0, -1, dtype=np.float64)  # U[:, j] is pi_1's (d - j)-th smallest-variance direction
        lam = 1.0 / (n ** -4.0 / s2 + 1.0)
    else:
        raise ValueError(f"unknown target {name!r}")
    Q = U.copy()
    R = (Q / np.sqrt(lam)[None, :]).T.copy()
    Sigma = (Q * lam[None, :]) @ Q.T
    Sigma = 0.5 * (Sigma + Sigma.T)
    return GaussianTarget(d=d, mu=np.zeros(d), Q=Q, lam=lam, R=R, Sigma=Sigma)


@dataclass
class TwistedTarget:
    d: int
    b: float
    V: np.ndarray        # eigenvectors of C, ascending eigenvalues (first = smallest)
    sig2: np.ndarray     # the eigenvalues (variances of u = V^T x under pi_1)
    R: np.ndarray        # Sigma^-1/2 V^T: y = R x has y_i = u_i / sigma_i
    mu: np.ndarray       # zeros (the maximiser of pi_5 / pi_6 is 0)
    c: np.ndarray        # twist weights on the odd rows (0-based) of y, zero elsewhere


def twisted_target(d: int, seed: int, b: float) -> TwistedTarget:
    """pi_5 (b = 0.3) / pi_6 (b = 2) of Section 3.1: pi_1 = N(0, C), C = (B + I)^-1,
    B = A A^T with A a seeded standard normal d x d matrix; V, sigma^2 the
    ordered eigendecomposition of C (smallest first); twist pairs i = 2, 4,
    ..., d/10 (1-based) with b_i = b sigma_i^-2 / sqrt(d).  The weights c_i =
    b_{i-1} sigma_{i-1}^2 / sigma_i of the whitened form are written to the
    odd rows k = i - 1 (0-based)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d))
    lamB, U = np.linalg.eigh(A @ A.T)                  # ascending eigenvalues of B
    sig2 = 1.0 / (lamB[::-1] + 1.0)                    # eigenvalues of C, ascending
    V = U[:, ::-1].copy()
    R = (V / np.sqrt(sig2)[None, :]).T.copy()
    c = np.zeros(d)
    for i in range(2, d // 10 + 1, 2):
        k = i - 1
        c[k] = (b / sig2[k - 1] / math.sqrt(d)) * sig2[k - 1] / math.sqrt(sig2[k])
    return TwistedTarget(d=d, b=b, V=V, sig2=sig2, R=R, mu=np.zeros(d), c=c)


def twisted_exact_draws(t: TwistedTarget, n: int, seed: int) -> np.ndarray:
    """n exact draws as a d x n array: w ~ N(0, diag(sigma^2)), u = phi^-1(w)
    (u_i = w_i - b_{i-1} w_{i-1}^2 on the twisted pairs), x = V u."""
    rng = np.random.default_rng(seed)
    w = np.sqrt(t.sig2)[:, None] * rng.standard_normal((t.d, n))
    u = w.copy()
    for i in range(2, t.d // 10 + 1, 2):
        k = i - 1
        u[k] = w[k] - (t.b / t.sig2[k - 1] / math.sqrt(t.d)) * w[k - 1] ** 2
    return t.V @ u


def twisted_warm_moments(t: TwistedTarget):
    """Exact raw moments (S, m) of pi_5 / pi_6 for the warm start, from the
    closed forms Section 3.1 gives for u = V^T x: on the twisted pairs
    E[u_i] = -b_{i-1} sigma_{i-1}^2, Var[u_i] = sigma_i^2 + 2 b_{i-1}^2
    sigma_{i-1}^4; elsewhere mean 0 and variance sigma_i^2 (u independent
    across pairs)."""
    mean = np.zeros(t.d)
    var = t.sig2.copy()
    for i in range(2, t.d // 10 + 1, 2):
        k = i - 1
        bk = t.b / t.sig2[k - 1] / math.sqrt(t.d)
        mean[k] = -bk * t.sig2[k - 1]
        var[k] = t.sig2[k] + 2.0 * bk * bk * t.sig2[k - 1] ** 2
    m = t.V @ mean
    return (t.V * var[None, :]) @ t.V.T + np.outer(m, m), m


@dataclass
class LogRegData:
    A: np.ndarray        # (n, d) float32
    y: np.ndarray        # (n,)   float32 in {0, 1}
    w_true: np.ndarray   # (d,)   float64
    prior_var: float


def logreg_data(n: int = 200000, d: int = 512, seed: int = 4, prior_var: float = 10.0) -> LogRegData:
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, d)) * (1.0 / math.sqrt(d))).astype(np.float32)
    w = rng.standard_normal(d)
    t = A.astype(np.float64) @ w
    p = 1.0 / (1.0 + np.exp(-t))
    y = (rng.random(n) < p).astype(np.float32)
    return LogRegData(A=A, y=y, w_true=w, prior_var=prior_var)


def logreg_laplace(data: LogRegData, iters: int = 8):
    """Laplace approximation of the logistic posterior (warm start only):
    the mode by Newton's method from w = 0 and the inverse Hessian there.
    Returns (mode, covariance)."""
    A = data.A.astype(np.float64)
    y = data.y.astype(np.float64)
    d = A.shape[1]
    w = np.zeros(d)
    for _ in range(iters):
        t = A @ w
        s = 1.0 / (1.0 + np.exp(-t))
        g = A.T @ (y - s) - w / data.prior_var
        Hm = (A * (s * (1.0 - s))[:, None]).T @ A + np.eye(d) / data.prior_var
        w = w + np.linalg.solve(Hm, g)
    t = A @ w
    s = 1.0 / (1.0 + np.exp(-t))
    Hm = (A * (s * (1.0 - s))[:, None]).T @ A + np.eye(d) / data.prior_var
    C = np.linalg.inv(Hm)
    return w, 0.5 * (C + C.T)


def batch_dims(n_targets: int = 48, lo: int = 128, hi: int = 3072) -> np.ndarray:
    rng = np.random.default_rng(999)
    u = rng.uniform(math.log(lo), math.log(hi), size=n_targets)
    return np.rint(np.exp(u)).astype(np.int64)


def draw_normals(d: int, P: int, n_steps: int, seed: int) -> np.ndarray:
    """(n_steps, P, d) float64 standard normals; W[t] is column-major d x P."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_steps, P, d))


def draw_uniforms(P: int, n_steps: int, seed: int, stages: int = 1) -> np.ndarray:
    """(n_steps, stages, P) float64 uniforms in the open interval (0, 1)."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 1 << 52, size=(n_steps, stages, P), dtype=np.int64)
    u = (k.astype(np.float64) + 0.5) * (2.0 ** -52)
    return u if stages > 1 else u[:, 0, :]


def unit_vectors(d: int, n: int, seed: int) -> np.ndarray:
    """n seeded random unit vectors as a d x n array."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((d, n))
    return v / np.linalg.norm(v, axis=0, keepdims=True)
