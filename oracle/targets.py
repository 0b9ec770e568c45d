"""Target log-densities, FP64, evaluated column-wise on a d x n block.

Only the unnormalised log-density log eta = log(Z pi) is needed by the sampler
(Section 2.1, eq. bayes: eta can be evaluated pointwise, pi cannot be sampled
directly).  All functions return log eta up to an additive constant.

Test infrastructure only (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import numpy as np


def gaussian_logpdf(R: np.ndarray, mu: np.ndarray, X: np.ndarray) -> np.ndarray:
    """log eta(x) = -1/2 ||R (x - mu)||^2 for each column x of X.

    R is any matrix with R^T R = Sigma^-1 (here the whitening
    diag(lambda^-1/2) Q^T).  The Gaussian test targets of Section 3.1 cost one
    dense matrix-vector product per evaluation, which this keeps.
    Pinned against -1/2 (x-mu)^T Sigma^-1 (x-mu) computed by a LAPACK solve.
    """
    Y = R @ (X - mu[:, None])
    return -0.5 * np.einsum("ij,ij->j", Y, Y)


def logreg_logpdf(A: np.ndarray, y: np.ndarray, prior_var: float, X: np.ndarray) -> np.ndarray:
    """Bayesian logistic regression posterior, unnormalised (Section 2.1, eq. bayes).

    log eta(w) = sum_j [ y_j t_j - softplus(t_j) ] - ||w||^2 / (2 prior_var),
    t = A w, with the stable softplus(t) = max(t, 0) + log1p(exp(-|t|)).
    The likelihood term equals sum_j [y_j log s(t_j) + (1-y_j) log(1 - s(t_j))]
    with s the logistic sigmoid; the tests pin it against that textbook form.
    The FP32 design is promoted to FP64 before the product.
    """
    T = A.astype(np.float64) @ X
    sp = np.maximum(T, 0.0) + np.log1p(np.exp(-np.abs(T)))
    yy = y.astype(np.float64)[:, None]
    return np.sum(yy * T - sp, axis=0) - np.sum(X * X, axis=0) / (2.0 * prior_var)


def twist(x: np.ndarray, b: float) -> np.ndarray:
    """The paper's twisting map phi on d = 2 (Section 3.1): (x1, x2 + b x1^2).

    Its Jacobian determinant is 1, so if x ~ N(0, C) then phi^-1 pushes the
    Gaussian density through without a volume factor.
    """
    out = np.array(x, dtype=np.float64, copy=True)
    out[1] = out[1] + b * out[0] ** 2
    return out


def twisted2d_logpdf(X: np.ndarray, b: float, var: np.ndarray) -> np.ndarray:
    """log density of the "boomerang" target pi = N(0, diag(var)) o phi on d = 2.

    pi(x) = N(phi(x); 0, diag(var)), exactly normalised because det(dphi) = 1.
    """
    Y = twist(X, b)
    return (-0.5 * (Y[0] ** 2 / var[0] + Y[1] ** 2 / var[1])
            - 0.5 * np.log((2.0 * np.pi) ** 2 * var[0] * var[1]))


def twisted_logpdf(R: np.ndarray, mu: np.ndarray, c: np.ndarray, X: np.ndarray) -> np.ndarray:
    """The twisted Gaussians of Section 3.1 (pi_5, pi_6) in whitened form.

    pi = pi_1 o V o phi o V^T with pi_1 = N(0, V Sigma V^T) and
    phi(u)_i = u_i + b_{i-1} u_{i-1}^2 on the pairs i = 2, 4, ..., d/10 (1-based).
    With y = R (x - mu), R = Sigma^-1/2 V^T (so y_i = u_i / sigma_i), the
    density is -1/2 sum_i z_i^2 with z_i = y_i + c_i y_{i-1}^2 on the twisted
    rows, c_i = b_{i-1} sigma_{i-1}^2 / sigma_i, and z_i = y_i elsewhere.  The
    pairs are rows (2k, 2k+1) 0-based; c is read at the odd rows only.  No
    Jacobian term: det(d phi) = 1.  Up to the normalising constant.
    """
    Y = R @ (X - mu[:, None])
    Z = Y.copy()
    Z[1::2] += c[1::2, None] * Y[0:Y.shape[0] - Y.shape[0] % 2:2] ** 2
    return -0.5 * np.sum(Z * Z, axis=0)


def twisted_u_moments(sig2: np.ndarray, b: float):
    """Exact mean and variance of u = V^T x under pi_5 / pi_6 (Section 3.1):
    for i = 2, 4, ..., d/10 (1-based), E[u_i] = -b_{i-1} sigma_{i-1}^2 and
    Var[u_i] = sigma_i^2 + 2 b_{i-1}^2 sigma_{i-1}^4 with b_i = b sigma_i^-2 / sqrt(d);
    mean 0 and variance sigma_i^2 for the other coordinates."""
    d = sig2.size
    mean = np.zeros(d)
    var = np.array(sig2, dtype=np.float64, copy=True)
    for i in range(2, d // 10 + 1, 2):
        k = i - 1                                        # 0-based twisted row; k - 1 is its partner
        bp = b / sig2[k - 1] / np.sqrt(d)
        mean[k] = -bp * sig2[k - 1]
        var[k] = sig2[k] + 2.0 * bp ** 2 * sig2[k - 1] ** 2
    return mean, var
