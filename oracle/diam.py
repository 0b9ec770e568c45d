"""DIAM with P concurrent chains, FP64, in the paper's order of operations.

Test infrastructure only (see ``oracle/__init__.py``).

The sampler follows Algorithm 1 (Section 4.3) for every chain, with the
concurrent-chain logistics of Section 2.4.1 in their M = 1 form: every n_lag
steps all P chains merge their local moments into the global ones (eqs.
mom2p, mom1p, mom2g, mom1g) and one shared proposal factor is refactorised
from the merged covariance (eq. sampcov).  Readings where the paper is
silent or garbled are stated at each use:

* The quadratic correction uses A^-1 (x - x_ref): the proposal (eq. diamnl)
  leaves N(x_ref, alpha^2 A A^T) invariant, and Algorithm 1 prints the
  x_ref = 0 case.  The factor 1/(2 alpha^2) uses the inflation alpha.
* After every proposal update the correction of the *current* states is
  recomputed under the new (A, x_ref); both states entering one acceptance
  ratio are then measured by the same kernel.
* x_ref = 0 until the first merge, then the merged mean, constant within a
  window.
* Every visited state of every step enters the moments, repeats after a
  rejection included; local moments use the running 1/(m n_lag) average
  (the printed recursion is off by a factor n_lag in one term).
* C_n uses the 1/n normalisation printed in eq. sampcov.
* Acceptance is strict: accept iff log u < log alpha; NaN rejects.
* Cholesky failure: retry on Cov + eps_j I with eps_j = 10^j * jitter0 *
  s, s = tr(Cov)/d if that is positive and finite else 1, j = 0, 1, ...,
  tries-1; if every try fails the previous factor is kept.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

OK = 0
E_NOT_PD = -4


def initial_beta(d):
    """Algorithm 1's initial step size min(2.4 / sqrt(d), 0.5)."""
    return min(2.4 / math.sqrt(d), 0.5)


def diam_proposal(X, x_ref, A, W, beta, alpha=1.0):
    """x' = x_ref + sqrt(1 - beta^2) (x - x_ref) + beta alpha A W
    (Section 2.3.4, eq. diam; the inflation alpha of eq. diamnl)."""
    rho = math.sqrt(1.0 - beta * beta)
    return x_ref[:, None] + rho * (X - x_ref[:, None]) + beta * alpha * (A @ W)


def rw_proposal(X, A, W, beta, alpha=1.0):
    """x' = x + beta alpha A W: the random walk of Section 2.3.1 (eq. rw), and
    adaptive Metropolis (Section 2.3.3) when A factors the sample covariance."""
    return X + beta * alpha * (A @ W)


def symmetric_log_accept_ratio(lp_new, lp_old):
    """log alpha(x, x') = log pi(x') - log pi(x): the proposal density of eq. rw
    is symmetric in (x, x')."""
    return lp_new - lp_old


def whiten(A, x_ref, X):
    """A^-1 (x - x_ref) for each column, by a triangular solve against the
    lower factor A (the product Algorithm 1 applies to every state)."""
    return sla.solve_triangular(A, X - x_ref[:, None], lower=True, check_finite=False)


def log_accept_ratio(lp_new, lp_old, Z_new, Z_old, alpha=1.0):
    """log alpha(x, x') of eq. accept for the DIAM kernel, as in Algorithm 1:
    log pi(x') + |z'|^2/(2 alpha^2) - (log pi(x) + |z|^2/(2 alpha^2))."""
    q_new = np.sum(Z_new * Z_new, axis=0)
    q_old = np.sum(Z_old * Z_old, axis=0)
    return (lp_new + q_new / (2.0 * alpha * alpha)) - (lp_old + q_old / (2.0 * alpha * alpha))


def accept_decisions(la, u):
    """Accept iff log u < log alpha (strict); NaN log alpha rejects."""
    la = np.asarray(la, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        acc = np.log(u) < la
    return acc & ~np.isnan(la)


def local_moments(Xw_p):
    """Local first two moments of one chain over one window of n_lag states
    (eqs. mom2p / mom1p with m = M = 1): S^p = (1/n_lag) sum x x^T,
    m^p = (1/n_lag) sum x.  Xw_p is d x n_lag."""
    n = Xw_p.shape[1]
    return (Xw_p @ Xw_p.T) / n, Xw_p.sum(axis=1) / n


def merge_global(S_glob, m_glob, N, locals_, n_lag):
    """Merge the P chains' local moments into the global ones (eqs. mom2g /
    mom1g).  With N prior samples and P chains of n_lag new samples each,
    S <- (N S + n_lag sum_p S^p) / (N + P n_lag), which is the printed
    ((k-1)/k) S + (1/(kP)) sum_p S^p when N = (k-1) P n_lag."""
    P = len(locals_)
    n_new = P * n_lag
    S_sum = np.zeros_like(S_glob)
    m_sum = np.zeros_like(m_glob)
    for S_p, m_p in locals_:
        S_sum += S_p
        m_sum += m_p
    tot = N + n_new
    S = (N / tot) * S_glob + (n_lag / tot) * S_sum
    m = (N / tot) * m_glob + (n_lag / tot) * m_sum
    return S, m, tot


def local_global_moments(S_glob, m_glob, N, S_p, m_p, n_p):
    """Chain p's local update of the global moments (eqs. mom2pg / mom1pg):
    with N global samples and the chain's n_p = m n_lag samples of the current
    batch, S^{p,glob} = (N S^glob + n_p S^p) / (N + n_p) and likewise the
    mean; the printed weights k M P n_lag / ((k M P + m) n_lag) and
    m n_lag / ((k M P + m) n_lag) are the case N = k M P n_lag."""
    tot = N + n_p
    return (N / tot) * S_glob + (n_p / tot) * S_p, (N / tot) * m_glob + (n_p / tot) * m_p


def sample_covariance(S, m):
    """C = S - m m^T (eq. sampcov)."""
    return S - np.outer(m, m)


def cholesky_jitter(C, jitter0=1e-12, tries=13):
    """Lower Cholesky factor of C, with the diagonal-jitter retry rule.

    Returns (L, j) where j = -1 if C itself factored, j >= 0 the jitter level
    used, or (None, tries) if every try failed.  A try fails when LAPACK's
    potrf meets a non-positive or NaN pivot.
    """
    d = C.shape[0]

    def chol(M):
        try:
            L = np.linalg.cholesky(M)
        except np.linalg.LinAlgError:
            return None
        return L if np.all(np.isfinite(L)) else None

    L = chol(C)
    if L is not None:
        return L, -1
    tr = float(np.trace(C)) / d
    s = tr if (tr > 0.0 and math.isfinite(tr)) else 1.0
    for j in range(tries):
        L = chol(C + ((10.0 ** j) * jitter0 * s) * np.eye(d))
        if L is not None:
            return L, j
    return None, tries


PROPOSALS = ("diam", "am", "pcn", "rw")


@dataclass
class DiamOracle:
    """P chains of Algorithm 1 sharing one proposal factor (M = 1).

    ``logpi`` maps a d x n block to n log-densities.  States are d x P.

    ``proposal`` selects the family of Section 2.3 run through the same
    logistics: "diam" (eq. diamnl, factor and pivot adapted), "am" (eq. rw
    with the adapted factor, Section 2.3.3), "pcn" (eq. pcn: the DIAM formula
    with the factor and pivot fixed after initialisation or a warm start) and
    "rw" (eq. rw with a fixed factor).  Under the fixed families an update
    adapts beta only.
    """
    logpi: object
    d: int
    P: int
    n_lag: int
    beta: float
    alpha: float = 1.0
    jitter0: float = 1e-12
    jitter_tries: int = 13
    X: np.ndarray = None
    x_ref: np.ndarray = None
    A: np.ndarray = None
    S_glob: np.ndarray = None
    m_glob: np.ndarray = None
    N: float = 0.0
    lp: np.ndarray = None
    Z: np.ndarray = None
    window: list = field(default_factory=list)
    n_accepted: np.ndarray = None
    last_jitter: int = -1
    # step-size adaptation of Algorithm 1: None, or (acc_min, acc_max, factor, beta_max)
    adapt: tuple = None
    win_acc: int = 0
    win_steps: int = 0
    proposal: str = "diam"
    # concurrent-chain logistics of Section 2.4.1: M intervals of n_lag steps
    # per batch; between global merges every chain refactorises from its own
    # local update of the global moments (eqs. mom2pg, mom1pg, cov2pg)
    M: int = 1
    Ap: np.ndarray = None          # P x d x d per-chain factors (None: all chains use A)
    xrp: np.ndarray = None         # d x P per-chain pivots
    loc_S: np.ndarray = None       # P x d x d chain-local second moments of the batch (eq. mom2p)
    loc_m: np.ndarray = None       # d x P chain-local means (eq. mom1p)
    loc_n: float = 0.0             # samples per chain in the batch so far (m n_lag)
    m_int: int = 0                 # intervals merged in the current batch

    def __post_init__(self):
        if self.proposal not in PROPOSALS:
            raise ValueError(f"unknown proposal {self.proposal!r}")
        if self.M < 1 or (self.M > 1 and self.proposal != "diam"):
            raise ValueError("M >= 1; M > 1 runs the DIAM proposal")
        d, P = self.d, self.P
        self._reset_local()
        if self.X is None:
            self.X = np.zeros((d, P))
        self.X = np.array(self.X, dtype=np.float64, copy=True)
        self.x_ref = np.zeros(d)
        self.A = np.eye(d)
        self.S_glob = np.zeros((d, d))
        self.m_glob = np.zeros(d)
        self.N = 0.0
        self.lp = self.logpi(self.X)
        self.Z = whiten(self.A, self.x_ref, self.X)
        self.n_accepted = np.zeros(P, dtype=np.int64)

    # -- warm start: seed the global moments, then factorise once ----------
    def seed_moments(self, S0, m0, N0):
        """Replace the global moments, then refactorise (under every family:
        this is how a fixed family receives its prior factor and mean)."""
        self.S_glob = np.array(S0, dtype=np.float64, copy=True)
        self.m_glob = np.array(m0, dtype=np.float64, copy=True)
        self.N = float(N0)
        self._reset_local()
        self.adapt_beta()
        return self.refactor()

    def _reset_local(self):
        """Start a batch: clear the chain-local accumulators.  The per-chain
        factors stay until a global refactorisation succeeds (it recomputes
        every z under the shared pair)."""
        self.loc_S = np.zeros((self.P, self.d, self.d))
        self.loc_m = np.zeros((self.d, self.P))
        self.loc_n = 0.0
        self.m_int = 0

    @property
    def walk(self):
        return self.proposal in ("am", "rw")

    # -- one step of all P chains (Algorithm 1, loop body) -----------------
    def step(self, W, u):
        if self.walk:
            Xp = rw_proposal(self.X, self.A, W, self.beta, self.alpha)
            lpp = self.logpi(Xp)
            if np.any(np.isposinf(lpp)):
                raise FloatingPointError("log density returned +inf")
            la = symmetric_log_accept_ratio(lpp, self.lp)
            Zp = self.Z
        else:
            if self.Ap is None:
                Xp = diam_proposal(self.X, self.x_ref, self.A, W, self.beta, self.alpha)
                Zp = whiten(self.A, self.x_ref, Xp)
            else:                                   # every chain with its own factor and pivot
                Xp = np.empty_like(self.X)
                Zp = np.empty_like(self.Z)
                for p in range(self.P):
                    A, xr = self.Ap[p], self.xrp[:, p]
                    Xp[:, p:p + 1] = diam_proposal(self.X[:, p:p + 1], xr, A, W[:, p:p + 1], self.beta, self.alpha)
                    Zp[:, p:p + 1] = whiten(A, xr, Xp[:, p:p + 1])
            lpp = self.logpi(Xp)
            if np.any(np.isposinf(lpp)):
                raise FloatingPointError("log density returned +inf")
            la = log_accept_ratio(lpp, self.lp, Zp, self.Z, self.alpha)
        acc = accept_decisions(la, u)
        self.X[:, acc] = Xp[:, acc]
        self.Z[:, acc] = Zp[:, acc]
        self.lp[acc] = lpp[acc]
        self.n_accepted += acc
        self.win_acc += int(acc.sum())
        self.win_steps += 1
        self.window.append(self.X.copy())
        return acc, la

    # -- two-stage delayed acceptance with a surrogate ---------------------
    def step_delayed(self, W, u1, u2, surrogate, s_cur):
        """One step with a cheap first stage (Christen & Fox 2005).

        Stage 1 runs the DIAM acceptance with the surrogate log-density in
        place of log pi.  Survivors face stage 2 with
        log alpha_2 = (log pi(x') - log pi(x)) - (s(x') - s(x)),
        which makes the composite kernel reversible for pi itself.  Under the
        random-walk families stage 1 is the symmetric ratio of s.  Returns
        (accepted, stage-1 survivors, updated s_cur)."""
        if self.M > 1:
            raise ValueError("delayed acceptance runs with M = 1")
        if self.walk:
            Xp = rw_proposal(self.X, self.A, W, self.beta, self.alpha)
            Zp = self.Z
            sp = surrogate(Xp)
            la1 = symmetric_log_accept_ratio(sp, s_cur)
        else:
            Xp = diam_proposal(self.X, self.x_ref, self.A, W, self.beta, self.alpha)
            Zp = whiten(self.A, self.x_ref, Xp)
            sp = surrogate(Xp)
            la1 = log_accept_ratio(sp, s_cur, Zp, self.Z, self.alpha)
        pass1 = accept_decisions(la1, u1)
        acc = np.zeros(self.P, dtype=bool)
        if np.any(pass1):
            idx = np.nonzero(pass1)[0]
            lpp = self.logpi(Xp[:, idx])
            la2 = (lpp - self.lp[idx]) - (sp[idx] - s_cur[idx])
            ok = accept_decisions(la2, u2[idx])
            sel = idx[ok]
            acc[sel] = True
            self.lp[sel] = lpp[ok]
        self.X[:, acc] = Xp[:, acc]
        self.Z[:, acc] = Zp[:, acc]
        s_new = s_cur.copy()
        s_new[acc] = sp[acc]
        self.n_accepted += acc
        self.win_acc += int(acc.sum())
        self.win_steps += 1
        self.window.append(self.X.copy())
        return acc, pass1, s_new

    # -- every n_lag steps: merge, then refactorise -------------------------
    def merge_moments(self):
        if len(self.window) == 0:
            raise RuntimeError("empty window")
        n = len(self.window)
        Xw = np.stack(self.window, axis=2)            # d x P x n
        self.window = []
        if self.M == 1:
            locals_ = [local_moments(Xw[:, p, :]) for p in range(self.P)]
            self.S_glob, self.m_glob, self.N = merge_global(self.S_glob, self.m_glob, self.N, locals_, n)
            return
        # M > 1: fold the interval into the running chain-local moments (eqs.
        # mom2p / mom1p, sample-count weights); every M intervals merge them
        for p in range(self.P):
            S_w, m_w = local_moments(Xw[:, p, :])
            tot = self.loc_n + n
            self.loc_S[p] = (self.loc_n / tot) * self.loc_S[p] + (n / tot) * S_w
            self.loc_m[:, p] = (self.loc_n / tot) * self.loc_m[:, p] + (n / tot) * m_w
        self.loc_n += n
        self.m_int += 1
        if self.m_int == self.M:
            locals_ = [(self.loc_S[p], self.loc_m[:, p]) for p in range(self.P)]
            self.S_glob, self.m_glob, self.N = merge_global(self.S_glob, self.m_glob, self.N, locals_, self.loc_n)
            self._reset_local()

    def adapt_beta(self):
        """Algorithm 1's update block: the acceptance ratio of the steps since
        the last update, pooled over the chains, moves beta up by the factor
        (capped at beta_max) above the band and down by it below the band."""
        if self.adapt is not None and self.win_steps > 0:
            acc_min, acc_max, factor, beta_max = self.adapt
            rate = self.win_acc / (self.P * self.win_steps)
            if rate > acc_max:
                self.beta = min(self.beta * factor, beta_max)
            elif rate < acc_min:
                self.beta = self.beta / factor
        self.win_acc = 0
        self.win_steps = 0

    def update_proposal(self):
        self.adapt_beta()
        if self.proposal in ("pcn", "rw"):
            return OK
        if self.M > 1 and self.m_int > 0:
            return self.refactor_local()
        return self.refactor()

    def refactor_local(self):
        """Between global merges: chain p's factor A_p = chol(C^{p,glob}) and
        pivot m^{p,glob} (eqs. mom2pg, mom1pg, cov2pg), with the jitter rule
        per chain; a chain whose every try fails keeps its factor and pivot.
        Its z is recomputed under the new pair."""
        if self.Ap is None:
            self.Ap = np.repeat(self.A[None, :, :], self.P, axis=0)
            self.xrp = np.repeat(self.x_ref[:, None], self.P, axis=1)
        status, jmax = OK, -1
        for p in range(self.P):
            S_pg, m_pg = local_global_moments(self.S_glob, self.m_glob, self.N, self.loc_S[p], self.loc_m[:, p],
                                              self.loc_n)
            A, j = cholesky_jitter(sample_covariance(S_pg, m_pg), self.jitter0, self.jitter_tries)
            jmax = max(jmax, j)
            if A is None:
                status = E_NOT_PD
                continue
            self.Ap[p] = A
            self.xrp[:, p] = m_pg
            self.Z[:, p:p + 1] = whiten(A, m_pg, self.X[:, p:p + 1])
        self.last_jitter = jmax
        return status

    def refactor(self):
        C = sample_covariance(self.S_glob, self.m_glob)
        A, j = cholesky_jitter(C, self.jitter0, self.jitter_tries)
        self.last_jitter = j
        if A is None:
            return E_NOT_PD
        self.A = A
        self.x_ref = self.m_glob.copy()
        self.Z = whiten(self.A, self.x_ref, self.X)
        self.Ap = None
        self.xrp = None
        return OK

    def run_window(self, W, U):
        """n_lag steps with W[t] (P x d, i.e. d x P column-major) and U[t]
        (P), then the merge and the update.  Returns the acceptance count."""
        acc = np.zeros(self.P, dtype=np.int64)
        for t in range(W.shape[0]):
            a, _ = self.step(W[t].T, U[t])
            acc += a
        self.merge_moments()
        self.update_proposal()
        return acc
