"""Step-by-step comparison of the HIP sampler with the oracle, shared by the
GPU parity tests.

Both sides take the same normals W and uniforms U.  The bar (FP64) is the
oracle's accept decisions, step for step, and log alpha within the near-tie
threshold.  A near-tie (|log alpha - log u| below the threshold) is a step at
which two correct implementations may legitimately decide differently; there
the oracle is made to take the GPU's decision (its uniform is replaced by one
that forces it) and the comparison goes on, so every later step, merge and
update of the run is still compared.  The forcing is checked: at a forced
step the oracle's own log alpha must lie within the threshold of the GPU's,
i.e. the step really is a tie for both sides.
"""
import numpy as np

# log(2^-60) = -41.6 lies below every log alpha that is within a near-tie of
# log u for a uniform of (0, 1) drawn as (k + 0.5) 2^-52 (log u >= -36.7);
# log(inf) lies above every finite log alpha.
_FORCE_ACCEPT = 2.0 ** -60
_FORCE_REJECT = np.inf


def forced_uniforms(u, acc, near):
    """Uniforms with which the oracle takes the decisions `acc` where `near`."""
    u = np.array(u, dtype=np.float64, copy=True)
    u[near & acc] = _FORCE_ACCEPT
    u[near & ~acc] = _FORCE_REJECT
    return u


def oracle_follow(o, W, U, acc_g, la_g, tie, where="", stats=None):
    """Step the oracle `o` through n steps next to the GPU's results.

    W: n x P x d normals, U: n x P uniforms, acc_g: n x P GPU decisions,
    la_g: n x P GPU log alphas.  Away from near-ties (|la_g - log u| >= tie)
    the oracle's own decision must equal the GPU's; at a near-tie the oracle
    is forced to the GPU's decision.  Every log alpha must agree within `tie`
    (non-finite values must be non-finite on both sides).  `tie` is a number
    or a function of the oracle (called before each step) giving one
    threshold per chain.  Returns (accepted, forced) counts; `stats` (a
    dict) receives the largest |log alpha difference| / threshold seen."""
    n, P = U.shape
    accepted = forced = 0
    for t in range(n):
        lu = np.log(U[t])
        tv = tie(o) if callable(tie) else tie
        tie_t = np.broadcast_to(np.asarray(tv, dtype=np.float64), (P,))
        with np.errstate(invalid="ignore"):
            near = np.abs(la_g[t] - lu) < tie_t
        acc_o, la_o = o.step(W[t].T, forced_uniforms(U[t], acc_g[t], near))
        fin = np.isfinite(la_o)
        assert np.array_equal(fin, np.isfinite(la_g[t])), (where, t, np.nonzero(fin != np.isfinite(la_g[t])))
        err = np.abs(la_g[t][fin] - la_o[fin])
        assert np.all(err <= tie_t[fin]), (where, t, float(np.max(err / tie_t[fin])))
        if stats is not None and err.size:
            stats["max_ratio"] = max(stats.get("max_ratio", 0.0), float(np.max(err / tie_t[fin])))
        with np.errstate(invalid="ignore"):
            own = (lu < la_o) & ~np.isnan(la_o)
        far = ~near
        assert np.array_equal(own[far], acc_g[t][far]), (where, t, np.nonzero(own[far] != acc_g[t][far]))
        assert np.array_equal(acc_o, acc_g[t]), (where, t)
        accepted += int(acc_o.sum())
        forced += int(near.sum())
    return accepted, forced


def assert_few_forced(forced, decisions, where="", frac=0.01):
    """A run in which more than `frac` of the decisions (and more than 2) were
    forced compared too little to count."""
    assert forced <= max(2, int(frac * decisions)), (where, forced, decisions)
