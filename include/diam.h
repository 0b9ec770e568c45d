/* diam.h - C ABI of libdiam: dimension-independent adaptive Metropolis (DIAM)
 * with P periodically synchronised chains on one AMD Instinct MI355X (gfx950).
 *
 * Method: Chen, Keyes, Law, Ltaief, "Accelerated dimension-independent
 * adaptive Metropolis", arXiv:1506.05741.  The library runs, for all P chains
 * at once, the loop of Algorithm 1 (Section 4.3) with the concurrent-chain
 * logistics of Section 2.4.1 taken with M = 1 (all chains merge their moments
 * every n_lag steps and share one proposal factor):
 *
 *   proposal      x' = x_ref + sqrt(1-beta^2) (x - x_ref) + beta alpha A W
 *                 (Section 2.3.4, eqs. diam and diamnl)
 *   acceptance    log alpha = log pi(x') + |z'|^2/(2 alpha^2)
 *                             - log pi(x) - |z|^2/(2 alpha^2),
 *                 z = A^-1 (x - x_ref)   (Section 2.2 eq. accept, in the form
 *                 Algorithm 1 prints, with the pivot x_ref restored)
 *   moments       running raw first and second moments of every visited
 *                 state (eqs. mom2p/mom1p/mom2g/mom1g), C = S - m m^T
 *                 (eq. sampcov)
 *   refactorise   A = chol(C) every n_lag steps, x_ref = m.
 *
 * Conventions
 *   - Every pointer argument is a DEVICE pointer unless marked "host".
 *   - Matrices are column-major with leading dimension d; chain p is
 *     column p of a d x P state matrix.  Exception: the Gaussian target's
 *     R is row-major (R[i*d + k]).
 *   - The caller owns every device buffer (workspace, x0, W, U, target
 *     arrays, trace); the library owns only the opaque context.  Buffers must
 *     outlive the context.  The library never allocates device memory.
 *   - All work is enqueued on the stream given to diam_init, in order.
 *     diam_update_proposal synchronises that stream (it reads the Cholesky
 *     status back); every other call is asynchronous.
 *   - Every call returns a diam_status; a negative value is an error and
 *     diam_last_error() (per host thread) describes it.  No call throws.
 *   - Precision: DIAM_FP64 runs every stage in FP64.  DIAM_FP32 runs the
 *     proposal contraction, the target contraction and the window scatter on
 *     FP32 MFMA.  DIAM_MIXED runs the proposal contraction and the scatter on
 *     BF16 MFMA with FP32 accumulation and the target contraction on FP32
 *     MFMA.  In every precision the chain states, z, log densities, the
 *     acceptance test, the moment accumulators and the Cholesky factorisation
 *     are FP64, and the factor and normals are rounded to the format the
 *     contraction consumes, with the acceptance using exactly those rounded
 *     values (the MH ratio stays exact for the kernel actually applied).
 *   - Determinism: with fixed inputs (or a fixed seed) results are bitwise
 *     reproducible run to run; no floating-point atomics are used.
 */
#ifndef DIAM_H
#define DIAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct diam_ctx diam_ctx; /* opaque */

typedef enum {
  DIAM_OK = 0,
  DIAM_E_ARG = -1,    /* invalid argument (null pointer, size, too-small workspace) */
  DIAM_E_STATE = -2,  /* call out of order (see each call) */
  DIAM_E_HIP = -3,    /* a HIP runtime call or kernel launch failed */
  DIAM_E_NOT_PD = -4, /* Cholesky failed at every jitter level; previous factor kept */
  DIAM_E_TARGET = -5  /* the target log density returned +inf, or (mixed form, Gaussian
                         target) a proposal left the half range of the scaled
                         operands: more than about 1000 spreads from the mean,
                         the spread taken at the last update */
} diam_status;

typedef enum { DIAM_FP64 = 0, DIAM_FP32 = 1, DIAM_MIXED = 2 } diam_precision;

typedef enum { DIAM_TGT_GAUSS = 0, DIAM_TGT_LOGREG = 1 } diam_target_kind;

/* Proposal family (Section 2.3).  W ~ N(0, I); A is the lower proposal factor
 * and x_ref the pivot held by the context.
 * DIAM_PROP_DIAM: eq. diamnl, x' = x_ref + rho (x - x_ref) + beta alpha A W with
 *   rho = sqrt(1 - beta^2); log alpha adds |z'|^2/(2 alpha^2) - |z|^2/(2 alpha^2),
 *   z = A^-1 (x - x_ref) (the reference Gaussian N(x_ref, alpha^2 A A^T) the
 *   proposal leaves invariant).  Each diam_update_proposal refactorises A from
 *   the merged covariance and moves x_ref to the merged mean.
 * DIAM_PROP_AM: adaptive Metropolis (Section 2.3.3): the random walk of eq. rw,
 *   x' = x + beta alpha A W, with A refactorised at every update as above.  The
 *   proposal is symmetric: log alpha = log pi(x') - log pi(x).
 * DIAM_PROP_PCN: preconditioned Crank-Nicolson (Section 2.3.2, eq. pcn): the
 *   DIAM formula with A and x_ref fixed, i.e. reversible for the prior
 *   N(x_ref, alpha^2 A A^T).  They start as A = I, x_ref = 0 (diam_init); a
 *   diam_seed_moments call sets them once from the moments it is given (a
 *   prior's covariance and mean).  diam_update_proposal adapts beta only.
 * DIAM_PROP_RW: random walk (Section 2.3.1, eq. rw), x' = x + beta alpha A W
 *   with A fixed as for pCN; symmetric acceptance as for AM.
 * Under AM and RW the context still carries z (advanced as z + beta alpha W)
 * so that fields keep their meaning; it does not enter log alpha. */
typedef enum { DIAM_PROP_DIAM = 0, DIAM_PROP_AM = 1, DIAM_PROP_PCN = 2, DIAM_PROP_RW = 3 } diam_proposal;

/* Sampler configuration (host struct, copied by diam_init). */
typedef struct {
  int32_t d;            /* dimension of the state, >= 1 */
  int32_t P;            /* number of concurrent chains, >= 1 */
  int32_t n_lag;        /* steps between proposal updates (Section 2.4.1) */
  int32_t precision;    /* diam_precision */
  double beta;          /* step size, 0 < beta <= 1 (eq. diam) */
  double alpha;         /* inflation factor, >= 1 (eq. diamnl); 1 for Gaussian targets */
  uint64_t seed;        /* Philox4x32-10 key for internally drawn W and U */
  double jitter0;       /* Cholesky retry: eps_j = 10^j jitter0 s, s = tr(C)/d (1 if not > 0) */
  int32_t jitter_tries; /* number of retry levels j = 0 .. jitter_tries-1 */
  int32_t surrogate;    /* learned part (MLP d-256-256-1, delayed acceptance): 0 none; 1 the
                           surrogate is the network; 2 residual form, the surrogate is
                           network(x) - |A^-1 (x - x_ref)|^2 / (2 alpha^2) (DIAM and pCN
                           proposals only, else DIAM_E_ARG) */
  int64_t train_max;    /* most (x, log pi(x)) pairs diam_surrogate_train will be given */
  int32_t proposal;     /* diam_proposal; 0 (DIAM) for a zero-initialised config */
  int32_t M;            /* intervals of n_lag steps per batch (Section 2.4.1); 0 or 1: every
                           merge is global and all chains share one factor.  M > 1: between
                           global merges (every M-th diam_merge_moments) each chain
                           proposes with its own factor and pivot from its local update of
                           the global moments (eqs. mom2pg, mom1pg, cov2pg).  M > 1 needs
                           DIAM_FP64, DIAM_PROP_DIAM, no surrogate and P <= 65535. */
} diam_config;

/* Target log density (Section 2.1: only the unnormalised density is needed).
 * DIAM_TGT_GAUSS: log pi(x) = -1/2 ||R (x - mu)||^2, R d x d row-major with
 * R^T R = Sigma^-1 (any square root of the precision); mu and R 16-byte
 * aligned (else DIAM_E_ARG).  R is FP64 for
 * DIAM_FP64 and FP32 otherwise; mu is FP64.  Evaluating it costs one dense
 * d x d by d x P contraction per step, the cost model of the paper's test
 * targets (Section 3.1).
 * DIAM_TGT_LOGREG: Bayesian logistic regression (eq. bayes with a Bernoulli
 * likelihood and a N(0, prior_var I) prior):
 *   log pi(w) = sum_j [ y_j t_j - softplus(t_j) ] - |w|^2 / (2 prior_var),
 *   t = A w, A n_obs x d row-major FP32, y in {0, 1} FP32.
 * The contraction runs on FP32 MFMA (the data are FP32) with the per-row
 * terms summed in FP64; the prior is FP64.
 * Twisted Gaussians (DIAM_TGT_GAUSS with twist non-NULL; Section 3.1's pi_5
 * and pi_6, pi_1 o V o phi o V^T with det(d phi) = 1): with y = R (x - mu),
 *   log pi(x) = -1/2 sum_i z_i^2,  z_{2k+1} = y_{2k+1} + twist[2k+1] y_{2k}^2,
 *   z_{2k} = y_{2k}  (0-based; twist at even rows is ignored).
 * For the paper's targets R = Sigma^-1/2 V^T (V, Sigma the eigendecomposition
 * of pi_1's covariance, smallest first), mu = 0 and twist[i] = b / (sqrt(d)
 * sigma_i) on the rows i = 1, 3, ..., d/10 - 1, zero elsewhere.  twist: d
 * FP64 on the device, 8-byte aligned; the batched form does not take it. */
typedef struct {
  int32_t kind;
  int32_t reserved;
  const double* mu;     /* Gaussian */
  const void* R;        /* Gaussian */
  const float* A;       /* logistic */
  const float* y;       /* logistic */
  int64_t n_obs;        /* logistic */
  double prior_var;     /* logistic */
  const double* twist;  /* Gaussian, optional: twisted Gaussian weights (d) */
} diam_target;

/* Fields readable with diam_get (device-to-device copy, asynchronous). */
typedef enum {
  DIAM_F_X = 0,       /* d x P f64  current states */
  DIAM_F_Z = 1,       /* d x P f64  A^-1 (x - x_ref) of the current states */
  DIAM_F_LOGP = 2,    /* P f64      log pi of the current states */
  DIAM_F_ZQ = 3,      /* P f64      |z|^2 of the current states */
  DIAM_F_XREF = 4,    /* d f64      pivot x_ref */
  DIAM_F_L = 5,       /* d x d f64  proposal factor A (lower; rounded to the
                                    contraction format in FP32/MIXED) */
  DIAM_F_S = 6,       /* d x d f64  global raw second moment S^glob */
  DIAM_F_M = 7,       /* d f64      global mean m^glob */
  DIAM_F_XI = 8,      /* d x P n f64/f32: beta alpha A W of the last
                                    diam_step_batch call (n = its n_steps) */
  DIAM_F_LA = 9,      /* n x P f64  log alpha of each step of the last call */
  DIAM_F_ACC = 10,    /* n x P u8   accept decision of each step of the last call */
  DIAM_F_NACC = 11,   /* P int32    accepted proposals since init (internal counter) */
  DIAM_F_W = 12,      /* d x P n    normals drawn by the last call when W was NULL:
                                    f64 (FP64), f32 (FP32), bf16 hi part (MIXED) */
  DIAM_F_WLO = 13,    /* d x P n    bf16 lo part of those normals (MIXED only) */
  DIAM_F_U = 14,      /* n x P (x2 under delayed acceptance) f64: uniforms drawn by
                                    the last call when U was NULL */
  DIAM_F_SURR = 15,   /* P f64      network output r at the current states (delayed acceptance on) */
  DIAM_F_NPASS = 16,  /* P int32    stage-1 survivors since delayed acceptance was enabled */
  DIAM_F_MLP_PARAMS = 17, /* nparam f32 master weights W1 (256 x d), b1, W2 (256 x 256), b2, W3 (256), b3 */
  DIAM_F_MLP_GRAD = 18,   /* nparam f32 gradient of the last training step */
  DIAM_F_MLP_BATCH = 19,  /* batch int32 training-pair indices of the last training step */
  DIAM_F_MLP_STATS = 20,  /* 2d + 2 f32: input mean, input 1/std, output mean, output std */
  DIAM_F_LP = 21,         /* P x d x d f64 per-chain factors (M > 1; chain p at p d^2,
                             column-major, lower; meaningful while per-chain factors are
                             in use, i.e. after a local update) */
  DIAM_F_XREFP = 22       /* d x P f64 per-chain pivots (M > 1, as DIAM_F_LP) */
} diam_field;

typedef struct {
  int64_t steps;          /* steps taken since init */
  int32_t steps_in_window;/* steps since the last merge */
  int32_t last_jitter;    /* -1: C factored as is; j >= 0: jitter level; tries: failed */
  double n_samples;       /* N: sample count of the global moments (incl. seeded N0) */
  int64_t windows;        /* merges since init */
  int64_t last_call_steps;/* n_steps of the last diam_step_batch */
  double beta;            /* current step size (changes under diam_set_beta_adaptation) */
} diam_stats;

/* Bytes of workspace diam_init needs for cfg (host).  Returns DIAM_E_ARG on a
 * bad configuration or target (the logistic target sizes its partial sums
 * by n_obs). */
int diam_workspace_bytes(const diam_config* cfg, const diam_target* tgt, size_t* bytes);

/* Create a sampler.  x0: d x P initial states (copied).  Initial proposal:
 * A = I, x_ref = 0 (Algorithm 1 initialisation, x_ref zero until the first
 * merge); global moments empty (N = 0).  workspace: >= diam_workspace_bytes,
 * 256-byte aligned.  hip_stream: a hipStream_t (NULL = default stream).
 * Evaluates log pi(x0) on the GPU before returning (asynchronously). */
int diam_init(diam_ctx** out, const diam_config* cfg, const diam_target* tgt, void* workspace, size_t ws_bytes,
              const double* x0, void* hip_stream);

/* Advance all P chains by n_steps steps of Algorithm 1.
 * Requires steps_in_window + n_steps <= n_lag (else DIAM_E_STATE).
 * W: d x P x n_steps f64 standard normals (step-major, each step a d x P
 *    column-major block), or NULL to draw them with Philox4x32-10 from the
 *    configured seed.  In FP32/MIXED they are rounded to FP32 (MIXED: split
 *    into bf16 hi + lo) and the acceptance uses the rounded values.
 * U: P x n_steps f64 uniforms in (0, 1) (step-major; 2P per step under
 *    delayed acceptance), or NULL for Philox.
 *    Accept iff log u < log alpha; a NaN log alpha rejects (Section 2.2).
 * W and U must be 16-byte aligned (else DIAM_E_ARG).
 * n_accepted: P int32 counters incremented per accepted proposal, or NULL.
 * The batch of search directions beta alpha A W for the n_steps steps is
 * formed in one contraction first, as Algorithm 1 does every n_lag steps. */
int diam_step_batch(diam_ctx* ctx, int32_t n_steps, const double* W, const double* U, int32_t* n_accepted);

/* Merge the states visited since the last merge (P chains x steps_in_window,
 * repeats after rejection included) into the global moments, eqs. mom2p,
 * mom1p, mom2g, mom1g with sample-count weights:
 *   S <- (N S + sum x x^T) / (N + K),  m <- (N m + sum x) / (N + K),  N += K.
 * Requires steps_in_window >= 1 (else DIAM_E_STATE).
 * M > 1: the window is folded into each chain's local sums instead (eqs.
 * mom2p, mom1p); every M-th call merges the P chains' local sums of the
 * batch into the global moments as above (eqs. mom2g, mom1g) and starts a
 * new batch. */
int diam_merge_moments(diam_ctx* ctx);

/* Refactorise: C = S - m m^T (eq. sampcov); A = chol(C) in FP64, retrying on
 * C + eps_j I (eps_j = 10^j jitter0 tr(C)/d) when a pivot is not positive;
 * then x_ref = m and z = A^-1 (x - x_ref) for every current state (FP64
 * triangular solve).  jitter_used (host, may be NULL): -1, the level j, or
 * jitter_tries when every try failed (then DIAM_E_NOT_PD, previous factor and
 * pivot kept).  Requires steps_in_window == 0.  Synchronises the stream.
 * Beta adaptation (diam_set_beta_adaptation) runs first.  Under the fixed
 * proposals (DIAM_PROP_PCN, DIAM_PROP_RW) only beta is adapted: A, x_ref and z
 * stay, and jitter_used gets -1.
 * M > 1, inside a batch (after a merge that was not global): every chain p
 * gets C_p = S^{p,glob} - m^{p,glob} m^{p,glob}^T from its local update of
 * the global moments, A_p = chol(C_p) with the jitter rule, x_ref_p =
 * m^{p,glob} and z_p = A_p^-1 (x_p - x_ref_p); a chain failing every level
 * keeps its pair (DIAM_E_NOT_PD is returned, the others are updated);
 * jitter_used gets the largest level used.  After a global merge the update
 * above runs and, on success, all chains share the new factor again.
 * Errors flagged by the steps since the last update come first, as
 * DIAM_E_TARGET (the update is then not made, the flag is cleared).  Mixed
 * form with a Gaussian target: the update also chooses the power-of-two
 * scales that bring x - mu and R into the half range of the target
 * contraction (coordinate k by 2^(6 - e_k), sigma_k < 2^e_k the larger of the
 * states' largest |x_k - mu_k| and the factor's row norm; each row of R to a
 * largest entry in [2^14, 2^15)). */
int diam_update_proposal(diam_ctx* ctx, int32_t* jitter_used);

/* Warm start: replace the global moments by (S0, m0) with pseudo-count N0
 * (device S0 d x d, m0 d), then diam_update_proposal.  Requires
 * steps_in_window == 0.  Under the fixed proposals this is the one call that
 * sets A = chol(S0 - m0 m0^T) and x_ref = m0 (with the jitter rule).  With
 * M > 1 it also starts a new batch (chain-local sums cleared). */
int diam_seed_moments(diam_ctx* ctx, const double* S0, const double* m0, double N0, int32_t* jitter_used);

/* Record per-step traces for effective-sample-size estimates: for each later
 * step t (counted from this call) trace[(t * (1 + n_proj) + f) * P + p] gets
 * f = 0: log pi of chain p's state after the step, f >= 1: proj[:, f-1]^T x.
 * proj: d x n_proj f64 (n_proj <= 4).  capacity: steps the trace can hold;
 * recording stops when full.  trace == NULL disables. proj and trace 16-byte aligned. */
int diam_set_trace(diam_ctx* ctx, const double* proj, int32_t n_proj, double* trace, int64_t capacity);

/* ---- learned-part form (requires cfg.surrogate = 1 or 2) -----------------
 * Network: r(x) = sd * (W3 h2 + b3) + mean, h2 = gelu(W2 h1 + b2),
 * h1 = gelu(W1 xs + b1), xs = (x - in_mean) / in_std, exact GELU a Phi(a);
 * hidden widths 256 and 256.  The forward pass uses the bf16 roundings of FP32
 * master weights with FP32 MFMA accumulation; training (FP32 MFMA forward and
 * backward, Adam) runs on the GPU.  Surrogate of log pi: s = r (form 1), or
 * s(x) = r(x) - |z(x)|^2 / (2 alpha^2), z = A^-1 (x - x_ref) under the current
 * factor (form 2: the network models what the proposal's Gaussian
 * N(x_ref, alpha^2 A A^T) leaves out; that Gaussian part of s cancels the
 * proposal correction in stage 1).
 *
 * Train on n pairs (X: d x n f64, lp: n f64 = log pi(X), n <= cfg.train_max):
 * regression target lp (form 1) or lp + |z|^2/(2 alpha^2) under the factor
 * current at the call (form 2); input and output standardisation from the
 * pairs, He-normal initialisation from seed, then `steps` Adam steps (lr,
 * beta1 0.9, beta2 0.999, eps 1e-8) on minibatches of `batch` <= max(P, 512)
 * pairs drawn with replacement by Philox; mean squared error on the
 * standardised target.  loss (host, may be NULL): the mean loss of the last
 * 50 steps.  Synchronises the stream.  DIAM_E_STATE while delayed acceptance
 * is on. */
int diam_surrogate_train(diam_ctx* ctx, const double* X, const double* lp, int64_t n, int32_t steps, int32_t batch,
                         double lr, uint64_t seed, double* loss);
/* Network output r of n states (X: d x n f64, n <= max(P, 512)) into out (n f64). */
int diam_surrogate_eval(diam_ctx* ctx, const double* X, int32_t n, double* out);
/* Two-stage delayed acceptance (Christen & Fox 2005) in later steps when
 * on != 0 (logistic target, trained network; else DIAM_E_STATE): stage 1
 * accepts with log u1 < s(x') - s(x) + (|z'|^2 - |z|^2)/(2 alpha^2), which is
 * r(x') - r(x) in form 2; only stage-1 survivors are evaluated exactly
 * (packed, so the target contraction shrinks with them) and accepted with
 * log u2 < (log pi(x') - log pi(x)) - (s(x') - s(x)), so pi stays invariant.
 * The network must stay fixed while it is on.  U per step then holds two
 * rows of P uniforms (stage 1, stage 2). */
int diam_set_delayed_acceptance(diam_ctx* ctx, int32_t on);

/* Step-size adaptation of Algorithm 1 (its update block): at every
 * diam_update_proposal the acceptance ratio of the steps since the previous
 * update, pooled over the P chains, moves beta to min(beta * factor,
 * beta_max) when it exceeds acc_max and to beta / factor when it is below
 * acc_min (the paper's band for DIAM is 0.3 .. 0.5, Section 3.2; it gives no
 * factor).  beta is constant within a window, so the proposal and the
 * z-recurrence of every step use one beta.  on = 0 keeps the current beta.
 * DIAM_E_ARG unless 0 <= acc_min < acc_max <= 1, factor > 1 and
 * 0 < beta_max <= 1.  The current beta is in diam_stats. */
int diam_set_beta_adaptation(diam_ctx* ctx, int32_t on, double acc_min, double acc_max, double factor, double beta_max);

/* ---- convergence diagnostic -------------------------------------------------
 * Potential scale reduction factor of the P chains (Section 2.4.2, eqs. winco,
 * btwco and psrf) with M = 1: chain p's local moments are the averages over
 * its n visited states since the diagnostic was enabled, the global mean is
 * the average of the chain means, and for every coordinate i
 *   B_i = n/(P-1) sum_p (m^p - m^glob)_i^2,  W_i = n/((n-1) P) sum_p C^p_ii,
 *   R_i = (n-1)/n + (P+1)/(P n) B_i / W_i,   diagnostic sqrt(R_i).
 * diam_psrf_enable(ctx, 1) zeroes the per-chain accumulators (d x P FP64
 * means and sums of squared deviations, in the workspace); every later
 * diam_merge_moments folds the window's stored states into them (the values
 * the moment merge uses: the shift from the window's pivot in FP64, FP32 or
 * bf16, plus the pivot, merged window by window in FP64 by the pairwise
 * update).  on = 0 stops folding and keeps the accumulators. */
int diam_psrf_enable(diam_ctx* ctx, int32_t on);
/* sqrt(R_i), i < d, into out (device, d f64; NULL: an internal buffer) and,
 * when worst (host) is non-NULL, max_i (sqrt(R_i) - 1) (NaN when some W_i is
 * 0, e.g. a coordinate that never moved), which synchronises the stream.
 * DIAM_E_STATE unless the diagnostic is enabled, P >= 2 and at least two
 * states per chain have been folded. */
int diam_psrf(diam_ctx* ctx, double* out, double* worst);
/* Stopping errors of the experiments (Section 3.3) against a known target:
 * cov_rel (host) = |S - m m^T - Sigma|_F / |Sigma|_F with the merged raw
 * second moment S and mean m (eq. sampcov), and mean_abs (host, may be NULL)
 * = |m - mu|_2 when mu is non-NULL, else NaN.  Sigma: device d x d f64
 * (symmetric, so either layout), mu: device d f64.  FP64 sums in a fixed
 * order; synchronises the stream. */
int diam_moment_error(diam_ctx* ctx, const double* Sigma, const double* mu, double* cov_rel, double* mean_abs);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * stopping errors for moments the caller holds, without a context or a
 * workspace.  S: d x d f64 raw second moment, m: d f64 mean (device; e.g.
 * read with diam_get or diam_batch_get), Sigma and mu as in
 * diam_moment_error; cov_rel and mean_abs (host) as there.  hip_stream: a
 * hipStream_t of the current device (NULL = default stream); synchronises
 * it.  The reduction partials live in a static device array of the library
 * (1024 partial triples and the two results, 24.6 KB per GPU, held until the
 * process ends): the grid is capped at 1024 workgroups, so every d >= 1 fits
 * (d < 1 is DIAM_E_ARG).  Every call on one GPU shares that array: calls that
 * overlap on one GPU (other host threads, other streams) race and must be
 * serialised by the caller.  Nothing in the array must start at zero: each
 * call writes every partial it reads.  Calls no allocating routine. */
int diam_moment_error_noalloc(const double* S, const double* m, int32_t d, const double* Sigma, const double* mu,
                              double* cov_rel, double* mean_abs, void* hip_stream);

/* ---- batched form ---------------------------------------------------------
 * G independent Gaussian problems of dimensions dims[g] (each target as in
 * diam_target, R FP32), P chains each, one shared n_lag.  Every call serves
 * all problems: each phase of a window is one grouped launch whose
 * workgroups are mapped to (problem, tile) by a tile list built at init, and
 * with graphs on (the default) the whole window, its n_lag-step loop
 * included, is captured once into a hipGraph and replayed.  Arithmetic is
 * FP32 on MFMA with FP64 states, moments, Cholesky and log-acceptance, the
 * same kernels as DIAM_FP32 of the single-problem calls: with the default
 * target tile shape and the same normals and uniforms, every problem's
 * states, moments and factor are bitwise those of a separate sampler.  Every
 * problem uses the DIAM proposal (DIAM_PROP_DIAM). */
typedef struct {
  int32_t G;            /* number of problems, 1 .. 4096 */
  int32_t P;            /* chains per problem */
  int32_t n_lag;        /* even; P * n_lag <= 4096 (one FP32 span of the scatter) */
  int32_t precision;    /* DIAM_FP32 */
  double beta, alpha;
  uint64_t seed;        /* Philox key of the normals and uniforms */
  double jitter0;
  int32_t jitter_tries;
  int32_t reserved;
} diam_batch_config;
typedef struct diam_batch diam_batch;

/* Workspace bytes for the problem set (host; dims: host array of G). */
int diam_batch_workspace_bytes(const diam_batch_config* cfg, const int32_t* dims, size_t* bytes);
/* Create the batch.  mu, R, x0: host arrays of G device pointers (mu[g]: d_g
 * f64, R[g]: d_g x d_g f32 row-major, x0[g]: d_g x P f64, copied).  Each
 * problem starts as diam_init does (A = I, x_ref = 0, log pi(x0)).  Returns
 * after the initial evaluation (synchronises the stream). */
int diam_batch_init(diam_batch** out, const diam_batch_config* cfg, const int32_t* dims, const double* const* mu,
                    const float* const* R, void* workspace, size_t ws_bytes, const double* const* x0,
                    void* hip_stream);
/* Warm start of every problem (S0[g], m0[g] device pointers, common N0), then
 * the refactorisation; jitter (host, G, may be NULL) as diam_update_proposal. */
int diam_batch_seed_moments(diam_batch* b, const double* const* S0, const double* const* m0, double N0,
                            int32_t* jitter);
/* One window of every problem: Philox normals and uniforms, the proposal
 * contraction, n_lag steps (target contraction + accept/reject), the moment
 * merge and the refactorisation (failed factorisations retried with the
 * jitter rule, per problem).  jitter: host array of G or NULL.  Returns
 * DIAM_E_NOT_PD if some problem failed at every level (it keeps its factor),
 * DIAM_E_TARGET on +inf from a target.  Synchronises the batch's stream. */
int diam_batch_window(diam_batch* b, int32_t* jitter);
/* Target tile shape (0 .. 4: rows x k-groups 32x2, 64x1, 64x2, 128x2, 32x4;
 * 32 chains per tile).  Default 2, the single-problem kernel's shape. */
int diam_batch_set_tiles(diam_batch* b, int32_t choice);
/* Time every target tile shape on this problem set (reps launches each) and
 * keep the fastest; choice (host, may be NULL) gets it, us (host array of 5,
 * may be NULL) the microseconds per launch of each. */
int diam_batch_autotune(diam_batch* b, int32_t reps, int32_t* choice, double* us);
/* Graph capture of the window on (default) or off (eager launches). */
int diam_batch_set_graph(diam_batch* b, int32_t on);
/* The n_lag-step loop of every window as one persistent launch (on != 0)
 * instead of three grouped launches per step (default off).  A fixed grid of
 * co-resident workgroups takes (problem, phase, tile) items of the loop from
 * a device queue in order; each problem advances through its own phases
 * (target tiles, decisions, update chunks) as soon as their inputs are
 * ready, without a device-wide barrier between steps.  Same kernels bodies
 * as the grouped launches with the default tile shape, so results are
 * bitwise those of the graph or eager windows (and of separate samplers).
 * Needs every d <= 4096 (else DIAM_E_ARG); sets the default target tile
 * shape, after which diam_batch_set_tiles and diam_batch_autotune return
 * DIAM_E_STATE.  Every wait inside the loop is bounded: a wait that gives up
 * makes the loop stop and diam_batch_window return DIAM_E_HIP (the window's
 * results are then invalid).  Works with and without graph capture. */
int diam_batch_set_persistent(diam_batch* b, int32_t on);
/* Per-problem fields at a window boundary: DIAM_F_X, Z, LOGP, ZQ, XREF, L, S,
 * M, LA, ACC (last window, n_lag x P), NACC, W (last window's normals, ld x
 * P n_lag f32 with ld = d rounded up to a multiple of 4; rows >= d unused),
 * U (last window's uniforms, n_lag x P f64). */
int diam_batch_field_bytes(diam_batch* b, int32_t g, int32_t field, size_t* bytes);
int diam_batch_get(diam_batch* b, int32_t g, int32_t field, void* dst, size_t bytes);
/* steps, windows and n_samples of the batch (the other members are not used). */
int diam_batch_get_stats(diam_batch* b, diam_stats* out);
void diam_batch_destroy(diam_batch* b);

/* Bytes of a field (host). */
int diam_field_bytes(diam_ctx* ctx, int32_t field, size_t* bytes);
/* Copy a field into dst (device); bytes must equal diam_field_bytes. */
int diam_get(diam_ctx* ctx, int32_t field, void* dst, size_t bytes);
/* Counters (host struct); does not synchronise. */
int diam_get_stats(diam_ctx* ctx, diam_stats* out);

/* Per-stage timing with HIP events recorded on the sampler's stream around
 * each kernel group (the events are collected at the synchronisation inside
 * diam_update_proposal and in diam_profile_read).  Stages: */
enum {
  DIAM_ST_RNG = 0,      /* Philox normals / uniforms, conversion of caller normals */
  DIAM_ST_PROPOSAL = 1, /* batched beta alpha A W contraction */
  DIAM_ST_TARGET = 2,   /* target log-density contraction (one event pair per step) */
  DIAM_ST_STEP = 3,     /* accept / reject + next proposal (one event pair per step) */
  DIAM_ST_MERGE = 4,    /* window transpose, scatter (SYRK), row sums, fold */
  DIAM_ST_CHOL = 5,     /* covariance assembly + blocked Cholesky (every try) */
  DIAM_ST_WHITEN = 6,   /* factor rounding, pivot copy, z = A^-1 (x - x_ref) */
  DIAM_ST_SURROGATE = 7, /* surrogate forward pass + stage-1 screen and survivor packing (per step) */
  DIAM_ST_TRAIN = 8,    /* surrogate standardisation, initialisation and Adam steps */
  DIAM_ST_PSRF = 9,     /* folding a merged window into the PSRF accumulators */
  DIAM_NSTAGES = 10
};
/* Enable (on != 0) or disable event timing.  Enabling creates the events. */
int diam_profile_enable(diam_ctx* ctx, int32_t on);
/* Synchronise the stream, then copy per-stage totals (host arrays of
 * DIAM_NSTAGES): milliseconds and number of timed regions.  reset != 0 zeroes
 * the totals afterwards. */
int diam_profile_read(diam_ctx* ctx, double* ms, int64_t* count, int32_t reset);

/* Message for the last non-OK status on this host thread. */
const char* diam_last_error(void);

/* Release the context (does not free caller buffers). */
void diam_destroy(diam_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* DIAM_H */
