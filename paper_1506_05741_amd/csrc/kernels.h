// Host-side launch wrappers for the DIAM kernels (all stream-ordered).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dk {

enum Prec { P64 = 0, P32 = 1, PMIX = 2 };

// Tile of the Gaussian target contraction (rows of R per partial sum).
constexpr int TGT_BM = 64;
// Rows of the state matrices handled by one step-kernel workgroup.
constexpr int STEP_RCH = 128;
// Cholesky / triangular-solve block size.
constexpr int CHOL_NB = 64;

inline int tgt_row_blocks(int d) { return (d + TGT_BM - 1) / TGT_BM; }
inline int step_chunks(int d) { return (d + STEP_RCH - 1) / STEP_RCH; }

// Target contractions write per-row-block partial sums of log-density
// contributions: log pi(x_p) = sum_rb part[p][rb] (+ the prior, for the
// logistic target, added by the step kernel).
// Gaussian: part[p][rb] = -1/2 sum over rows of block rb of (R (x_p - mu))_i^2.
// twist (optional, d FP64): the twisted Gaussians (Section 3.1): row 2k+1's
// y gains twist[2k+1] * y_{2k}^2 before it is squared.
hipError_t tgt_gauss(Prec prec, const void* R, const void* V, int d, int P, double* part, hipStream_t s,
                     const double* twist = nullptr);
// Mixed form, Gaussian: the same partials from two-part half splits of
// scaled R and V (FP32-equivalent products); needs tgt_h2_ok(d, P) and Yp
// scratch of tgt_h2_scratch_bytes.  h2_scales computes the coordinate scales
// vsc (d floats) from the states X (d x P) about mu and the lower factor L
// (d x d column-major FP64; states_only: from the states' spread alone, for
// evaluating the states themselves), then the row scales rsc (d FP64) and both parts
// of the scaled R (FP32 row-major) into R2 (2 d^2 halves, each part in
// 16 x 32 blocks ordered by column block, then row block); h2_split_v writes
// both parts of the scaled X - mu into V2 (2 d P halves).  The step kernel
// writes V2 itself (vh, vsc) after that.
bool tgt_h2_ok(int d, int P);
size_t tgt_h2_scratch_bytes(int d, int P);
hipError_t h2_scales(const double* X, const double* mu, const double* L, const float* R, int d, int P, float* vsc,
                     uint16_t* R2, double* rsc, hipStream_t s, int states_only = 0);
hipError_t h2_split_v(const double* X, const double* mu, const float* vsc, int d, int P, uint16_t* V2,
                      hipStream_t s);
// Products into the K-split partials Yp, then their reduction into part; with
// part = nullptr the products only (the reduction then runs in step_h2).
hipError_t tgt_gauss_h2(const uint16_t* R2, const uint16_t* V2, const double* rsc, int d, int P, float* Yp,
                        double* part, hipStream_t s, const double* twist = nullptr);
// Logistic: part[p][rb] = sum_{j in rb} y_j t_jp - softplus(t_jp), t = A x'
// (A n_obs x d row-major FP32, V d x P FP32); columns >= *nact skipped.
int logreg_row_blocks(long n_obs);
hipError_t tgt_logreg(const float* A, const float* y, long n_obs, const float* V, int d, int P, const int* nact,
                      double* part, hipStream_t s);

// Buffers of the MLP surrogate (all device, FP32 unless noted).
struct MlpBufs {
  int D, H, d_state;
  float *master, *eff, *grad, *m;        // nparam each (m holds Adam m then v: 2 nparam)
  float *in_mean, *in_scale, *stats;      // D, D, 2 (out mean, out std)
  float *Xs, *ts;                         // standardised training pairs (D x ntrain, ntrain)
  float *xb, *tb;                         // minibatch / evaluation input (D x nmax, nmax)
  float *a1, *h1, *a2, *h2, *ga1, *ga2;   // H x nmax
  float *out, *gout, *loss;               // nmax, nmax, 1
  int* bidx;                              // nmax (minibatch indices)
};
size_t mlp_nparam(int D, int H);
hipError_t mlp_prepare(const MlpBufs& b, const double* X, const double* lp, long n, uint64_t seed, hipStream_t s);
hipError_t mlp_train_step(const MlpBufs& b, long n, int nb, long tau, uint64_t seed, float lr, hipStream_t s);
hipError_t mlp_forward(const MlpBufs& b, const float* xs, int n, hipStream_t s);
// s_out[j] = surrogate log density of column j of X64 (FP64) or X32 (FP32), d x n
hipError_t mlp_eval(const MlpBufs& b, const double* X64, const float* X32, int n, double* s_out, hipStream_t s);
// Delayed acceptance stage 1 from the network's hidden layer h2 (filled by
// mlp_forward-equivalent GEMMs on V), survivor packing into Vs.
hipError_t da_screen(const MlpBufs& b, const float* V, int d, int P, int nch, const double* s_cur,
                     const double* zq_part, const double* zq, const double* u1, double inv2a2, int resid,
                     double* s_new, uint8_t* pass, int* slot, int* idx, int* nsurv, int* npass, float* Vs,
                     hipStream_t s);
// t = lp + c zq
hipError_t axpy_f64(const double* lp, const double* zq, double c, long n, double* t, hipStream_t s);

// Xi = c L W over ncols columns; L lower (d x d): f64/f32 column-major,
// bf16 as hi then lo row-major copies; W: f64/f32 column-major, bf16 as hi
// and lo arrays.
hipError_t trigemm(Prec prec, const void* L, const void* W, const void* Wlo, void* Xi, int d, long ncols, double c,
                   hipStream_t s);

// Scatter of the shifted window Xs (d x K): FP64 result G stored in the upper
// triangle (G(i,j), i >= j, at row j, column i), plus row sums h.
// f64/f32: column-major Xs (ld = d); bf16: row-major transposed window (ld = K).
size_t syrk_scratch_bytes(int prec, int d, long K);
// Xw: the window (col-major d x K); Xt: room for its row-major copy (bf16 only)
hipError_t syrk_window(Prec prec, const void* Xw, void* Xt, int d, long K, double* G, double* h, void* scratch,
                       hipStream_t s);

// Fold the window into the global moments (counts N -> N + K).
hipError_t fold_moments(const double* G, const double* h, const double* sft, double N, long K, double* S, double* m,
                        int d, hipStream_t s);
// Cov = S - m m^T + eps I into the lower triangle of C (upper zeroed); trace -> *tr.
hipError_t cov_assemble(const double* S, const double* m, double eps, double* C, double* tr, int d, hipStream_t s);
// In-place lower Cholesky; *info = 0 on success, else 1 + first failing column.
// Linv: chol_scratch_bytes(d) of scratch (inverses of the diagonal blocks).
size_t chol_scratch_bytes(int d);
hipError_t potrf(double* A, int d, int* info, double* Linv, hipStream_t s);
// Round the factor to the working precision in place and emit the low-precision
// copy (f32 column-major, or bf16 hi and lo row-major: L~ = hi + lo); no-op
// for P64.
hipError_t round_factor(Prec prec, double* L, void* Llow, int d, hipStream_t s);
// Z = L^-1 (X - xr) in place of Z (d x P); then zq[p] = ||z_p||^2.
hipError_t trsm_whiten(const double* L, const double* X, const double* xr, double* Z, double* zq, double* Linv, int d,
                       int P, hipStream_t s);

// Normals for steps [s0, s0 + n) of P chains; layout per step d x P column-major.
hipError_t normals(Prec prec, uint64_t seed, long s0, int n, int d, int P, void* W, void* Wlo, hipStream_t s);
// Uniforms for steps [s0, s0 + n), `stages` per step: U[t][g][p].
hipError_t uniforms(uint64_t seed, long s0, int n, int P, int stages, double* U, hipStream_t s);
// Caller FP64 normals -> working format (f32, or bf16 hi/lo).
hipError_t convert_normals(Prec prec, const double* W64, long count, void* W, void* Wlo, hipStream_t s);

struct StepArgs {
  int d, P, prec;
  double rho, c, inv2a2;                  // sqrt(1-beta^2), beta*alpha, 1/(2 alpha^2)
  const double* xr;                       // d
  const double* mu;                       // d (Gaussian target)
  double* X;                              // d x P
  double* Z;                              // d x P
  void* V;                                // d x P, f64 or f32 target input
  // accept half (t >= 0)
  int do_accept;
  const void* xi_cur;                     // d x P (f64 or f32)
  const void* w_cur; const void* wlo_cur; // d x P
  const double* lpp_part;                 // P x nrb (chain-major)
  int nrb;
  const double* zq_part_cur;              // P x nch (chain-major)
  const double* lp_cur; const double* zq_cur;
  double* lp_nxt; double* zq_nxt;
  const double* u;                        // P
  int* nacc;                              // P, accumulated
  double* la_out; uint8_t* acc_out;       // P each (this step)
  void* win; long win_col0;               // window store column offset (t_win * P)
  double* trace_lp;                       // P or null
  const double* proj; int nproj; double* proj_part;  // d x nproj; nch x nproj x P
  int* err;
  // propose half (next step)
  int do_propose;
  const void* xi_nxt;
  const void* w_nxt; const void* wlo_nxt;
  double* zq_part_nxt;                    // P x nch
  // target variants
  int v32;                                // write V as FP32 whatever the precision
  double prior_w;                         // > 0: add -prior_w |x|^2 to log pi (pq partials)
  const double* pq_part_cur;              // P x nch
  double* pq_part_nxt;                    // P x nch
  // delayed acceptance (second stage on stage-1 survivors)
  int da;
  const uint8_t* pass1;                   // P
  const int* slot;                        // P: survivor slot (column of lpp_part) or -1
  const double* s_new;                    // P: surrogate at the proposals
  const double* s_in; double* s_out;      // P: surrogate at the current states
  const double* u2;                       // P
  int da_resid;                           // residual surrogate r(x) - |z|^2/(2 alpha^2)
  int fuse_dec;                           // set by step(): the update kernel takes the decision itself
  uint16_t* vh;                           // non-null: write V as two half parts of (x - mu) vsc (d x P each) instead
  const float* vsc;                       // d: power-of-two coordinate scales for vh
  int ldv;                                // leading dimension of V (0: d)
  int ldw;                                // leading dimension of Xi and W (0: d)
  int32_t* wacc;                          // P: accepted proposals since the last update (optional)
};
hipError_t step(const StepArgs& a, hipStream_t s);
// One accepting step of the mixed form with the half target's reduction:
// the products of tgt_gauss_h2 (called with part = nullptr) in Yp, reduced,
// decided and applied in one launch (no delayed acceptance; d a multiple of
// 256 up to 4096).
bool step_h2_ok(int d, int P, int nrb);
hipError_t step_h2(const StepArgs& a, const float* Yp, const double* rsc, double* part, const double* twist,
                   hipStream_t s);
// PSRF accumulators (Section 2.4.2, M = 1): merge the nw stored states of
// each chain of the window (store shifted by xr, column p + P t) into the
// running per-chain means and sums of squared deviations (d x P each) that
// already hold n0 states per chain; finalize writes sqrt(R_i) for i < d.
hipError_t psrf_accumulate(Prec prec, const void* win, int d, int P, int nw, const double* xr, double n0, double* mean,
                           double* m2, hipStream_t s);
hipError_t psrf_finalize(const double* mean, const double* m2, int d, int P, double n, double* out, hipStream_t s);
// Stopping errors (Section 3.3): scratch[0] = |S - m m^T - Sigma|_F / |Sigma|_F,
// scratch[1] = |m - mu|_2 (0 when mu is null); scratch of moment_err_scratch_bytes():
// the two results, then 3 partial sums per workgroup of at most MERR_BLOCKS.
// Every partial is written before it is read: nothing must start at zero.
constexpr int MERR_BLOCKS = 1024;
constexpr size_t MERR_SCRATCH_DOUBLES = 2 + 3 * (size_t)MERR_BLOCKS;
size_t moment_err_scratch_bytes();
hipError_t moment_error(const double* S, const double* m, const double* Sigma, const double* mu, int d, double* scratch,
                        hipStream_t s);

// V = X - mu (mu may be null; FP64 or FP32 V), Z = X, for the initial evaluation.
hipError_t init_eval(int v64, const double* X, const double* mu, void* V, double* Z, int d, int P, hipStream_t s);
// lp[p] = sum_rb part[p][rb] - prior_w |x_p|^2; zq[p] = ||Z_p||^2.
hipError_t init_finish(const double* part, int nrb, const double* Z, const double* X, double prior_w, double* lp,
                       double* zq, int d, int P, hipStream_t s);
// trace[t][1 + k][p] = sum_ch proj_part[t][ch][k][p]
hipError_t proj_reduce(const double* proj_part, int n, int nch, int nproj, int P, double* trace, int nfun,
                       hipStream_t s);

// ---- batched form: G independent Gaussian problems, FP32 path ----------------
// Per-problem device buffers (FP64 state and moments, FP32 operands).
struct BProb {
  int d, nch, nrb, nb;              // dimension, step chunks, target row blocks, Cholesky blocks
  int ld;                           // d rounded up to a multiple of 4 (padded target operands)
  const float* R;                   // d x d row-major
  const float* Rp;                  // R zero-padded to ld x ld (16-byte rows for the target tiles)
  float* Vp;                        // ld x P, x' - mu with zero padding rows
  float* Lp;                        // FP32 factor zero-padded to ld x ld (column-major)
  const double* mu;                 // d
  double *X, *Z, *xr, *lp, *zq;     // d x P, d x P, d, 2 x P, 2 x P
  double *zq_part, *lpp_part, *la;  // 2 x P x nch, P x nrb, n x P
  uint8_t* acc;                     // n x P
  float *V, *W, *Xi, *win;          // d x P; W and Xi ld x P n; win d x P n
  double *S, *m, *L, *C, *Linv, *G, *h;
  float* Llow;                      // d x d
  int *nacc, *info;
};
struct BTile { int g, a, b; };      // problem, tile coordinates
struct BStep {
  int t, n, P;                      // step in the window (-1: first proposal only), n_lag, chains
  double rho, c, inv2a2;
  const double* U;                  // (g n + t) P + p
  int* err;
};
// The n_lag step loop of a window as one persistent launch: a fixed grid of
// workgroups takes items from a device queue in order; an item is one
// (problem, phase, tile) of one step.  Phases of a step of problem g, each
// needing all of the previous one: kind 0 target tiles (64-row tile a,
// 32-chain tile b), kind 1 the decisions of all P chains, kind 2 the update
// of 128-row chunk a for all P chains.  items[] lists one step (every step
// runs the same list); problem g's counter done[g] counts its finished items,
// and an item of step t waits until done[g] >= t * per_step[g] + need.
struct PItem { int kind, g, a, b, need; };
struct PCtl {
  int* qctr;            // next queue position (zero before the launch)
  int* done;            // G counters (zero before the launch)
  const int* per_step;  // G: items of problem g per step
  int* err;             // bit 1 (2) set when a wait gives up after spin_max polls
  int spin_max;
};
constexpr int PERSIST_THREADS = 512;
// Target tile rows the persistent loop uses (the default tile shape: 64 rows,
// two k-groups), so the decisions' partial sums fit one wavefront.
constexpr int PERSIST_TGT_CFG = 2;
// Problems whose update items take the chain's decision themselves (bitwise
// the decision item's sums), so the persistent loop needs no decision item.
__host__ __device__ inline bool persist_fused_decision(int d, int nrb, int nch) { return (d & 1) == 0 && nrb <= 64 && nch <= 64; }
hipError_t g_persist(const BProb* pr, const PItem* items, int nitems, const BStep& st, const PCtl& ctl, int grid,
                     hipStream_t s);
// Workgroups of the persistent loop that fit one CU at once.
int g_persist_blocks_per_cu();
constexpr int G_TGT_CONFIGS = 5;    // target tile shapes the autotuner chooses from
int g_tgt_bm(int cfg);
hipError_t g_tgt(int cfg, const BProb* pr, const BTile* tl, int ntiles, int P, hipStream_t s);
hipError_t g_step(const BProb* pr, const BTile* dec_tl, int ndec, const BTile* tl, int ntiles, const BStep& st,
                  hipStream_t s);
hipError_t g_trigemm(const BProb* pr, const BTile* tl, int ntiles, int ncols, double c, hipStream_t s);
hipError_t g_scatter(const BProb* pr, const BTile* syrk_tl, int nsyrk, const BTile* row_tl, int nrow, int K,
                     hipStream_t s);
hipError_t g_fold(const BProb* pr, const BTile* dd_tl, int ndd, const BTile* d_tl, int nd, const double* N, double K,
                  hipStream_t s);
hipError_t g_cov(const BProb* pr, const BTile* dd_tl, int ndd, hipStream_t s);
hipError_t g_chol_step(const BProb* pr, const BTile* diag, int ndiag, const BTile* panel, int npanel,
                       const BTile* upd, int nupd, int jb, hipStream_t s);
hipError_t g_adopt(const BProb* pr, const BTile* dd_tl, int ndd, hipStream_t s);
hipError_t g_sub_ref(const BProb* pr, const BTile* dp_tl, int ndp, int P, hipStream_t s);
hipError_t g_tri_inv(const BProb* pr, const BTile* tl, int n, hipStream_t s);
hipError_t g_trsm_step(const BProb* pr, const BTile* diag, int ndiag, const BTile* upd, int nupd, int jb, int P,
                       hipStream_t s);
hipError_t g_colnorm(const BProb* pr, const BTile* tl, int n, hipStream_t s);
hipError_t g_rng(uint64_t seed, const long* win, long nW, long nU, int P, float* W, double* U, hipStream_t s);
hipError_t g_bump(long* win, double* N, double K, hipStream_t s);

// ---- concurrent-chain logistics with M > 1 (local.hip), FP64 ------------------
// Xi[:, tP+p] = c L_p W[:, tP+p] + one_minus_rho (xrp[:, p] - xr), n steps
// (step-major columns); Lp: P lower d x d column-major factors.  P <= 65535.
hipError_t pc_gemm(const double* Lp, const double* W, const double* xrp, const double* xr, double* Xi, int d, int P,
                   int n, double c, double one_minus_rho, hipStream_t s);
// Gp[p] += sum_t y y^T, hp[:, p] += sum_t y over n stored steps (y = win column tP+p).
hipError_t pc_scatter(const double* win, double* Gp, double* hp, int d, int P, int n, hipStream_t s);
// Chain-local update of the global moments (S, m, N) with the chain's sums
// (G, h) of n samples shifted by sft: Spg, mpg.
hipError_t pc_moments(const double* S, const double* m, double N, const double* G, const double* h,
                      const double* sft, double n, double* Spg, double* mpg, int d, hipStream_t s);
// All chains at once: C_p (lower, zeros above) and m_pg into Cp (P x d x d) and
// mpgp (d x P), bitwise the one-chain pc_moments + cov_assemble.
hipError_t pc_cov(const double* S, const double* m, double N, const double* Gp, const double* hp, const double* sft,
                  double n, double* Cp, double* mpgp, int d, int P, hipStream_t s);
// Lp[p] = L, xrp[:, p] = xr for every chain.
hipError_t pc_bcast(const double* L, const double* xr, double* Lp, double* xrp, int d, int P, hipStream_t s);
// Lp[p] = Cp[p], xrp[:, p] = mpgp[:, p] for the chains with skip[p] == 0.
hipError_t pc_adopt(const double* Cp, const double* mpgp, const int* skip, double* Lp, double* xrp, int d, int P,
                    hipStream_t s);
// nprob independent potrf (problem z: A + z sA, Linv + z sL, info[z]; info
// zeroed by the caller) and whitenings (z_p = L_p^-1 (x_p - xr_p) and |z_p|^2
// for the chains with skip[p] == 0), bitwise the one-problem calls.
hipError_t potrf_batched(double* A, long sA, int d, int* info, double* Linv, long sL, int nprob, hipStream_t s);
hipError_t trsm_whiten_batched(const double* L, long sA, const double* X, const double* xrp, double* Z, double* zq,
                               double* Linv, long sL, int d, int P, const int* skip, hipStream_t s);
// G = sum_p Gp[p], h = sum_p hp[:, p].
hipError_t pc_sum(const double* Gp, const double* hp, double* G, double* h, int d, int P, hipStream_t s);

}  // namespace dk
