// Host runtime of libdiam: workspace layout, call-order state machine and the
// orchestration of the kernels per call of the C ABI (include/diam.h).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "../../include/diam.h"
#include "kernels.h"

using dk::Prec;

static thread_local char g_err[512] = "";

// shared with the batched runtime (batch.hip)
int diam_fail_v(int code, const char* fmt, va_list ap) {
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  return code;
}

static int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  diam_fail_v(code, fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess) return fail(DIAM_E_HIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

namespace {

struct Status {  // device-side status words, read back by update_proposal
  int info;
  int err;
  double trace;
};

struct Layout {
  size_t X, Z, V, lp, zq, lpp_part, zq_part, pq_part, nacc, wacc, la, acc, U, W, Wlo, Xi, win, wint, xr, S, m, L, Lnew, Llow,
      h, syrk, status, proj_part, linv;
  // learned-part form
  size_t mlp_master, mlp_eff, mlp_grad, mlp_m, mlp_in_mean, mlp_in_scale, mlp_stats, mlp_Xs, mlp_ts, mlp_xb, mlp_tb,
      mlp_a1, mlp_h1, mlp_a2, mlp_h2, mlp_ga1, mlp_ga2, mlp_out, mlp_gout, mlp_loss, mlp_bidx, s_cur, s_new, pass1,
      slot, idx, nsurv, npass, Vs, t64, Zs;
  // two-part half target (mixed form, Gaussian)
  size_t R2, V2, vsc, rsc, Yp;
  // PSRF accumulators
  size_t pmean, pm2, pout, merr;
  // per-chain factors and local sums (M > 1)
  size_t Lp, Gp, hp, xrp, Spg, mpg, Cp, mpgp, pinfo, linvb;
  size_t total;
};

constexpr int MLP_H = 256;      // hidden widths of the surrogate
constexpr int MLP_NMIN = 512;   // activation buffers hold max(P, MLP_NMIN) samples
constexpr int LOSS_HIST = 64;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int elem_bytes_ctr(int prec) { return prec == DIAM_FP64 ? 8 : 4; }

int target_row_blocks(const diam_config& c, const diam_target& t) {
  return t.kind == DIAM_TGT_LOGREG ? dk::logreg_row_blocks(t.n_obs) : dk::tgt_row_blocks(c.d);
}

bool use_h2(const diam_config& c, const diam_target& t) {
  return c.precision == DIAM_MIXED && t.kind == DIAM_TGT_GAUSS && dk::tgt_h2_ok(c.d, c.P);
}

Layout make_layout(const diam_config& c, const diam_target& tg) {
  const size_t d = c.d, P = c.P, nl = c.n_lag;
  const size_t dP = d * P, dd = d * d, win = d * P * nl;
  const int nrb = target_row_blocks(c, tg), nch = dk::step_chunks(c.d);
  const int eb = elem_bytes_ctr(c.precision);
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += align256(bytes ? bytes : 1);
    return r;
  };
  L.X = take(dP * 8);
  L.Z = take(dP * 8);
  L.V = take(dP * 8);
  L.lp = take(2 * P * 8);
  L.zq = take(2 * P * 8);
  L.lpp_part = take((size_t)nrb * P * 8);
  L.zq_part = take(2 * (size_t)nch * P * 8);
  L.pq_part = take(2 * (size_t)nch * P * 8);
  L.nacc = take(P * 4);
  L.wacc = take(P * 4);
  L.la = take(nl * P * 8);
  L.acc = take(nl * P);
  L.U = take(2 * nl * P * 8);
  L.W = take(win * (c.precision == DIAM_MIXED ? 2 : eb));
  L.Wlo = take(c.precision == DIAM_MIXED ? win * 2 : 0);
  L.Xi = take(win * eb);
  L.win = take(win * (c.precision == DIAM_MIXED ? 2 : eb));
  L.wint = take(c.precision == DIAM_MIXED ? win * 2 : 0);
  L.xr = take(d * 8);
  L.S = take(dd * 8);
  L.m = take(d * 8);
  L.L = take(dd * 8);
  L.Lnew = take(dd * 8);
  L.Llow = take(c.precision == DIAM_FP64 ? 0 : dd * 4);  // f32, or bf16 hi + lo
  L.h = take(d * 8);
  L.syrk = take(dk::syrk_scratch_bytes(c.precision, c.d, (long)P * nl));
  L.status = take(sizeof(Status));
  L.proj_part = take(nl * (size_t)nch * 4 * P * 8);
  L.linv = take(dk::chol_scratch_bytes(c.d));
  const bool h2 = use_h2(c, tg);
  L.R2 = take(h2 ? 2 * dd * 2 : 0);
  L.V2 = take(h2 ? 2 * dP * 2 : 0);
  L.vsc = take(h2 ? d * 4 : 0);
  L.rsc = take(h2 ? d * 8 : 0);
  L.Yp = take(h2 ? dk::tgt_h2_scratch_bytes(c.d, c.P) : 0);
  L.pmean = take(dP * 8);
  L.pm2 = take(dP * 8);
  L.pout = take(d * 8);
  L.merr = take(dk::moment_err_scratch_bytes());
  const bool lg = c.M > 1;
  L.Lp = take(lg ? P * dd * 8 : 0);
  L.Gp = take(lg ? P * dd * 8 : 0);
  L.hp = take(lg ? dP * 8 : 0);
  L.xrp = take(lg ? dP * 8 : 0);
  L.Spg = take(lg ? dd * 8 : 0);
  L.mpg = take(lg ? d * 8 : 0);
  L.Cp = take(lg ? P * dd * 8 : 0);
  L.mpgp = take(lg ? dP * 8 : 0);
  L.pinfo = take(lg ? P * 4 : 0);
  L.linvb = take(lg ? P * dk::chol_scratch_bytes(c.d) : 0);
  if (c.surrogate) {
    const size_t np = dk::mlp_nparam(c.d, MLP_H), H = MLP_H;
    const size_t nmax = P > (size_t)MLP_NMIN ? P : (size_t)MLP_NMIN, nt = (size_t)c.train_max;
    L.mlp_master = take(np * 4);
    L.mlp_eff = take(np * 4);
    L.mlp_grad = take(np * 4);
    L.mlp_m = take(2 * np * 4);
    // input mean, input 1/std, output mean and std in one block (one field)
    L.mlp_in_mean = take((2 * d + 2) * 4);
    L.mlp_in_scale = L.mlp_in_mean + d * 4;
    L.mlp_stats = L.mlp_in_mean + 2 * d * 4;
    L.mlp_Xs = take(d * nt * 4);
    L.mlp_ts = take(nt * 4);
    L.mlp_xb = take(d * nmax * 4);
    L.mlp_tb = take(nmax * 4);
    L.mlp_a1 = take(H * nmax * 4);
    L.mlp_h1 = take(H * nmax * 4);
    L.mlp_a2 = take(H * nmax * 4);
    L.mlp_h2 = take(H * nmax * 4);
    L.mlp_ga1 = take(H * nmax * 4);
    L.mlp_ga2 = take(H * nmax * 4);
    L.mlp_out = take(nmax * 4);
    L.mlp_gout = take(nmax * 4);
    L.mlp_loss = take(LOSS_HIST * 4);
    L.mlp_bidx = take(nmax * 4);
    L.s_cur = take(2 * P * 8);
    L.s_new = take(P * 8);
    L.pass1 = take(P);
    L.slot = take(P * 4);
    L.idx = take(P * 4);
    L.nsurv = take(4);
    L.npass = take(P * 4);
    L.Vs = take(dP * 4);
    L.t64 = take(c.surrogate == 2 ? nt * 8 : 0);
    L.Zs = take(c.surrogate == 2 ? d * nmax * 8 : 0);
  }
  L.total = o;
  return L;
}

}  // namespace

struct diam_ctx {
  diam_config cfg;
  diam_target tgt;
  Prec prec;
  hipStream_t stream;
  char* ws;
  Layout lay;
  // device pointers
  double *X, *Z, *lp, *zq, *lpp_part, *zq_part, *pq_part, *la, *U, *xr, *S, *m, *L, *Lnew, *h, *proj_part, *linv;
  // target
  int logreg;
  int h2;          // two-part half target contraction
  uint16_t *R2, *V2;
  float* vsc;
  double* rsc;
  float* Yp;
  double prior_w;
  // PSRF
  double *pmean, *pm2, *pout, *merr;
  // local-global logistics (M > 1): per-chain pairs, chain-local sums of the batch
  double *Lp, *Gp, *hp, *xrp, *Spg, *mpg, *Cp, *mpgp, *linvb;
  int32_t* pinfo;  // per-chain factorisation status (0: factored)
  int m_int;      // intervals merged in the current batch
  double loc_n;   // samples per chain in the current batch
  int pc_on;      // chains propose with their own pairs
  int psrf_on;
  double psrf_n;  // states per chain folded since enabling
  // learned-part form
  dk::MlpBufs mlp;
  double *s_cur, *s_new;
  uint8_t* pass1;
  int *slot, *idx, *nsurv, *npass;
  float* Vs;
  double *t64, *Zs;
  int trained, da_on;
  int32_t last_batch;
  void *V, *W, *Wlo, *Xi, *win, *wint, *Llow, *syrk;
  int32_t* nacc;
  int32_t* wacc;  // accepted proposals per chain since the last update (step-size adaptation)
  uint8_t* acc;
  Status* status;
  int nrb, nch;
  int cur;  // parity of the double-buffered per-chain scalars
  // host state
  int64_t steps;
  int32_t siw;
  int32_t last_jitter;
  double N;
  int64_t windows;
  int64_t last_call_steps;
  int64_t win_steps;  // steps since the last update
  // step-size adaptation (Algorithm 1): band, factor, cap
  int adapt_on;
  double acc_min, acc_max, adapt_factor, beta_max;
  int last_call_stages;
  int last_call_caller_w;   // last call's Xi is at Xi offset 0
  // event timing
  bool prof_on;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_tag;
  int ev_used;
  double prof_ms[DIAM_NSTAGES];
  int64_t prof_cnt[DIAM_NSTAGES];
  // trace
  const double* proj;
  int nproj;
  double* trace;
  int64_t trace_cap, trace_pos;
};

static int check_cfg(const diam_config* c) {
  if (!c) return fail(DIAM_E_ARG, "null config");
  if (c->d < 1 || c->P < 1 || c->n_lag < 1) return fail(DIAM_E_ARG, "d, P and n_lag must be >= 1");
  if (c->precision < DIAM_FP64 || c->precision > DIAM_MIXED) return fail(DIAM_E_ARG, "unknown precision %d", c->precision);
  if (!(c->beta > 0.0 && c->beta <= 1.0)) return fail(DIAM_E_ARG, "beta must lie in (0, 1]");
  if (!(c->alpha >= 1.0)) return fail(DIAM_E_ARG, "alpha must be >= 1");
  if (!(c->jitter0 > 0.0) || c->jitter_tries < 0 || c->jitter_tries > 300)
    return fail(DIAM_E_ARG, "jitter0 must be > 0 and 0 <= jitter_tries <= 300");
  // 32-bit tile indices: the window holds P * n_lag columns of d rows
  if ((long)c->P * c->n_lag > (1L << 30) || c->d > (1 << 20)) return fail(DIAM_E_ARG, "problem too large");
  if ((long)c->d * c->d > (1L << 34)) return fail(DIAM_E_ARG, "d too large");
  if (c->surrogate < 0 || c->surrogate > 2) return fail(DIAM_E_ARG, "surrogate must be 0, 1 or 2");
  if (c->train_max < 0 || c->train_max > (1L << 31)) return fail(DIAM_E_ARG, "train_max out of range");
  if (c->proposal < DIAM_PROP_DIAM || c->proposal > DIAM_PROP_RW) return fail(DIAM_E_ARG, "unknown proposal %d", c->proposal);
  if (c->M < 0) return fail(DIAM_E_ARG, "M must be >= 0");
  if (c->M > 1 && (c->precision != DIAM_FP64 || c->proposal != DIAM_PROP_DIAM || c->surrogate || c->P > 65535))
    return fail(DIAM_E_ARG, "M > 1 needs DIAM_FP64, the DIAM proposal, no surrogate and P <= 65535");
  // the residual surrogate subtracts the reference Gaussian that only DIAM and pCN carry
  if (c->surrogate == 2 && (c->proposal == DIAM_PROP_AM || c->proposal == DIAM_PROP_RW))
    return fail(DIAM_E_ARG, "the residual surrogate needs the DIAM or pCN proposal");
  return DIAM_OK;
}

// random-walk family (eq. rw): no contraction toward the pivot, symmetric acceptance
static bool walk_proposal(const diam_config& c) { return c.proposal == DIAM_PROP_AM || c.proposal == DIAM_PROP_RW; }
// factor and pivot fixed after initialisation or a warm start
static bool fixed_factor(const diam_config& c) { return c.proposal == DIAM_PROP_PCN || c.proposal == DIAM_PROP_RW; }

static int check_target(const diam_config* c, const diam_target* t) {
  if (!t) return fail(DIAM_E_ARG, "null target");
  if (t->kind == DIAM_TGT_GAUSS) {
    if (!t->mu || !t->R) return fail(DIAM_E_ARG, "Gaussian target needs mu and R");
    if ((uintptr_t)t->mu % 16 || (uintptr_t)t->R % 16) return fail(DIAM_E_ARG, "mu and R must be 16-byte aligned");
    if ((uintptr_t)t->twist % 8) return fail(DIAM_E_ARG, "twist must be 8-byte aligned");
  } else if (t->kind == DIAM_TGT_LOGREG) {
    if (t->twist) return fail(DIAM_E_ARG, "twist applies to the Gaussian target only");
    if (!t->A || !t->y || t->n_obs < 1 || t->n_obs > (1L << 30)) return fail(DIAM_E_ARG, "logistic target needs A, y, n_obs >= 1");
    if (!(t->prior_var > 0.0)) return fail(DIAM_E_ARG, "prior_var must be > 0");
  } else {
    return fail(DIAM_E_ARG, "unknown target kind %d", t->kind);
  }
  return DIAM_OK;
}

extern "C" int diam_workspace_bytes(const diam_config* cfg, const diam_target* tgt, size_t* bytes) {
  int r = check_cfg(cfg);
  if (r) return r;
  r = check_target(cfg, tgt);
  if (r) return r;
  if (!bytes) return fail(DIAM_E_ARG, "null bytes");
  *bytes = make_layout(*cfg, *tgt).total;
  return DIAM_OK;
}

static double* dptr(diam_ctx* c, size_t off) { return (double*)(c->ws + off); }

__global__ void k_identity(double* L, int d) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < (long)d * d) L[e] = ((e % d) == (e / d)) ? 1.0 : 0.0;
}
__global__ void k_fill(double* p, long n, double v) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = v;
}
__global__ void k_fill_i32(int32_t* p, long n) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = 0;
}

// Clears the Cholesky words; the target error word only when clear_err.
__global__ void k_clear_status(Status* s, int clear_err) {
  if (threadIdx.x == 0) {
    s->info = 0;
    s->trace = 0.0;
    if (clear_err) s->err = 0;
  }
}

static unsigned nblk(long n) { return (unsigned)((n + 255) / 256); }

// start a batch of the local-global logistics: chain-local sums cleared
static void reset_local(diam_ctx* c) {
  const long dd = (long)c->cfg.d * c->cfg.d, dP = (long)c->cfg.d * c->cfg.P;
  hipLaunchKernelGGL(k_fill, dim3(nblk(dd * c->cfg.P)), dim3(256), 0, c->stream, c->Gp, dd * c->cfg.P, 0.0);
  hipLaunchKernelGGL(k_fill, dim3(nblk(dP)), dim3(256), 0, c->stream, c->hp, dP, 0.0);
  c->m_int = 0;
  c->loc_n = 0.0;
}

static int prof_flush(diam_ctx* c) {
  if (c->ev_used == 0) return DIAM_OK;
  HIPCHK(hipEventSynchronize(c->ev[c->ev_used - 1]));
  for (int i = 0; i + 1 < c->ev_used; i += 2) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
    c->prof_ms[c->ev_tag[i]] += ms;
    c->prof_cnt[c->ev_tag[i]] += 1;
  }
  c->ev_used = 0;
  return DIAM_OK;
}

// Open a timed region; returns the event slot or -1 when timing is off.
static int prof_begin(diam_ctx* c, int stage) {
  if (!c->prof_on) return -1;
  if (c->ev_used + 2 > (int)c->ev.size() && prof_flush(c) != DIAM_OK) return -1;
  const int i = c->ev_used;
  if (hipEventRecord(c->ev[i], c->stream) != hipSuccess) return -1;
  c->ev_tag[i] = stage;
  c->ev_used += 2;
  return i;
}
static void prof_end(diam_ctx* c, int slot) {
  if (slot >= 0) (void)hipEventRecord(c->ev[slot + 1], c->stream);
}

static void prof_release(diam_ctx* c) {
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  c->ev_tag.clear();
  c->ev_used = 0;
  c->prof_on = false;
}

extern "C" int diam_profile_enable(diam_ctx* c, int32_t on) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (on && !c->prof_on) {
    const int n = 2 * (c->cfg.n_lag * 3 + 64);
    c->ev.resize(n);
    c->ev_tag.assign(n, 0);
    for (int i = 0; i < n; ++i) {
      hipError_t e = hipEventCreate(&c->ev[i]);
      if (e != hipSuccess) {
        c->ev.resize(i);
        prof_release(c);
        return fail(DIAM_E_HIP, "hipEventCreate: %s", hipGetErrorString(e));
      }
    }
    c->ev_used = 0;
    c->prof_on = true;
  } else if (!on && c->prof_on) {
    int r = prof_flush(c);
    prof_release(c);
    return r;
  }
  return DIAM_OK;
}

extern "C" int diam_profile_read(diam_ctx* c, double* ms, int64_t* count, int32_t reset) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  int r = prof_flush(c);
  if (r) return r;
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int k = 0; k < DIAM_NSTAGES; ++k) {
    if (ms) ms[k] = c->prof_ms[k];
    if (count) count[k] = c->prof_cnt[k];
    if (reset) {
      c->prof_ms[k] = 0.0;
      c->prof_cnt[k] = 0;
    }
  }
  return DIAM_OK;
}

extern "C" int diam_init(diam_ctx** out, const diam_config* cfg, const diam_target* tgt, void* workspace,
                         size_t ws_bytes, const double* x0, void* hip_stream) {
  if (!out) return fail(DIAM_E_ARG, "null out");
  *out = nullptr;
  int r = check_cfg(cfg);
  if (r) return r;
  r = check_target(cfg, tgt);
  if (r) return r;
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(DIAM_E_ARG, "workspace null or not 256-byte aligned");
  if (!x0) return fail(DIAM_E_ARG, "null x0");
  Layout lay = make_layout(*cfg, *tgt);
  if (ws_bytes < lay.total) return fail(DIAM_E_ARG, "workspace too small: %zu < %zu", ws_bytes, lay.total);
  diam_ctx* c = new (std::nothrow) diam_ctx();
  if (!c) return fail(DIAM_E_ARG, "host allocation failed");
  c->cfg = *cfg;
  c->tgt = *tgt;
  c->prec = (Prec)cfg->precision;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  c->lay = lay;
  c->X = dptr(c, lay.X);
  c->Z = dptr(c, lay.Z);
  c->V = c->ws + lay.V;
  c->lp = dptr(c, lay.lp);
  c->zq = dptr(c, lay.zq);
  c->lpp_part = dptr(c, lay.lpp_part);
  c->zq_part = dptr(c, lay.zq_part);
  c->pq_part = dptr(c, lay.pq_part);
  c->logreg = tgt->kind == DIAM_TGT_LOGREG;
  c->h2 = use_h2(*cfg, *tgt);
  c->R2 = (uint16_t*)(c->ws + lay.R2);
  c->V2 = (uint16_t*)(c->ws + lay.V2);
  c->vsc = (float*)(c->ws + lay.vsc);
  c->rsc = (double*)(c->ws + lay.rsc);
  c->Yp = (float*)(c->ws + lay.Yp);
  c->prior_w = c->logreg ? 1.0 / (2.0 * tgt->prior_var) : 0.0;
  c->trained = 0;
  c->da_on = 0;
  c->last_batch = 0;
  if (cfg->surrogate) {
    dk::MlpBufs& b = c->mlp;
    b.D = cfg->d;
    b.H = MLP_H;
    b.d_state = cfg->d;
    auto fp = [&](size_t off) { return (float*)(c->ws + off); };
    b.master = fp(lay.mlp_master);
    b.eff = fp(lay.mlp_eff);
    b.grad = fp(lay.mlp_grad);
    b.m = fp(lay.mlp_m);
    b.in_mean = fp(lay.mlp_in_mean);
    b.in_scale = fp(lay.mlp_in_scale);
    b.stats = fp(lay.mlp_stats);
    b.Xs = fp(lay.mlp_Xs);
    b.ts = fp(lay.mlp_ts);
    b.xb = fp(lay.mlp_xb);
    b.tb = fp(lay.mlp_tb);
    b.a1 = fp(lay.mlp_a1);
    b.h1 = fp(lay.mlp_h1);
    b.a2 = fp(lay.mlp_a2);
    b.h2 = fp(lay.mlp_h2);
    b.ga1 = fp(lay.mlp_ga1);
    b.ga2 = fp(lay.mlp_ga2);
    b.out = fp(lay.mlp_out);
    b.gout = fp(lay.mlp_gout);
    b.loss = fp(lay.mlp_loss);
    b.bidx = (int*)(c->ws + lay.mlp_bidx);
    c->s_cur = dptr(c, lay.s_cur);
    c->s_new = dptr(c, lay.s_new);
    c->pass1 = (uint8_t*)(c->ws + lay.pass1);
    c->slot = (int*)(c->ws + lay.slot);
    c->idx = (int*)(c->ws + lay.idx);
    c->nsurv = (int*)(c->ws + lay.nsurv);
    c->npass = (int*)(c->ws + lay.npass);
    c->Vs = fp(lay.Vs);
    c->t64 = dptr(c, lay.t64);
    c->Zs = dptr(c, lay.Zs);
  } else {
    c->mlp = dk::MlpBufs{};
    c->s_cur = c->s_new = nullptr;
    c->pass1 = nullptr;
    c->slot = c->idx = c->nsurv = c->npass = nullptr;
    c->Vs = nullptr;
    c->t64 = c->Zs = nullptr;
  }
  c->nacc = (int32_t*)(c->ws + lay.nacc);
  c->wacc = (int32_t*)(c->ws + lay.wacc);
  c->la = dptr(c, lay.la);
  c->acc = (uint8_t*)(c->ws + lay.acc);
  c->U = dptr(c, lay.U);
  c->W = c->ws + lay.W;
  c->Wlo = c->ws + lay.Wlo;
  c->Xi = c->ws + lay.Xi;
  c->win = c->ws + lay.win;
  c->pmean = dptr(c, lay.pmean);
  c->pm2 = dptr(c, lay.pm2);
  c->pout = dptr(c, lay.pout);
  c->merr = dptr(c, lay.merr);
  c->psrf_on = 0;
  c->psrf_n = 0.0;
  c->Lp = dptr(c, lay.Lp);
  c->Gp = dptr(c, lay.Gp);
  c->hp = dptr(c, lay.hp);
  c->xrp = dptr(c, lay.xrp);
  c->Spg = dptr(c, lay.Spg);
  c->mpg = dptr(c, lay.mpg);
  c->Cp = dptr(c, lay.Cp);
  c->mpgp = dptr(c, lay.mpgp);
  c->linvb = dptr(c, lay.linvb);
  c->pinfo = (int32_t*)(c->ws + lay.pinfo);
  c->m_int = 0;
  c->loc_n = 0.0;
  c->pc_on = 0;
  c->wint = c->ws + lay.wint;
  c->xr = dptr(c, lay.xr);
  c->S = dptr(c, lay.S);
  c->m = dptr(c, lay.m);
  c->L = dptr(c, lay.L);
  c->Lnew = dptr(c, lay.Lnew);
  c->Llow = c->ws + lay.Llow;
  c->h = dptr(c, lay.h);
  c->syrk = c->ws + lay.syrk;
  c->status = (Status*)(c->ws + lay.status);
  c->proj_part = dptr(c, lay.proj_part);
  c->linv = dptr(c, lay.linv);
  c->nrb = target_row_blocks(*cfg, *tgt);
  c->nch = dk::step_chunks(cfg->d);
  c->cur = 0;
  c->steps = 0;
  c->siw = 0;
  c->last_jitter = -1;
  c->win_steps = 0;
  c->adapt_on = 0;
  c->N = 0.0;
  c->windows = 0;
  c->last_call_steps = 0;
  c->last_call_stages = 1;
  c->proj = nullptr;
  c->nproj = 0;
  c->trace = nullptr;
  c->trace_cap = c->trace_pos = 0;
  c->prof_on = false;
  c->ev_used = 0;
  for (int k = 0; k < DIAM_NSTAGES; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_cnt[k] = 0;
  }

  const int d = cfg->d, P = cfg->P;
  const long dd = (long)d * d, dP = (long)d * P;
  hipStream_t s = c->stream;
  auto bail = [&](int code) {
    delete c;
    return code;
  };
#define HIPCHK_INIT(expr)                                                                              \
  do {                                                                                                 \
    hipError_t _e = (expr);                                                                            \
    if (_e != hipSuccess) return bail(fail(DIAM_E_HIP, "%s: %s", #expr, hipGetErrorString(_e)));      \
  } while (0)
  HIPCHK_INIT(hipMemcpyAsync(c->X, x0, dP * sizeof(double), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_identity, dim3(nblk(dd)), dim3(256), 0, s, c->L, d);
  hipLaunchKernelGGL(k_fill, dim3(nblk(d)), dim3(256), 0, s, c->xr, (long)d, 0.0);
  hipLaunchKernelGGL(k_fill, dim3(nblk(d)), dim3(256), 0, s, c->m, (long)d, 0.0);
  hipLaunchKernelGGL(k_fill, dim3(nblk(dd)), dim3(256), 0, s, c->S, dd, 0.0);
  if (cfg->M > 1) reset_local(c);
  hipLaunchKernelGGL(k_fill_i32, dim3(nblk(P)), dim3(256), 0, s, c->nacc, (long)P);
  hipLaunchKernelGGL(k_fill_i32, dim3(nblk(P)), dim3(256), 0, s, c->wacc, (long)P);
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, c->status, 1);
  HIPCHK_INIT(hipGetLastError());
  HIPCHK_INIT(dk::round_factor(c->prec, c->L, c->Llow, d, s));
  // log pi(x0) and z0 = x0 (A = I, x_ref = 0)
  if (c->logreg) {
    HIPCHK_INIT(dk::init_eval(0, c->X, nullptr, c->V, c->Z, d, P, s));
    HIPCHK_INIT(dk::tgt_logreg(tgt->A, tgt->y, tgt->n_obs, (const float*)c->V, d, P, nullptr, c->lpp_part, s));
  } else {
    HIPCHK_INIT(dk::init_eval(c->prec == dk::P64, c->X, tgt->mu, c->V, c->Z, d, P, s));
    if (c->h2) {
      // log pi(x0) at scales from the states' spread, then the scales of the
      // proposals (the identity factor's spread included)
      HIPCHK_INIT(dk::h2_scales(c->X, tgt->mu, c->L, (const float*)tgt->R, d, P, c->vsc, c->R2, c->rsc, s, 1));
      HIPCHK_INIT(dk::h2_split_v(c->X, tgt->mu, c->vsc, d, P, c->V2, s));
      HIPCHK_INIT(dk::tgt_gauss_h2(c->R2, c->V2, c->rsc, d, P, c->Yp, c->lpp_part, s, tgt->twist));
      HIPCHK_INIT(dk::h2_scales(c->X, tgt->mu, c->L, (const float*)tgt->R, d, P, c->vsc, c->R2, c->rsc, s, 0));
    } else {
      HIPCHK_INIT(dk::tgt_gauss(c->prec, tgt->R, c->V, d, P, c->lpp_part, s, tgt->twist));
    }
  }
  HIPCHK_INIT(dk::init_finish(c->lpp_part, c->nrb, c->Z, c->X, c->prior_w, c->lp, c->zq, d, P, s));
  if (cfg->surrogate) hipLaunchKernelGGL(k_fill_i32, dim3(nblk(P)), dim3(256), 0, s, c->npass, (long)P);
#undef HIPCHK_INIT
  *out = c;
  return DIAM_OK;
}

extern "C" int diam_step_batch(diam_ctx* c, int32_t n, const double* W, const double* U, int32_t* n_accepted) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (n < 0) return fail(DIAM_E_ARG, "n_steps < 0");
  if (n == 0) return DIAM_OK;
  if (c->siw + n > c->cfg.n_lag)
    return fail(DIAM_E_STATE, "steps_in_window %d + n_steps %d exceeds n_lag %d", c->siw, n, c->cfg.n_lag);
  if ((uintptr_t)W % 16 || (uintptr_t)U % 16) return fail(DIAM_E_ARG, "W and U must be 16-byte aligned");
  const int d = c->cfg.d, P = c->cfg.P;
  const long dP = (long)d * P;
  hipStream_t s = c->stream;
  const Prec prec = c->prec;
  const int eb = (prec == dk::P64) ? 8 : 4;
  const int wb = (prec == dk::P64) ? 8 : (prec == dk::P32 ? 4 : 2);

  // normals for this call: caller FP64 W (used in place in FP64) or Philox
  const void* Wp = c->W;
  const void* Wlop = c->Wlo;
  int ps = prof_begin(c, DIAM_ST_RNG);
  if (W) {
    if (prec == dk::P64) Wp = W;
    else HIPCHK(dk::convert_normals(prec, W, (long)n * dP, c->W, c->Wlo, s));
  } else {
    HIPCHK(dk::normals(prec, c->cfg.seed, c->steps, n, d, P, c->W, c->Wlo, s));
  }
  const int stages = c->da_on ? 2 : 1;
  const double* Up = U;
  if (!Up) {
    HIPCHK(dk::uniforms(c->cfg.seed, c->steps, n, P, stages, c->U, s));
    Up = c->U;
  }
  prof_end(c, ps);
  const double beta = c->cfg.beta, alpha = c->cfg.alpha;
  const double cc = beta * alpha;
  const void* Lmat = (prec == dk::P64) ? (const void*)c->L : (const void*)c->Llow;
  // search directions of the whole batch (Algorithm 1: beta alpha A [W ... W])
  ps = prof_begin(c, DIAM_ST_PROPOSAL);
  if (c->pc_on)  // every chain about its own pair (M > 1, FP64)
    HIPCHK(dk::pc_gemm(c->Lp, (const double*)Wp, c->xrp, c->xr, (double*)c->Xi, d, P, n, cc,
                       1.0 - sqrt(1.0 - beta * beta), s));
  else
    HIPCHK(dk::trigemm(prec, Lmat, Wp, Wlop, c->Xi, d, (long)n * P, cc, s));
  prof_end(c, ps);

  auto at = [](const void* base, long elem, int bytes) { return (const void*)((const char*)base + elem * bytes); };
  const bool tracing = c->trace && c->trace_pos + n <= c->trace_cap;
  const int nfun = 1 + c->nproj;

  dk::StepArgs a{};
  a.d = d;
  a.P = P;
  a.prec = prec;
  const bool walk = walk_proposal(c->cfg);
  a.rho = walk ? 1.0 : sqrt(1.0 - beta * beta);
  a.c = cc;
  a.inv2a2 = walk ? 0.0 : 1.0 / (2.0 * alpha * alpha);
  a.xr = c->xr;
  a.mu = c->logreg ? nullptr : c->tgt.mu;
  a.X = c->X;
  a.Z = c->Z;
  a.V = c->V;
  a.nrb = c->nrb;
  a.nacc = n_accepted ? n_accepted : c->nacc;
  a.wacc = c->wacc;
  a.win = c->win;
  a.err = &c->status->err;
  a.v32 = c->logreg;
  a.vh = c->h2 ? c->V2 : nullptr;
  a.vsc = c->vsc;
  a.prior_w = c->prior_w;
  a.proj = c->proj;
  a.nproj = tracing ? c->nproj : 0;
  // proposal of the first step
  a.do_accept = 0;
  a.do_propose = 1;
  a.xi_nxt = c->Xi;
  a.w_nxt = Wp;
  a.wlo_nxt = Wlop;
  a.zq_part_nxt = c->zq_part + (long)c->cur * c->nch * P;
  a.pq_part_nxt = c->pq_part + (long)c->cur * c->nch * P;
  ps = prof_begin(c, DIAM_ST_STEP);
  HIPCHK(dk::step(a, s));
  prof_end(c, ps);
  // mixed Gaussian form: the target's K-split reduction runs inside the step
  const bool fuse_h2 = c->h2 && !c->da_on && dk::step_h2_ok(d, P, c->nrb);
  for (int t = 0; t < n; ++t) {
    const int cu = c->cur, nx = cu ^ 1;
    const double* u_t = Up + (long)t * stages * P;
    if (c->da_on) {
      // stage 1 on the surrogate, then the exact target on the survivors only
      ps = prof_begin(c, DIAM_ST_SURROGATE);
      HIPCHK(dk::da_screen(c->mlp, (const float*)c->V, d, P, c->nch, c->s_cur + (long)cu * P,
                           c->zq_part + (long)cu * c->nch * P, c->zq + (long)cu * P, u_t, a.inv2a2,
                           c->cfg.surrogate == 2, c->s_new, c->pass1, c->slot, c->idx, c->nsurv, c->npass, c->Vs,
                           s));
      prof_end(c, ps);
    }
    ps = prof_begin(c, DIAM_ST_TARGET);
    if (c->logreg)
      HIPCHK(dk::tgt_logreg(c->tgt.A, c->tgt.y, c->tgt.n_obs, c->da_on ? c->Vs : (const float*)c->V, d, P,
                            c->da_on ? c->nsurv : nullptr, c->lpp_part, s));
    else if (c->h2)
      HIPCHK(dk::tgt_gauss_h2(c->R2, c->V2, c->rsc, d, P, c->Yp, fuse_h2 ? nullptr : c->lpp_part, s, c->tgt.twist));
    else
      HIPCHK(dk::tgt_gauss(prec, c->tgt.R, c->V, d, P, c->lpp_part, s, c->tgt.twist));
    prof_end(c, ps);
    a.do_accept = 1;
    a.xi_cur = at(c->Xi, (long)t * dP, eb);
    a.w_cur = at(Wp, (long)t * dP, wb);
    a.wlo_cur = at(Wlop, (long)t * dP, 2);
    a.lpp_part = c->lpp_part;
    a.zq_part_cur = c->zq_part + (long)cu * c->nch * P;
    a.lp_cur = c->lp + (long)cu * P;
    a.zq_cur = c->zq + (long)cu * P;
    a.lp_nxt = c->lp + (long)nx * P;
    a.zq_nxt = c->zq + (long)nx * P;
    a.u = u_t;
    a.pq_part_cur = c->pq_part + (long)cu * c->nch * P;
    a.pq_part_nxt = c->pq_part + (long)nx * c->nch * P;
    a.da = c->da_on;
    if (c->da_on) {
      a.pass1 = c->pass1;
      // target partials of survivors are packed by stage-1 slot
      a.slot = c->slot;
      a.s_new = c->s_new;
      a.s_in = c->s_cur + (long)cu * P;
      a.s_out = c->s_cur + (long)nx * P;
      a.u2 = u_t + P;
      a.da_resid = c->cfg.surrogate == 2;
    }
    a.la_out = c->la + (long)t * P;
    a.acc_out = c->acc + (long)t * P;
    a.win_col0 = (long)(c->siw + t) * P;
    a.trace_lp = tracing ? c->trace + ((c->trace_pos + t) * nfun) * P : nullptr;
    a.proj_part = c->proj_part + (long)t * c->nch * (c->nproj > 0 ? c->nproj : 1) * P;
    a.do_propose = (t + 1 < n) ? 1 : 0;
    a.xi_nxt = at(c->Xi, (long)(t + 1) * dP, eb);
    a.w_nxt = at(Wp, (long)(t + 1) * dP, wb);
    a.wlo_nxt = at(Wlop, (long)(t + 1) * dP, 2);
    a.zq_part_nxt = c->zq_part + (long)nx * c->nch * P;
    ps = prof_begin(c, DIAM_ST_STEP);
    if (fuse_h2) HIPCHK(dk::step_h2(a, c->Yp, c->rsc, c->lpp_part, c->tgt.twist, s));
    else HIPCHK(dk::step(a, s));
    prof_end(c, ps);
    c->cur = nx;
  }
  if (tracing && c->nproj > 0)
    HIPCHK(dk::proj_reduce(c->proj_part, n, c->nch, c->nproj, P, c->trace + c->trace_pos * nfun * P, nfun, s));
  if (tracing) c->trace_pos += n;
  c->siw += n;
  c->win_steps += n;
  c->steps += n;
  c->last_call_steps = n;
  c->last_call_stages = stages;
  return DIAM_OK;
}

// ---- learned-part form -------------------------------------------------------
static int need_surrogate(diam_ctx* c) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (!c->cfg.surrogate) return fail(DIAM_E_STATE, "the context was created without surrogate buffers");
  return DIAM_OK;
}

extern "C" int diam_surrogate_train(diam_ctx* c, const double* X, const double* lp, int64_t n, int32_t steps,
                                    int32_t batch, double lr, uint64_t seed, double* loss) {
  int r = need_surrogate(c);
  if (r) return r;
  if (c->da_on) return fail(DIAM_E_STATE, "surrogate must stay fixed while delayed acceptance is on");
  if (!X || !lp) return fail(DIAM_E_ARG, "null training data");
  if (n < 2 || n > c->cfg.train_max) return fail(DIAM_E_ARG, "n = %ld outside [2, train_max = %ld]", (long)n,
                                                 (long)c->cfg.train_max);
  const int nmax = c->cfg.P > MLP_NMIN ? c->cfg.P : MLP_NMIN;
  if (steps < 0 || batch < 1 || batch > nmax) return fail(DIAM_E_ARG, "steps >= 0, 1 <= batch <= %d", nmax);
  if (!(lr > 0.0)) return fail(DIAM_E_ARG, "lr must be > 0");
  hipStream_t s = c->stream;
  const int ps = prof_begin(c, DIAM_ST_TRAIN);
  const double* target = lp;
  if (c->cfg.surrogate == 2) {
    // residual form: the network learns log pi(x) + |z(x)|^2 / (2 alpha^2)
    // with z under the current factor and pivot
    const int d = c->cfg.d, chunk = nmax;
    for (long k0 = 0; k0 < n; k0 += chunk) {
      const int nc = (int)(n - k0 < chunk ? n - k0 : chunk);
      HIPCHK(dk::trsm_whiten(c->L, X + k0 * d, c->xr, c->Zs, c->t64 + k0, c->linv, d, nc, s));
    }
    HIPCHK(dk::axpy_f64(lp, c->t64, 1.0 / (2.0 * c->cfg.alpha * c->cfg.alpha), n, c->t64, s));
    target = c->t64;
  }
  HIPCHK(dk::mlp_prepare(c->mlp, X, target, n, seed, s));
  dk::MlpBufs b = c->mlp;
  for (int t = 0; t < steps; ++t) {
    b.loss = c->mlp.loss + (t % LOSS_HIST);
    HIPCHK(dk::mlp_train_step(b, n, batch, t, seed, (float)lr, s));
  }
  prof_end(c, ps);
  c->trained = 1;
  c->last_batch = batch;
  if (loss) {
    float h[LOSS_HIST];
    HIPCHK(hipMemcpyAsync(h, c->mlp.loss, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int k = steps < 50 ? steps : 50;
    double acc = 0.0;
    for (int t = steps - k; t < steps; ++t) acc += h[t % LOSS_HIST];
    *loss = k ? acc / k : NAN;
  } else {
    HIPCHK(hipStreamSynchronize(s));
  }
  return DIAM_OK;
}

extern "C" int diam_surrogate_eval(diam_ctx* c, const double* X, int32_t n, double* out) {
  int r = need_surrogate(c);
  if (r) return r;
  if (!c->trained) return fail(DIAM_E_STATE, "surrogate not trained");
  const int nmax = c->cfg.P > MLP_NMIN ? c->cfg.P : MLP_NMIN;
  if (!X || !out || n < 0 || n > nmax) return fail(DIAM_E_ARG, "need X, out and 0 <= n <= %d", nmax);
  if (n == 0) return DIAM_OK;
  HIPCHK(dk::mlp_eval(c->mlp, X, nullptr, n, out, c->stream));
  return DIAM_OK;
}

extern "C" int diam_set_delayed_acceptance(diam_ctx* c, int32_t on) {
  int r = need_surrogate(c);
  if (r) return r;
  if (!on) {
    c->da_on = 0;
    return DIAM_OK;
  }
  if (!c->logreg) return fail(DIAM_E_STATE, "delayed acceptance needs the logistic target");
  if (!c->trained) return fail(DIAM_E_STATE, "surrogate not trained");
  if (c->da_on) return DIAM_OK;
  // surrogate at the current states; survivor counters restart
  HIPCHK(dk::mlp_eval(c->mlp, c->X, nullptr, c->cfg.P, c->s_cur + (long)c->cur * c->cfg.P, c->stream));
  hipLaunchKernelGGL(k_fill_i32, dim3(nblk(c->cfg.P)), dim3(256), 0, c->stream, c->npass, (long)c->cfg.P);
  HIPCHK(hipGetLastError());
  c->da_on = 1;
  return DIAM_OK;
}

extern "C" int diam_merge_moments(diam_ctx* c) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (c->siw < 1) return fail(DIAM_E_STATE, "no steps since the last merge");
  const int d = c->cfg.d, P = c->cfg.P;
  const long K = (long)c->siw * P;
  hipStream_t s = c->stream;
  const int ps = prof_begin(c, DIAM_ST_MERGE);
  double* G = c->Lnew;  // scratch until the next factorisation
  bool global = true;
  long Kg = K;
  if (c->cfg.M > 1) {
    // chain-local sums of the batch (eqs. mom2p, mom1p); every M-th interval
    // the P chains' sums are merged into the global moments (eqs. mom2g, mom1g)
    HIPCHK(dk::pc_scatter((const double*)c->win, c->Gp, c->hp, d, P, c->siw, s));
    c->loc_n += (double)c->siw;
    c->m_int += 1;
    global = c->m_int == c->cfg.M;
    if (global) {
      HIPCHK(dk::pc_sum(c->Gp, c->hp, G, c->h, d, P, s));
      Kg = (long)llround(c->loc_n) * P;
    }
  } else {
    HIPCHK(dk::syrk_window(c->prec, c->win, c->wint, d, K, G, c->h, c->syrk, s));
  }
  if (global) HIPCHK(dk::fold_moments(G, c->h, c->xr, c->N, Kg, c->S, c->m, d, s));
  prof_end(c, ps);
  if (c->psrf_on) {
    // the store still holds the window's states and xr its pivot
    const int pp = prof_begin(c, DIAM_ST_PSRF);
    HIPCHK(dk::psrf_accumulate(c->prec, c->win, d, P, c->siw, c->xr, c->psrf_n, c->pmean, c->pm2, s));
    prof_end(c, pp);
    c->psrf_n += (double)c->siw;
  }
  if (global) {
    c->N += (double)Kg;
    if (c->cfg.M > 1) reset_local(c);
  }
  c->siw = 0;
  c->windows += 1;
  return DIAM_OK;
}

extern "C" int diam_set_beta_adaptation(diam_ctx* c, int32_t on, double acc_min, double acc_max, double factor,
                                        double beta_max) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (on) {
    if (!(acc_min >= 0.0 && acc_min < acc_max && acc_max <= 1.0))
      return fail(DIAM_E_ARG, "need 0 <= acc_min < acc_max <= 1");
    if (!(factor > 1.0) || !std::isfinite(factor)) return fail(DIAM_E_ARG, "factor must be finite and > 1");
    if (!(beta_max > 0.0 && beta_max <= 1.0)) return fail(DIAM_E_ARG, "beta_max must lie in (0, 1]");
    c->acc_min = acc_min;
    c->acc_max = acc_max;
    c->adapt_factor = factor;
    c->beta_max = beta_max;
  }
  c->adapt_on = on ? 1 : 0;
  return DIAM_OK;
}

extern "C" int diam_psrf_enable(diam_ctx* c, int32_t on) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (on) c->psrf_n = 0.0;  // zeroed lazily: the first fold after this overwrites
  c->psrf_on = on ? 1 : 0;
  return DIAM_OK;
}

extern "C" int diam_psrf(diam_ctx* c, double* out, double* worst) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (!c->psrf_on) return fail(DIAM_E_STATE, "the PSRF diagnostic is not enabled");
  const int d = c->cfg.d, P = c->cfg.P;
  if (P < 2) return fail(DIAM_E_STATE, "the PSRF needs at least two chains");
  if (c->psrf_n < 2.0) return fail(DIAM_E_STATE, "the PSRF needs at least two folded states per chain (%g)", c->psrf_n);
  double* o = out ? out : c->pout;
  HIPCHK(dk::psrf_finalize(c->pmean, c->pm2, d, P, c->psrf_n, o, c->stream));
  if (worst) {
    std::vector<double> h(d);
    HIPCHK(hipMemcpyAsync(h.data(), o, d * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    double w = -INFINITY;
    for (int i = 0; i < d; ++i) {
      if (std::isnan(h[i])) { w = NAN; break; }
      w = std::max(w, h[i] - 1.0);
    }
    *worst = w;
  }
  return DIAM_OK;
}

extern "C" int diam_moment_error(diam_ctx* c, const double* Sigma, const double* mu, double* cov_rel,
                                 double* mean_abs) {
  if (!c || !Sigma || !cov_rel) return fail(DIAM_E_ARG, "null argument");
  HIPCHK(dk::moment_error(c->S, c->m, Sigma, mu, c->cfg.d, c->merr, c->stream));
  double h[2];
  HIPCHK(hipMemcpyAsync(h, c->merr, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *cov_rel = h[0];
  if (mean_abs) *mean_abs = mu ? h[1] : NAN;
  return DIAM_OK;
}

static int read_status(diam_ctx* c, Status* st) {
  HIPCHK(hipMemcpyAsync(st, c->status, sizeof(Status), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return DIAM_OK;
}

// Error words flagged by the steps since the last update: bit 0, a target
// log density of +inf; bit 1, a proposal outside the half range of the
// mixed-form Gaussian target's scaled operands (more than about 1000 spreads
// from the target mean, where the spread is the larger of the states' largest
// deviation and the proposal scale at the last update).  Cleared once reported.
static int status_error(diam_ctx* c, int err) {
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, c->stream, c->status, 1);
  if (err & 1) return fail(DIAM_E_TARGET, "the target log density returned +inf");
  return fail(DIAM_E_TARGET, "a proposal left the range of the mixed-form target's scaled half operands");
}

// Mixed-form Gaussian target: coordinate and row scales of the half operands
// from the current states and factor (kept until the next update).
static int refresh_h2(diam_ctx* c) {
  if (!c->h2) return DIAM_OK;
  HIPCHK(dk::h2_scales(c->X, c->tgt.mu, c->L, (const float*)c->tgt.R, c->cfg.d, c->cfg.P, c->vsc, c->R2, c->rsc,
                       c->stream));
  return DIAM_OK;
}

// C = S - m m^T (eq. sampcov) assembled into Lnew and factored in place,
// retrying on C + eps_j I, eps_j = 10^j jitter0 tr(C)/d (1 if not > 0), when a
// pivot is not positive.  *j: -1, the level used, or jitter_tries when every
// try failed.  Also reports a target error flagged by the steps before.
static int factor_jitter(diam_ctx* c, const double* S, const double* m, int* j) {
  const int d = c->cfg.d;
  hipStream_t s = c->stream;
  Status st;
  int ps = prof_begin(c, DIAM_ST_CHOL);
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, c->status, 0);
  HIPCHK(dk::cov_assemble(S, m, 0.0, c->Lnew, &c->status->trace, d, s));
  HIPCHK(dk::potrf(c->Lnew, d, &c->status->info, c->linv, s));
  prof_end(c, ps);
  int r = read_status(c, &st);
  if (r) return r;
  r = prof_flush(c);
  if (r) return r;
  if (st.err) return status_error(c, st.err);
  *j = -1;
  if (st.info != 0) {
    const double tr = st.trace / d;
    const double sc = (tr > 0.0 && isfinite(tr)) ? tr : 1.0;
    *j = c->cfg.jitter_tries;
    for (int q = 0; q < c->cfg.jitter_tries; ++q) {
      const double eps = pow(10.0, q) * c->cfg.jitter0 * sc;
      ps = prof_begin(c, DIAM_ST_CHOL);
      hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, c->status, 0);
      HIPCHK(dk::cov_assemble(S, m, eps, c->Lnew, nullptr, d, s));
      HIPCHK(dk::potrf(c->Lnew, d, &c->status->info, c->linv, s));
      prof_end(c, ps);
      r = read_status(c, &st);
      if (r) return r;
      if (st.info == 0) {
        *j = q;
        break;
      }
    }
  }
  return DIAM_OK;
}

// M > 1 inside a batch: every chain's factor and pivot from its local update
// of the global moments (eqs. mom2pg, mom1pg, cov2pg) and z of the chain under
// its new pair.  All chains are assembled, factored and whitened in batched
// launches; a chain whose factorisation fails gets the jitter rule alone, and
// keeps its pair if every level fails.
static int update_local(diam_ctx* c, int32_t* jitter_used) {
  const int d = c->cfg.d, P = c->cfg.P;
  const long dd = (long)d * d, sL = (long)(dk::chol_scratch_bytes(d) / sizeof(double));
  hipStream_t s = c->stream;
  int ps = prof_begin(c, DIAM_ST_CHOL);
  if (!c->pc_on) {  // first local update of the batch: every chain starts from the shared pair
    HIPCHK(dk::pc_bcast(c->L, c->xr, c->Lp, c->xrp, d, P, s));
    c->pc_on = 1;
  }
  hipLaunchKernelGGL(k_fill_i32, dim3(nblk(P)), dim3(256), 0, s, c->pinfo, (long)P);
  HIPCHK(dk::pc_cov(c->S, c->m, c->N, c->Gp, c->hp, c->xr, c->loc_n, c->Cp, c->mpgp, d, P, s));
  HIPCHK(dk::potrf_batched(c->Cp, dd, d, c->pinfo, c->linvb, sL, P, s));
  prof_end(c, ps);
  std::vector<int32_t> info(P);
  HIPCHK(hipMemcpyAsync(info.data(), c->pinfo, P * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  Status st;
  int r = read_status(c, &st);  // synchronises: info is on the host
  if (r) return r;
  r = prof_flush(c);
  if (r) return r;
  if (st.err) return status_error(c, st.err);
  int jmax = -1, failed = 0;
  for (int p = 0; p < P; ++p) {
    if (info[p] == 0) continue;
    HIPCHK(dk::pc_moments(c->S, c->m, c->N, c->Gp + p * dd, c->hp + (long)p * d, c->xr, c->loc_n, c->Spg, c->mpg,
                          d, s));
    int j = -1;
    r = factor_jitter(c, c->Spg, c->mpg, &j);
    if (r) return r;
    jmax = std::max(jmax, j);
    if (j == c->cfg.jitter_tries) {
      failed += 1;  // its status word stays set: factor and pivot kept
      continue;
    }
    HIPCHK(hipMemcpyAsync(c->Cp + p * dd, c->Lnew, dd * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(c->mpgp + (long)p * d, c->mpg, d * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemsetAsync(c->pinfo + p, 0, sizeof(int32_t), s));
  }
  ps = prof_begin(c, DIAM_ST_WHITEN);
  HIPCHK(dk::pc_adopt(c->Cp, c->mpgp, c->pinfo, c->Lp, c->xrp, d, P, s));
  HIPCHK(dk::trsm_whiten_batched(c->Lp, dd, c->X, c->xrp, c->Z, c->zq + (long)c->cur * P, c->linvb, sL, d, P,
                                 c->pinfo, s));
  prof_end(c, ps);
  c->last_jitter = jmax;
  if (jitter_used) *jitter_used = jmax;
  if (failed)
    return fail(DIAM_E_NOT_PD, "%d chain covariances not positive definite at any of %d jitter levels", failed,
                c->cfg.jitter_tries);
  return DIAM_OK;
}

static int update_impl(diam_ctx* c, int32_t* jitter_used, bool refactor) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (c->siw != 0) return fail(DIAM_E_STATE, "update inside a window (steps_in_window = %d)", c->siw);
  const int d = c->cfg.d, P = c->cfg.P;
  hipStream_t s = c->stream;
  Status st;
  // step-size adaptation (Algorithm 1, update block): the acceptance ratio of
  // the steps since the last update, pooled over the chains, against the band
  if (c->adapt_on && c->win_steps > 0) {
    std::vector<int32_t> wa(P);
    HIPCHK(hipMemcpyAsync(wa.data(), c->wacc, P * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    long tot = 0;
    for (int p = 0; p < P; ++p) tot += wa[p];
    const double rate = (double)tot / ((double)P * (double)c->win_steps);
    if (rate > c->acc_max) c->cfg.beta = std::min(c->cfg.beta * c->adapt_factor, c->beta_max);
    else if (rate < c->acc_min) c->cfg.beta = c->cfg.beta / c->adapt_factor;
  }
  hipLaunchKernelGGL(k_fill_i32, dim3(nblk(P)), dim3(256), 0, s, c->wacc, (long)P);
  c->win_steps = 0;
  if (!refactor) {  // fixed factor: beta only; still report a target error of the past steps
    if (jitter_used) *jitter_used = -1;
    int r = read_status(c, &st);
    if (r) return r;
    r = prof_flush(c);
    if (r) return r;
    if (st.err) return status_error(c, st.err);
    return refresh_h2(c);
  }
  if (c->cfg.M > 1 && c->m_int > 0) return update_local(c, jitter_used);
  int j = -1;
  int r = factor_jitter(c, c->S, c->m, &j);
  if (r) return r;
  c->last_jitter = j;
  if (jitter_used) *jitter_used = j;
  if (j == c->cfg.jitter_tries)
    return fail(DIAM_E_NOT_PD, "covariance not positive definite at any of %d jitter levels", c->cfg.jitter_tries);
  double* t = c->L;
  c->L = c->Lnew;
  c->Lnew = t;
  c->pc_on = 0;  // every chain shares the new pair again
  const int ps = prof_begin(c, DIAM_ST_WHITEN);
  HIPCHK(dk::round_factor(c->prec, c->L, c->Llow, d, s));
  HIPCHK(hipMemcpyAsync(c->xr, c->m, d * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(dk::trsm_whiten(c->L, c->X, c->xr, c->Z, c->zq + (long)c->cur * P, c->linv, d, P, s));
  const int r2 = refresh_h2(c);
  prof_end(c, ps);
  return r2;
}

extern "C" int diam_update_proposal(diam_ctx* c, int32_t* jitter_used) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  return update_impl(c, jitter_used, !fixed_factor(c->cfg));
}

extern "C" int diam_seed_moments(diam_ctx* c, const double* S0, const double* m0, double N0, int32_t* jitter_used) {
  if (!c || !S0 || !m0) return fail(DIAM_E_ARG, "null argument");
  if (!(N0 >= 0.0)) return fail(DIAM_E_ARG, "N0 must be >= 0");
  if (c->siw != 0) return fail(DIAM_E_STATE, "seed inside a window");
  const int d = c->cfg.d;
  HIPCHK(hipMemcpyAsync(c->S, S0, (size_t)d * d * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->m, m0, (size_t)d * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->N = N0;
  if (c->cfg.M > 1) reset_local(c);
  return update_impl(c, jitter_used, true);
}

extern "C" int diam_set_trace(diam_ctx* c, const double* proj, int32_t n_proj, double* trace, int64_t capacity) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (n_proj < 0 || n_proj > 4) return fail(DIAM_E_ARG, "n_proj must be in [0, 4]");
  if (n_proj > 0 && !proj) return fail(DIAM_E_ARG, "null proj");
  if (trace && capacity < 0) return fail(DIAM_E_ARG, "negative capacity");
  if ((uintptr_t)proj % 16 || (uintptr_t)trace % 16) return fail(DIAM_E_ARG, "proj and trace must be 16-byte aligned");
  c->proj = proj;
  c->nproj = trace ? n_proj : 0;
  c->trace = trace;
  c->trace_cap = trace ? capacity : 0;
  c->trace_pos = 0;
  return DIAM_OK;
}

static int field_info(diam_ctx* c, int32_t f, const void** src, size_t* bytes) {
  const size_t d = c->cfg.d, P = c->cfg.P, n = c->last_call_steps;
  switch (f) {
    case DIAM_F_X: *src = c->X; *bytes = d * P * 8; break;
    case DIAM_F_Z: *src = c->Z; *bytes = d * P * 8; break;
    case DIAM_F_LOGP: *src = c->lp + (long)c->cur * P; *bytes = P * 8; break;
    case DIAM_F_ZQ: *src = c->zq + (long)c->cur * P; *bytes = P * 8; break;
    case DIAM_F_XREF: *src = c->xr; *bytes = d * 8; break;
    case DIAM_F_L: *src = c->L; *bytes = d * d * 8; break;
    case DIAM_F_S: *src = c->S; *bytes = d * d * 8; break;
    case DIAM_F_M: *src = c->m; *bytes = d * 8; break;
    case DIAM_F_XI: *src = c->Xi; *bytes = d * P * n * (c->prec == dk::P64 ? 8 : 4); break;
    case DIAM_F_LA: *src = c->la; *bytes = n * P * 8; break;
    case DIAM_F_ACC: *src = c->acc; *bytes = n * P; break;
    case DIAM_F_NACC: *src = c->nacc; *bytes = P * 4; break;
    case DIAM_F_W: *src = c->W; *bytes = d * P * n * (c->prec == dk::P64 ? 8 : (c->prec == dk::P32 ? 4 : 2)); break;
    case DIAM_F_WLO:
      if (c->prec != dk::PMIX) return fail(DIAM_E_ARG, "DIAM_F_WLO exists only in DIAM_MIXED");
      *src = c->Wlo; *bytes = d * P * n * 2; break;
    case DIAM_F_U: *src = c->U; *bytes = n * P * 8 * c->last_call_stages; break;
    case DIAM_F_LP:
    case DIAM_F_XREFP:
      if (c->cfg.M <= 1) return fail(DIAM_E_ARG, "field %d exists only with M > 1", f);
      if (f == DIAM_F_LP) { *src = c->Lp; *bytes = P * d * d * 8; }
      else { *src = c->xrp; *bytes = d * P * 8; }
      break;
    case DIAM_F_SURR:
    case DIAM_F_NPASS:
    case DIAM_F_MLP_PARAMS:
    case DIAM_F_MLP_GRAD:
    case DIAM_F_MLP_BATCH:
    case DIAM_F_MLP_STATS: {
      if (!c->cfg.surrogate) return fail(DIAM_E_ARG, "field %d needs surrogate buffers", f);
      const size_t np = dk::mlp_nparam(c->cfg.d, MLP_H);
      if (f == DIAM_F_SURR) {
        if (!c->da_on) return fail(DIAM_E_STATE, "DIAM_F_SURR is kept only under delayed acceptance");
        *src = c->s_cur + (long)c->cur * P;
        *bytes = P * 8;
      } else if (f == DIAM_F_NPASS) {
        *src = c->npass; *bytes = P * 4;
      } else if (f == DIAM_F_MLP_PARAMS) {
        *src = c->mlp.master; *bytes = np * 4;
      } else if (f == DIAM_F_MLP_GRAD) {
        *src = c->mlp.grad; *bytes = np * 4;
      } else if (f == DIAM_F_MLP_BATCH) {
        *src = c->mlp.bidx; *bytes = (size_t)c->last_batch * 4;
      } else {
        *src = c->mlp.in_mean; *bytes = (2 * d + 2) * 4;
      }
      break;
    }
    default: return fail(DIAM_E_ARG, "unknown field %d", f);
  }
  return DIAM_OK;
}

extern "C" int diam_field_bytes(diam_ctx* c, int32_t field, size_t* bytes) {
  if (!c || !bytes) return fail(DIAM_E_ARG, "null argument");
  const void* src;
  return field_info(c, field, &src, bytes);
}

extern "C" int diam_get(diam_ctx* c, int32_t field, void* dst, size_t bytes) {
  if (!c || !dst) return fail(DIAM_E_ARG, "null argument");
  const void* src;
  size_t b;
  int r = field_info(c, field, &src, &b);
  if (r) return r;
  if (bytes != b) return fail(DIAM_E_ARG, "field %d has %zu bytes, got %zu", field, b, bytes);
  if (b) HIPCHK(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToDevice, c->stream));
  return DIAM_OK;
}

extern "C" int diam_get_stats(diam_ctx* c, diam_stats* out) {
  if (!c || !out) return fail(DIAM_E_ARG, "null argument");
  out->steps = c->steps;
  out->steps_in_window = c->siw;
  out->last_jitter = c->last_jitter;
  out->n_samples = c->N;
  out->windows = c->windows;
  out->last_call_steps = c->last_call_steps;
  out->beta = c->cfg.beta;
  return DIAM_OK;
}

extern "C" const char* diam_last_error(void) { return g_err; }

extern "C" void diam_destroy(diam_ctx* c) {
  if (!c) return;
  prof_release(c);
  delete c;
}
