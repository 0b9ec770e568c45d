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

static int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
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
  size_t X, Z, V, lp, zq, lpp_part, zq_part, nacc, la, acc, U, W, Wlo, Xi, win, wint, xr, S, m, L, Lnew, Llow, h,
      syrk, status, proj_part, linv, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int elem_bytes_ctr(int prec) { return prec == DIAM_FP64 ? 8 : 4; }

Layout make_layout(const diam_config& c) {
  const size_t d = c.d, P = c.P, nl = c.n_lag;
  const size_t dP = d * P, dd = d * d, win = d * P * nl;
  const int nrb = dk::tgt_row_blocks(c.d), nch = dk::step_chunks(c.d);
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
  L.nacc = take(P * 4);
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
  double *X, *Z, *lp, *zq, *lpp_part, *zq_part, *la, *U, *xr, *S, *m, *L, *Lnew, *h, *proj_part, *linv;
  void *V, *W, *Wlo, *Xi, *win, *wint, *Llow, *syrk;
  int32_t* nacc;
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
  return DIAM_OK;
}

extern "C" int diam_workspace_bytes(const diam_config* cfg, size_t* bytes) {
  int r = check_cfg(cfg);
  if (r) return r;
  if (!bytes) return fail(DIAM_E_ARG, "null bytes");
  *bytes = make_layout(*cfg).total;
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
    const int n = 2 * (c->cfg.n_lag * 2 + 64);
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
  if (!tgt || tgt->kind != DIAM_TGT_GAUSS || !tgt->mu || !tgt->R) return fail(DIAM_E_ARG, "bad target");
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(DIAM_E_ARG, "workspace null or not 256-byte aligned");
  if (!x0) return fail(DIAM_E_ARG, "null x0");
  Layout lay = make_layout(*cfg);
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
  c->nacc = (int32_t*)(c->ws + lay.nacc);
  c->la = dptr(c, lay.la);
  c->acc = (uint8_t*)(c->ws + lay.acc);
  c->U = dptr(c, lay.U);
  c->W = c->ws + lay.W;
  c->Wlo = c->ws + lay.Wlo;
  c->Xi = c->ws + lay.Xi;
  c->win = c->ws + lay.win;
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
  c->nrb = dk::tgt_row_blocks(cfg->d);
  c->nch = dk::step_chunks(cfg->d);
  c->cur = 0;
  c->steps = 0;
  c->siw = 0;
  c->last_jitter = -1;
  c->N = 0.0;
  c->windows = 0;
  c->last_call_steps = 0;
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
  hipLaunchKernelGGL(k_fill_i32, dim3(nblk(P)), dim3(256), 0, s, c->nacc, (long)P);
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, c->status, 1);
  HIPCHK_INIT(hipGetLastError());
  HIPCHK_INIT(dk::round_factor(c->prec, c->L, c->Llow, d, s));
  // log pi(x0) and z0 = x0 (A = I, x_ref = 0)
  HIPCHK_INIT(dk::init_eval(c->prec, c->X, tgt->mu, c->V, c->Z, d, P, s));
  HIPCHK_INIT(dk::tgt_gauss(c->prec, tgt->R, c->V, d, P, c->lpp_part, s));
  HIPCHK_INIT(dk::init_finish(c->lpp_part, c->nrb, c->Z, c->lp, c->zq, d, P, s));
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
  const double* Up = U;
  if (!Up) {
    HIPCHK(dk::uniforms(c->cfg.seed, c->steps, n, P, 1, c->U, s));
    Up = c->U;
  }
  prof_end(c, ps);
  const double beta = c->cfg.beta, alpha = c->cfg.alpha;
  const double cc = beta * alpha;
  const void* Lmat = (prec == dk::P64) ? (const void*)c->L : (const void*)c->Llow;
  // search directions of the whole batch (Algorithm 1: beta alpha A [W ... W])
  ps = prof_begin(c, DIAM_ST_PROPOSAL);
  HIPCHK(dk::trigemm(prec, Lmat, Wp, Wlop, c->Xi, d, (long)n * P, cc, s));
  prof_end(c, ps);

  auto at = [](const void* base, long elem, int bytes) { return (const void*)((const char*)base + elem * bytes); };
  const bool tracing = c->trace && c->trace_pos + n <= c->trace_cap;
  const int nfun = 1 + c->nproj;

  dk::StepArgs a{};
  a.d = d;
  a.P = P;
  a.prec = prec;
  a.rho = sqrt(1.0 - beta * beta);
  a.c = cc;
  a.inv2a2 = 1.0 / (2.0 * alpha * alpha);
  a.xr = c->xr;
  a.mu = c->tgt.mu;
  a.X = c->X;
  a.Z = c->Z;
  a.V = c->V;
  a.nrb = c->nrb;
  a.nacc = n_accepted ? n_accepted : c->nacc;
  a.win = c->win;
  a.err = &c->status->err;
  a.proj = c->proj;
  a.nproj = tracing ? c->nproj : 0;
  // proposal of the first step
  a.do_accept = 0;
  a.do_propose = 1;
  a.xi_nxt = c->Xi;
  a.w_nxt = Wp;
  a.wlo_nxt = Wlop;
  a.zq_part_nxt = c->zq_part + (long)c->cur * c->nch * P;
  ps = prof_begin(c, DIAM_ST_STEP);
  HIPCHK(dk::step(a, s));
  prof_end(c, ps);
  for (int t = 0; t < n; ++t) {
    ps = prof_begin(c, DIAM_ST_TARGET);
    HIPCHK(dk::tgt_gauss(prec, c->tgt.R, c->V, d, P, c->lpp_part, s));
    prof_end(c, ps);
    const int cu = c->cur, nx = cu ^ 1;
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
    a.u = Up + (long)t * P;
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
    HIPCHK(dk::step(a, s));
    prof_end(c, ps);
    c->cur = nx;
  }
  if (tracing && c->nproj > 0)
    HIPCHK(dk::proj_reduce(c->proj_part, n, c->nch, c->nproj, P, c->trace + c->trace_pos * nfun * P, nfun, s));
  if (tracing) c->trace_pos += n;
  c->siw += n;
  c->steps += n;
  c->last_call_steps = n;
  return DIAM_OK;
}

extern "C" int diam_merge_moments(diam_ctx* c) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (c->siw < 1) return fail(DIAM_E_STATE, "no steps since the last merge");
  const int d = c->cfg.d, P = c->cfg.P;
  const long K = (long)c->siw * P;
  hipStream_t s = c->stream;
  const void* Xs = c->win;
  const int ps = prof_begin(c, DIAM_ST_MERGE);
  if (c->prec == dk::PMIX) {
    HIPCHK(dk::transpose_bf16((const uint16_t*)c->win, (uint16_t*)c->wint, d, K, s));
    Xs = c->wint;
  }
  double* G = c->Lnew;  // scratch until the next factorisation
  HIPCHK(dk::syrk_window(c->prec, Xs, d, K, G, c->h, c->syrk, s));
  HIPCHK(dk::fold_moments(G, c->h, c->xr, c->N, K, c->S, c->m, d, s));
  prof_end(c, ps);
  c->N += (double)K;
  c->siw = 0;
  c->windows += 1;
  return DIAM_OK;
}

static int read_status(diam_ctx* c, Status* st) {
  HIPCHK(hipMemcpyAsync(st, c->status, sizeof(Status), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return DIAM_OK;
}

extern "C" int diam_update_proposal(diam_ctx* c, int32_t* jitter_used) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (c->siw != 0) return fail(DIAM_E_STATE, "update inside a window (steps_in_window = %d)", c->siw);
  const int d = c->cfg.d, P = c->cfg.P;
  hipStream_t s = c->stream;
  Status st;
  int ps = prof_begin(c, DIAM_ST_CHOL);
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, c->status, 0);
  HIPCHK(dk::cov_assemble(c->S, c->m, 0.0, c->Lnew, &c->status->trace, d, s));
  HIPCHK(dk::potrf(c->Lnew, d, &c->status->info, c->linv, s));
  prof_end(c, ps);
  int r = read_status(c, &st);
  if (r) return r;
  r = prof_flush(c);
  if (r) return r;
  if (st.err) {
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, c->status, 1);
    return fail(DIAM_E_TARGET, "the target log density returned +inf");
  }
  int j = -1;
  if (st.info != 0) {
    const double tr = st.trace / d;
    const double sc = (tr > 0.0 && isfinite(tr)) ? tr : 1.0;
    j = c->cfg.jitter_tries;
    for (int q = 0; q < c->cfg.jitter_tries; ++q) {
      const double eps = pow(10.0, q) * c->cfg.jitter0 * sc;
      ps = prof_begin(c, DIAM_ST_CHOL);
      hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, c->status, 0);
      HIPCHK(dk::cov_assemble(c->S, c->m, eps, c->Lnew, nullptr, d, s));
      HIPCHK(dk::potrf(c->Lnew, d, &c->status->info, c->linv, s));
      prof_end(c, ps);
      r = read_status(c, &st);
      if (r) return r;
      if (st.info == 0) {
        j = q;
        break;
      }
    }
  }
  c->last_jitter = j;
  if (jitter_used) *jitter_used = j;
  if (j == c->cfg.jitter_tries)
    return fail(DIAM_E_NOT_PD, "covariance not positive definite at any of %d jitter levels", c->cfg.jitter_tries);
  double* t = c->L;
  c->L = c->Lnew;
  c->Lnew = t;
  ps = prof_begin(c, DIAM_ST_WHITEN);
  HIPCHK(dk::round_factor(c->prec, c->L, c->Llow, d, s));
  HIPCHK(hipMemcpyAsync(c->xr, c->m, d * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(dk::trsm_whiten(c->L, c->X, c->xr, c->Z, c->zq + (long)c->cur * P, c->linv, d, P, s));
  prof_end(c, ps);
  return DIAM_OK;
}

extern "C" int diam_seed_moments(diam_ctx* c, const double* S0, const double* m0, double N0, int32_t* jitter_used) {
  if (!c || !S0 || !m0) return fail(DIAM_E_ARG, "null argument");
  if (!(N0 >= 0.0)) return fail(DIAM_E_ARG, "N0 must be >= 0");
  if (c->siw != 0) return fail(DIAM_E_STATE, "seed inside a window");
  const int d = c->cfg.d;
  HIPCHK(hipMemcpyAsync(c->S, S0, (size_t)d * d * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->m, m0, (size_t)d * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->N = N0;
  return diam_update_proposal(c, jitter_used);
}

extern "C" int diam_set_trace(diam_ctx* c, const double* proj, int32_t n_proj, double* trace, int64_t capacity) {
  if (!c) return fail(DIAM_E_ARG, "null context");
  if (n_proj < 0 || n_proj > 4) return fail(DIAM_E_ARG, "n_proj must be in [0, 4]");
  if (n_proj > 0 && !proj) return fail(DIAM_E_ARG, "null proj");
  if (trace && capacity < 0) return fail(DIAM_E_ARG, "negative capacity");
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
    case DIAM_F_U: *src = c->U; *bytes = n * P * 8; break;
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
  return DIAM_OK;
}

extern "C" const char* diam_last_error(void) { return g_err; }

extern "C" void diam_destroy(diam_ctx* c) {
  if (!c) return;
  prof_release(c);
  delete c;
}
