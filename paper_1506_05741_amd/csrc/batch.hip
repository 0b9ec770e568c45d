// Host runtime of the batched form (include/diam.h, diam_batch_*): G
// independent Gaussian problems of uneven dimension, P chains each, FP32
// contractions with FP64 states, moments and Cholesky.  One window of every
// problem is one sequence of grouped launches (a tile list per phase maps
// workgroups to problems); with graphs on, the whole window, its n_lag step
// loop included, is captured once into a hipGraph and replayed.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/diam.h"
#include "kernels.h"

int diam_fail_v(int code, const char* fmt, va_list ap);

static int bfail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  diam_fail_v(code, fmt, ap);
  va_end(ap);
  return code;
}

#define BCHK(expr)                                                                    \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) return bfail(DIAM_E_HIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

using dk::BProb;
using dk::BTile;

namespace {

constexpr int NB = dk::CHOL_NB;

inline int cdivh(long a, long b) { return (int)((a + b - 1) / b); }
inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
// leading dimension of the padded target and proposal operands (16-byte rows)
inline int pad4(int d) { return (d + 3) & ~3; }

struct Seg {
  long off = 0;
  int n = 0;
};

// Workspace offsets of one problem.
struct PLay {
  size_t X, Z, xr, lp, zq, zq_part, lpp_part, la, acc, V, Xi, win, S, m, L, C, Linv, G, h, Llow, nacc, Rp, Vp, Lp;
};

struct BLay {
  std::vector<PLay> p;
  std::vector<size_t> Woff;  // offset of each problem's normals inside W_all (floats)
  size_t W_all, U_all, info, win_ctr, N, err, probs, tiles, pitems, pstep, pctl, total;
  long nW, nU;
  long ntiles;
};

// Tile lists of every phase (host side, uploaded once).
struct Tiles {
  std::vector<BTile> all;
  Seg tgt[dk::G_TGT_CONFIGS], decide, step, trigemm, syrk, rowsum, dd, d1, dp, colnorm, triinv;
  std::vector<Seg> cdiag, cpanel, cupd, tdiag, tupd;
  std::vector<dk::PItem> pitems;  // one step of the persistent loop
  std::vector<int> pstep;         // items of problem g per step
  int max_nb = 0;
  Seg add(const std::vector<BTile>& v) {
    Seg s;
    s.off = (long)all.size();
    s.n = (int)v.size();
    all.insert(all.end(), v.begin(), v.end());
    return s;
  }
};

Tiles build_tiles(const std::vector<int>& dims, int P, int n) {
  Tiles T;
  const int G = (int)dims.size();
  std::vector<BTile> v;
  for (int c = 0; c < dk::G_TGT_CONFIGS; ++c) {
    v.clear();
    const int bm = dk::g_tgt_bm(c);
    for (int g = 0; g < G; ++g)
      for (int bx = 0; bx < cdivh(dims[g], bm); ++bx)
        for (int by = 0; by < cdivh(P, 32); ++by) v.push_back({g, bx, by});
    T.tgt[c] = T.add(v);
  }
  v.clear();
  for (int g = 0; g < G; ++g)
    for (int p = 0; p < P; ++p) v.push_back({g, 0, p});
  T.decide = T.add(v);
  v.clear();
  for (int g = 0; g < G; ++g)
    for (int ch = 0; ch < dk::step_chunks(dims[g]); ++ch)
      for (int pq = 0; pq < cdivh(P, 4); ++pq) v.push_back({g, ch, pq});
  T.step = T.add(v);
  v.clear();
  const long ncols = (long)P * n;
  for (int g = 0; g < G; ++g)
    for (int bx = 0; bx < cdivh(dims[g], 64); ++bx)
      for (int by = 0; by < cdivh(ncols, 64); ++by) v.push_back({g, bx, by});
  T.trigemm = T.add(v);
  v.clear();
  for (int g = 0; g < G; ++g) {
    const int nb = cdivh(dims[g], 64);
    for (int t = 0; t < nb * (nb + 1) / 2; ++t) v.push_back({g, t, 0});
  }
  T.syrk = T.add(v);
  v.clear();
  for (int g = 0; g < G; ++g)
    for (int bx = 0; bx < cdivh(dims[g], 64); ++bx) v.push_back({g, bx, 0});
  T.rowsum = T.add(v);
  v.clear();
  for (int g = 0; g < G; ++g)
    for (int b = 0; b < cdivh((long)dims[g] * dims[g], 256); ++b) v.push_back({g, b, 0});
  T.dd = T.add(v);
  v.clear();
  for (int g = 0; g < G; ++g)
    for (int b = 0; b < cdivh(dims[g], 256); ++b) v.push_back({g, b, 0});
  T.d1 = T.add(v);
  v.clear();
  for (int g = 0; g < G; ++g)
    for (int b = 0; b < cdivh((long)dims[g] * P, 256); ++b) v.push_back({g, b, 0});
  T.dp = T.add(v);
  v.clear();
  for (int g = 0; g < G; ++g)
    for (int p = 0; p < P; ++p) v.push_back({g, p, 0});
  T.colnorm = T.add(v);
  v.clear();
  for (int g = 0; g < G; ++g)
    for (int b = 0; b < cdivh(dims[g], NB); ++b) v.push_back({g, b, 0});
  T.triinv = T.add(v);
  for (int g = 0; g < G; ++g) T.max_nb = std::max(T.max_nb, cdivh(dims[g], NB));
  for (int jb = 0; jb < T.max_nb; ++jb) {
    std::vector<BTile> dg, pn, up, td, tu;
    for (int g = 0; g < G; ++g) {
      const int nb = cdivh(dims[g], NB);
      if (jb >= nb) continue;
      const int m = nb - jb - 1;
      dg.push_back({g, 0, 0});
      for (int i = 0; i < m; ++i) pn.push_back({g, i, 0});
      for (int t = 0; t < m * (m + 1) / 2; ++t) up.push_back({g, t, 0});
      for (int b = 0; b < cdivh(P, 64); ++b) td.push_back({g, b, 0});
      const int rem = dims[g] - std::min(dims[g], (jb + 1) * NB);
      for (int bx = 0; bx < cdivh(rem, 64); ++bx)
        for (int by = 0; by < cdivh(P, 64); ++by) tu.push_back({g, bx, by});
    }
    T.cdiag.push_back(T.add(dg));
    T.cpanel.push_back(T.add(pn));
    T.cupd.push_back(T.add(up));
    T.tdiag.push_back(T.add(td));
    T.tupd.push_back(T.add(tu));
  }
  // persistent loop: per step the target tiles of every problem (largest
  // problems first: the longest chains of dependent items start earliest),
  // then every problem's decisions, then the update chunks
  std::vector<int> order(G);
  for (int g = 0; g < G; ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return dims[x] > dims[y]; });
  const int pbm = dk::g_tgt_bm(dk::PERSIST_TGT_CFG);
  std::vector<int> ntg(G);
  T.pstep.assign(G, 0);
  for (int g : order) {
    ntg[g] = cdivh(dims[g], pbm) * cdivh(P, 32);
    for (int bx = 0; bx < cdivh(dims[g], pbm); ++bx)
      for (int by = 0; by < cdivh(P, 32); ++by) T.pitems.push_back({0, g, bx, by, 0});
  }
  // a decision item only where the update items cannot take the decision
  std::vector<int> ndec(G);
  for (int g = 0; g < G; ++g)
    ndec[g] = dk::persist_fused_decision(dims[g], cdivh(dims[g], pbm), dk::step_chunks(dims[g])) ? 0 : 1;
  for (int g : order)
    if (ndec[g]) T.pitems.push_back({1, g, 0, 0, ntg[g]});
  for (int g : order)
    for (int ch = 0; ch < dk::step_chunks(dims[g]); ++ch) T.pitems.push_back({2, g, ch, 0, ntg[g] + ndec[g]});
  for (int g = 0; g < G; ++g) T.pstep[g] = ntg[g] + ndec[g] + dk::step_chunks(dims[g]);
  return T;
}

BLay make_blay(const std::vector<int>& dims, int P, int n, long ntiles, long npitems) {
  BLay L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += a256(bytes);
    return r;
  };
  const int G = (int)dims.size();
  L.nW = 0;
  for (int g = 0; g < G; ++g) {
    L.Woff.push_back((size_t)L.nW);
    L.nW += (long)pad4(dims[g]) * P * n;
    L.nW = (L.nW + 63) / 64 * 64;  // 256-byte aligned problem slices
  }
  L.nU = (long)G * n * P;
  L.W_all = take((size_t)L.nW * 4);
  L.U_all = take((size_t)L.nU * 8);
  L.info = take((size_t)G * 4);
  L.win_ctr = take(8);
  L.N = take(8);
  L.err = take(8);
  L.probs = take(sizeof(BProb) * G);
  L.tiles = take(sizeof(BTile) * ntiles);
  L.ntiles = ntiles;
  L.pitems = take(sizeof(dk::PItem) * npitems);
  L.pstep = take(sizeof(int) * G);
  L.pctl = take(sizeof(int) * (G + 1));  // queue position, then the G counters
  for (int g = 0; g < G; ++g) {
    const size_t d = dims[g], dP = d * P, dd = d * d, win = dP * n;
    const int nch = dk::step_chunks(dims[g]);
    PLay q;
    q.X = take(dP * 8);
    q.Z = take(dP * 8);
    q.xr = take(d * 8);
    q.lp = take(2 * P * 8);
    q.zq = take(2 * P * 8);
    q.zq_part = take(2 * (size_t)nch * P * 8);
    q.lpp_part = take((size_t)cdivh(dims[g], 32) * P * 8);  // the smallest target tile has 32 rows
    q.la = take((size_t)n * P * 8);
    q.acc = take((size_t)n * P);
    q.V = take(dP * 4);
    q.Xi = take((size_t)pad4(dims[g]) * P * n * 4);
    q.win = take(win * 4);
    q.S = take(dd * 8);
    q.m = take(d * 8);
    q.L = take(dd * 8);
    q.C = take(dd * 8);
    q.Linv = take(dk::chol_scratch_bytes(dims[g]));
    q.G = take(dd * 8);
    q.h = take(d * 8);
    q.Llow = take(dd * 4);
    q.nacc = take((size_t)P * 4);
    const size_t ld = pad4(dims[g]);
    q.Rp = take(ld * ld * 4);
    q.Vp = take(ld * P * 4);
    q.Lp = take(ld * ld * 4);
    L.p.push_back(q);
  }
  L.total = o;
  return L;
}

int check_bcfg(const diam_batch_config* c, const int32_t* dims) {
  if (!c || !dims) return bfail(DIAM_E_ARG, "null config or dims");
  if (c->G < 1 || c->G > 4096) return bfail(DIAM_E_ARG, "G must lie in [1, 4096]");
  if (c->P < 1 || c->P > 4096) return bfail(DIAM_E_ARG, "P must lie in [1, 4096]");
  if (c->n_lag < 2 || (c->n_lag & 1)) return bfail(DIAM_E_ARG, "n_lag must be even and >= 2");
  if ((long)c->P * c->n_lag > 4096)
    return bfail(DIAM_E_ARG, "P * n_lag must be <= 4096 (one FP32 accumulation span of the scatter)");
  if (c->precision != DIAM_FP32) return bfail(DIAM_E_ARG, "the batched form runs DIAM_FP32 only");
  if (!(c->beta > 0.0 && c->beta <= 1.0)) return bfail(DIAM_E_ARG, "beta must lie in (0, 1]");
  if (!(c->alpha >= 1.0)) return bfail(DIAM_E_ARG, "alpha must be >= 1");
  if (!(c->jitter0 > 0.0) || c->jitter_tries < 0 || c->jitter_tries > 300)
    return bfail(DIAM_E_ARG, "jitter0 must be > 0 and 0 <= jitter_tries <= 300");
  for (int g = 0; g < c->G; ++g)
    if (dims[g] < 1 || dims[g] > 16384) return bfail(DIAM_E_ARG, "dims[%d] = %d outside [1, 16384]", g, dims[g]);
  return DIAM_OK;
}

__global__ void k_bfill_identity(double* L, int d) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < (long)d * d) L[e] = ((e % d) == (e / d)) ? 1.0 : 0.0;
}
// zero-padded copies for the target tiles: Rp (ld x ld) from R (d x d,
// row-major) and Vp (ld x P) from V (d x P)
__global__ void k_pad_rows(const float* src, int d, long ncols, int ld, float* dst, int rowmajor) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)ld * ncols) return;
  const int r = (int)(e % ld);
  const long c = e / ld;
  float v = 0.f;
  if (r < d && c < (rowmajor ? d : ncols)) v = src[r + c * d];
  dst[e] = v;
}

__global__ void k_bzero(char* p, long n) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = 0;
}

}  // namespace

struct diam_batch {
  diam_batch_config cfg;
  int G, P, n;
  std::vector<int> dims;
  hipStream_t user;   // caller's stream
  hipStream_t cs;     // private stream (graphs cannot be captured on the null stream)
  hipEvent_t ev_in, ev_out;
  char* ws;
  BLay lay;
  Tiles T;
  std::vector<BProb> hp;
  BProb* dp;
  BTile* dt;
  float* W_all;
  double* U_all;
  int* info;
  long* win_ctr;
  double* Nd;
  int* err;
  int tgt_cfg;
  double N;
  int64_t windows, steps;
  int use_graph;
  int persistent;       // the n_lag step loop as one persistent launch
  int pgrid;            // its workgroups (co-resident capacity, at most the items of one window)
  dk::PItem* pitems;
  int* pstep;
  int* pctl;
  hipGraph_t graph;
  hipGraphExec_t gexec;
  bool graph_valid;
};

static void set_nrb(diam_batch* b) {
  const int bm = dk::g_tgt_bm(b->tgt_cfg);
  for (int g = 0; g < b->G; ++g) b->hp[g].nrb = cdivh(b->dims[g], bm);
}

static int upload_probs(diam_batch* b, hipStream_t s) {
  BCHK(hipMemcpyAsync(b->dp, b->hp.data(), sizeof(BProb) * b->G, hipMemcpyHostToDevice, s));
  BCHK(hipStreamSynchronize(s));
  return DIAM_OK;
}

extern "C" int diam_batch_workspace_bytes(const diam_batch_config* cfg, const int32_t* dims, size_t* bytes) {
  int r = check_bcfg(cfg, dims);
  if (r) return r;
  if (!bytes) return bfail(DIAM_E_ARG, "null bytes");
  std::vector<int> dv(dims, dims + cfg->G);
  Tiles T = build_tiles(dv, cfg->P, cfg->n_lag);
  *bytes = make_blay(dv, cfg->P, cfg->n_lag, (long)T.all.size(), (long)T.pitems.size()).total;
  return DIAM_OK;
}

extern "C" int diam_batch_init(diam_batch** out, const diam_batch_config* cfg, const int32_t* dims,
                               const double* const* mu, const float* const* R, void* workspace, size_t ws_bytes,
                               const double* const* x0, void* hip_stream) {
  if (!out) return bfail(DIAM_E_ARG, "null out");
  *out = nullptr;
  int r = check_bcfg(cfg, dims);
  if (r) return r;
  if (!mu || !R || !x0) return bfail(DIAM_E_ARG, "null target or start arrays");
  for (int g = 0; g < cfg->G; ++g)
    if (!mu[g] || !R[g] || !x0[g]) return bfail(DIAM_E_ARG, "problem %d: null mu, R or x0", g);
  for (int g = 0; g < cfg->G; ++g)
    if ((uintptr_t)mu[g] % 16 || (uintptr_t)R[g] % 16) return bfail(DIAM_E_ARG, "problem %d: mu, R not 16-byte aligned", g);
  if (!workspace || ((uintptr_t)workspace & 255)) return bfail(DIAM_E_ARG, "workspace null or not 256-byte aligned");
  std::vector<int> dv(dims, dims + cfg->G);
  Tiles T = build_tiles(dv, cfg->P, cfg->n_lag);
  BLay L = make_blay(dv, cfg->P, cfg->n_lag, (long)T.all.size(), (long)T.pitems.size());
  if (ws_bytes < L.total) return bfail(DIAM_E_ARG, "workspace too small: %zu < %zu", ws_bytes, L.total);

  diam_batch* b = new (std::nothrow) diam_batch();
  if (!b) return bfail(DIAM_E_ARG, "out of host memory");
  b->cfg = *cfg;
  b->G = cfg->G;
  b->P = cfg->P;
  b->n = cfg->n_lag;
  b->dims = dv;
  b->user = (hipStream_t)hip_stream;
  b->ws = (char*)workspace;
  b->lay = L;
  b->T = T;
  b->tgt_cfg = 2;  // 64-row tiles, two k-groups: the single-problem kernel's shape
  b->N = 0.0;
  b->windows = b->steps = 0;
  b->use_graph = 1;
  b->graph = nullptr;
  b->gexec = nullptr;
  b->graph_valid = false;
  auto fail_init = [&](hipError_t e, const char* what) {
    if (b->cs) (void)hipStreamDestroy(b->cs);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    delete b;
    return bfail(DIAM_E_HIP, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e = hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking);
  if (e != hipSuccess) return fail_init(e, "hipStreamCreateWithFlags");
  e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e != hipSuccess) return fail_init(e, "hipEventCreate");
  e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e != hipSuccess) return fail_init(e, "hipEventCreate");

  char* w = b->ws;
  b->W_all = (float*)(w + L.W_all);
  b->U_all = (double*)(w + L.U_all);
  b->info = (int*)(w + L.info);
  b->win_ctr = (long*)(w + L.win_ctr);
  b->Nd = (double*)(w + L.N);
  b->err = (int*)(w + L.err);
  b->dp = (BProb*)(w + L.probs);
  b->dt = (BTile*)(w + L.tiles);
  b->pitems = (dk::PItem*)(w + L.pitems);
  b->pstep = (int*)(w + L.pstep);
  b->pctl = (int*)(w + L.pctl);
  b->persistent = 0;
  {
    int ncu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || ncu < 1)
      ncu = 1;
    const long cap = (long)dk::g_persist_blocks_per_cu() * ncu;
    const long items = (long)T.pitems.size() * cfg->n_lag;
    b->pgrid = (int)std::max(1L, std::min(cap, items));
  }
  b->hp.resize(b->G);
  for (int g = 0; g < b->G; ++g) {
    const PLay& q = L.p[g];
    BProb& p = b->hp[g];
    p.d = dv[g];
    p.nch = dk::step_chunks(dv[g]);
    p.nb = cdivh(dv[g], NB);
    p.R = R[g];
    p.mu = mu[g];
    p.X = (double*)(w + q.X);
    p.Z = (double*)(w + q.Z);
    p.xr = (double*)(w + q.xr);
    p.lp = (double*)(w + q.lp);
    p.zq = (double*)(w + q.zq);
    p.zq_part = (double*)(w + q.zq_part);
    p.lpp_part = (double*)(w + q.lpp_part);
    p.la = (double*)(w + q.la);
    p.acc = (uint8_t*)(w + q.acc);
    p.V = (float*)(w + q.V);
    p.W = b->W_all + L.Woff[g];
    p.Xi = (float*)(w + q.Xi);
    p.win = (float*)(w + q.win);
    p.S = (double*)(w + q.S);
    p.m = (double*)(w + q.m);
    p.L = (double*)(w + q.L);
    p.C = (double*)(w + q.C);
    p.Linv = (double*)(w + q.Linv);
    p.G = (double*)(w + q.G);
    p.h = (double*)(w + q.h);
    p.Llow = (float*)(w + q.Llow);
    p.nacc = (int*)(w + q.nacc);
    p.info = b->info + g;
    p.ld = pad4(dv[g]);
    p.Rp = (const float*)(w + q.Rp);
    p.Vp = (float*)(w + q.Vp);
    p.Lp = (float*)(w + q.Lp);
  }
  set_nrb(b);
  hipStream_t s = b->user;
#define BCHK_INIT(expr)                           \
  do {                                            \
    hipError_t _e = (expr);                       \
    if (_e != hipSuccess) return fail_init(_e, #expr); \
  } while (0)
  BCHK_INIT(hipMemcpyAsync(b->dt, T.all.data(), sizeof(BTile) * T.all.size(), hipMemcpyHostToDevice, s));
  BCHK_INIT(hipMemcpyAsync(b->pitems, T.pitems.data(), sizeof(dk::PItem) * T.pitems.size(), hipMemcpyHostToDevice, s));
  BCHK_INIT(hipMemcpyAsync(b->pstep, T.pstep.data(), sizeof(int) * T.pstep.size(), hipMemcpyHostToDevice, s));
  BCHK_INIT(hipMemcpyAsync(b->dp, b->hp.data(), sizeof(BProb) * b->G, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_bzero, dim3(1), dim3(256), 0, s, (char*)b->win_ctr, 8L);
  hipLaunchKernelGGL(k_bzero, dim3(1), dim3(256), 0, s, (char*)b->Nd, 8L);
  hipLaunchKernelGGL(k_bzero, dim3(1), dim3(256), 0, s, (char*)b->err, 8L);
  // initial state of every problem: A = I, x_ref = 0, empty moments, log pi(x0)
  for (int g = 0; g < b->G; ++g) {
    const BProb& p = b->hp[g];
    const int d = p.d, P = b->P;
    const long dP = (long)d * P, dd = (long)d * d;
    BCHK_INIT(hipMemcpyAsync(p.X, x0[g], dP * 8, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_bfill_identity, dim3(cdivh(dd, 256)), dim3(256), 0, s, p.L, d);
    hipLaunchKernelGGL(k_bzero, dim3(cdivh(d * 8, 256)), dim3(256), 0, s, (char*)p.xr, (long)d * 8);
    hipLaunchKernelGGL(k_bzero, dim3(cdivh(dd * 8, 256)), dim3(256), 0, s, (char*)p.S, dd * 8);
    hipLaunchKernelGGL(k_bzero, dim3(cdivh(d * 8, 256)), dim3(256), 0, s, (char*)p.m, (long)d * 8);
    hipLaunchKernelGGL(k_bzero, dim3(cdivh(P * 4, 256)), dim3(256), 0, s, (char*)p.nacc, (long)P * 4);
    BCHK_INIT(dk::round_factor(dk::P32, p.L, p.Llow, d, s));
    hipLaunchKernelGGL(k_pad_rows, dim3(cdivh((long)p.ld * p.ld, 256)), dim3(256), 0, s, (const float*)p.Llow, d,
                       (long)p.ld, p.ld, p.Lp, 1);
    BCHK_INIT(dk::init_eval(0, p.X, p.mu, p.V, p.Z, d, P, s));
    {
      const long nr = (long)p.ld * p.ld, nv = (long)p.ld * P;
      // row-major R: element (i, k) at i d + k -> treat as column k' = i of length d
      hipLaunchKernelGGL(k_pad_rows, dim3(cdivh(nr, 256)), dim3(256), 0, s, p.R, d, (long)p.ld, p.ld, (float*)p.Rp,
                         1);
      hipLaunchKernelGGL(k_pad_rows, dim3(cdivh(nv, 256)), dim3(256), 0, s, (const float*)p.V, d, (long)P, p.ld,
                         p.Vp, 0);
      BCHK_INIT(hipGetLastError());
    }
    BCHK_INIT(dk::tgt_gauss(dk::P32, p.R, p.V, d, P, p.lpp_part, s));
    BCHK_INIT(dk::init_finish(p.lpp_part, dk::tgt_row_blocks(d), p.Z, p.X, 0.0, p.lp, p.zq, d, P, s));
  }
  BCHK_INIT(hipStreamSynchronize(s));
#undef BCHK_INIT
  *out = b;
  return DIAM_OK;
}

// Refactorise every problem whose Cholesky status is nonzero, with the jitter
// rule, eagerly on the private stream; jitter (host, G) gets the levels.
static int retry_failed(diam_batch* b, int32_t* jitter, int* any_fail) {
  hipStream_t s = b->cs;
  std::vector<int> info(b->G);
  BCHK(hipMemcpyAsync(info.data(), b->info, sizeof(int) * b->G, hipMemcpyDeviceToHost, s));
  BCHK(hipStreamSynchronize(s));
  *any_fail = 0;
  double* tr_dev = b->hp[0].h;  // reuse: the row sums are dead after the fold
  for (int g = 0; g < b->G; ++g) {
    int j = -1;
    if (info[g] != 0) {
      const BProb& p = b->hp[g];
      const int d = p.d;
      tr_dev = p.h;
      BCHK(dk::cov_assemble(p.S, p.m, 0.0, p.C, tr_dev, d, s));
      double tr = 0.0;
      BCHK(hipMemcpyAsync(&tr, tr_dev, 8, hipMemcpyDeviceToHost, s));
      BCHK(hipStreamSynchronize(s));
      tr /= d;
      const double sc = (tr > 0.0 && isfinite(tr)) ? tr : 1.0;
      j = b->cfg.jitter_tries;
      for (int q = 0; q < b->cfg.jitter_tries; ++q) {
        const double eps = pow(10.0, q) * b->cfg.jitter0 * sc;
        int zero = 0;
        BCHK(hipMemcpyAsync(p.info, &zero, sizeof(int), hipMemcpyHostToDevice, s));
        BCHK(dk::cov_assemble(p.S, p.m, eps, p.C, nullptr, d, s));
        BCHK(dk::potrf(p.C, d, p.info, p.Linv, s));
        int st = 0;
        BCHK(hipMemcpyAsync(&st, p.info, sizeof(int), hipMemcpyDeviceToHost, s));
        BCHK(hipStreamSynchronize(s));
        if (st == 0) {
          j = q;
          break;
        }
      }
      if (j < b->cfg.jitter_tries) {
        BCHK(hipMemcpyAsync(p.L, p.C, (size_t)d * d * 8, hipMemcpyDeviceToDevice, s));
        BCHK(dk::round_factor(dk::P32, p.L, p.Llow, d, s));
        hipLaunchKernelGGL(k_pad_rows, dim3(cdivh((long)p.ld * p.ld, 256)), dim3(256), 0, s, (const float*)p.Llow, d,
                           (long)p.ld, p.ld, p.Lp, 1);
        BCHK(hipGetLastError());
        BCHK(hipMemcpyAsync(p.xr, p.m, (size_t)d * 8, hipMemcpyDeviceToDevice, s));
        BCHK(dk::trsm_whiten(p.L, p.X, p.xr, p.Z, p.zq, p.Linv, d, b->P, s));
      } else {
        *any_fail = 1;
      }
    }
    if (jitter) jitter[g] = j;
  }
  return DIAM_OK;
}

// Polls of a wait in the persistent loop before it gives up (a few seconds;
// a legitimate wait lasts well under a millisecond).
constexpr int PERSIST_SPIN_MAX = 4000000;

// One window of every problem on stream s (eager, or while capturing).
static int enqueue_window(diam_batch* b, hipStream_t s) {
  const int P = b->P, n = b->n;
  const long K = (long)P * n;
  const double beta = b->cfg.beta, alpha = b->cfg.alpha;
  const Tiles& T = b->T;
  auto tl = [&](const Seg& g) { return (const BTile*)(b->dt + g.off); };
  BCHK(dk::g_rng(b->cfg.seed, b->win_ctr, b->lay.nW, b->lay.nU, P, b->W_all, b->U_all, s));
  BCHK(dk::g_trigemm(b->dp, tl(T.trigemm), T.trigemm.n, (int)K, beta * alpha, s));
  dk::BStep st;
  st.n = n;
  st.P = P;
  st.rho = sqrt(1.0 - beta * beta);
  st.c = beta * alpha;
  st.inv2a2 = 1.0 / (2.0 * alpha * alpha);
  st.U = b->U_all;
  st.err = b->err;
  st.t = -1;
  BCHK(dk::g_step(b->dp, tl(T.decide), T.decide.n, tl(T.step), T.step.n, st, s));
  if (b->persistent) {
    // the n_lag steps of every problem: one launch over the item queue
    hipLaunchKernelGGL(k_bzero, dim3(cdivh((long)(b->G + 1) * 4, 256)), dim3(256), 0, s, (char*)b->pctl,
                       (long)(b->G + 1) * 4);
    BCHK(hipGetLastError());
    dk::PCtl ctl;
    ctl.qctr = b->pctl;
    ctl.done = b->pctl + 1;
    ctl.per_step = b->pstep;
    ctl.err = b->err;
    ctl.spin_max = PERSIST_SPIN_MAX;
    BCHK(dk::g_persist(b->dp, b->pitems, (int)T.pitems.size(), st, ctl, b->pgrid, s));
  } else {
    const Seg& tg = T.tgt[b->tgt_cfg];
    for (int t = 0; t < n; ++t) {
      BCHK(dk::g_tgt(b->tgt_cfg, b->dp, tl(tg), tg.n, P, s));
      st.t = t;
      BCHK(dk::g_step(b->dp, tl(T.decide), T.decide.n, tl(T.step), T.step.n, st, s));
    }
  }
  BCHK(dk::g_scatter(b->dp, tl(T.syrk), T.syrk.n, tl(T.rowsum), T.rowsum.n, (int)K, s));
  BCHK(dk::g_fold(b->dp, tl(T.dd), T.dd.n, tl(T.d1), T.d1.n, b->Nd, (double)K, s));
  BCHK(dk::g_bump(b->win_ctr, b->Nd, (double)K, s));
  BCHK(dk::g_cov(b->dp, tl(T.dd), T.dd.n, s));
  for (int jb = 0; jb < T.max_nb; ++jb)
    BCHK(dk::g_chol_step(b->dp, tl(T.cdiag[jb]), T.cdiag[jb].n, tl(T.cpanel[jb]), T.cpanel[jb].n, tl(T.cupd[jb]),
                         T.cupd[jb].n, jb, s));
  BCHK(dk::g_adopt(b->dp, tl(T.dd), T.dd.n, s));
  BCHK(dk::g_sub_ref(b->dp, tl(T.dp), T.dp.n, P, s));
  BCHK(dk::g_tri_inv(b->dp, tl(T.triinv), T.triinv.n, s));
  for (int jb = 0; jb < T.max_nb; ++jb)
    BCHK(dk::g_trsm_step(b->dp, tl(T.tdiag[jb]), T.tdiag[jb].n, tl(T.tupd[jb]), T.tupd[jb].n, jb, P, s));
  BCHK(dk::g_colnorm(b->dp, tl(T.colnorm), T.colnorm.n, s));
  return DIAM_OK;
}

static void drop_graph(diam_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->graph_valid = false;
}

static int capture(diam_batch* b) {
  drop_graph(b);
  BCHK(hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal));
  int r = enqueue_window(b, b->cs);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cs, &g);
  if (r) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (e != hipSuccess) return bfail(DIAM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  b->graph = g;
  e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return bfail(DIAM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  b->graph_valid = true;
  return DIAM_OK;
}

extern "C" int diam_batch_window(diam_batch* b, int32_t* jitter) {
  if (!b) return bfail(DIAM_E_ARG, "null batch");
  BCHK(hipEventRecord(b->ev_in, b->user));
  BCHK(hipStreamWaitEvent(b->cs, b->ev_in, 0));
  if (b->use_graph) {
    if (!b->graph_valid) {
      int r = capture(b);
      if (r) return r;
    }
    BCHK(hipGraphLaunch(b->gexec, b->cs));
  } else {
    int r = enqueue_window(b, b->cs);
    if (r) return r;
  }
  int any = 0;
  int r = retry_failed(b, jitter, &any);
  if (r) return r;
  int err = 0;
  BCHK(hipMemcpyAsync(&err, b->err, sizeof(int), hipMemcpyDeviceToHost, b->cs));
  BCHK(hipStreamSynchronize(b->cs));
  BCHK(hipEventRecord(b->ev_out, b->cs));
  BCHK(hipStreamWaitEvent(b->user, b->ev_out, 0));
  b->N += (double)b->P * b->n;
  b->windows += 1;
  b->steps += b->n;
  if (err) {
    hipLaunchKernelGGL(k_bzero, dim3(1), dim3(256), 0, b->cs, (char*)b->err, 8L);
    BCHK(hipStreamSynchronize(b->cs));
    if (err & 2) return bfail(DIAM_E_HIP, "the persistent step loop gave up waiting for an item (window lost)");
    return bfail(DIAM_E_TARGET, "a target log density returned +inf");
  }
  if (any) return bfail(DIAM_E_NOT_PD, "a covariance was not positive definite at any jitter level");
  return DIAM_OK;
}

extern "C" int diam_batch_seed_moments(diam_batch* b, const double* const* S0, const double* const* m0, double N0,
                                       int32_t* jitter) {
  if (!b || !S0 || !m0) return bfail(DIAM_E_ARG, "null argument");
  if (!(N0 >= 0.0)) return bfail(DIAM_E_ARG, "N0 must be >= 0");
  for (int g = 0; g < b->G; ++g)
    if (!S0[g] || !m0[g]) return bfail(DIAM_E_ARG, "problem %d: null S0 or m0", g);
  BCHK(hipEventRecord(b->ev_in, b->user));
  BCHK(hipStreamWaitEvent(b->cs, b->ev_in, 0));
  hipStream_t s = b->cs;
  for (int g = 0; g < b->G; ++g) {
    const BProb& p = b->hp[g];
    BCHK(hipMemcpyAsync(p.S, S0[g], (size_t)p.d * p.d * 8, hipMemcpyDeviceToDevice, s));
    BCHK(hipMemcpyAsync(p.m, m0[g], (size_t)p.d * 8, hipMemcpyDeviceToDevice, s));
  }
  BCHK(hipMemcpyAsync(b->Nd, &N0, 8, hipMemcpyHostToDevice, s));
  b->N = N0;
  // the window's update sequence, eagerly: covariance, Cholesky, adoption, whitening
  const Tiles& T = b->T;
  auto tl = [&](const Seg& g) { return (const BTile*)(b->dt + g.off); };
  BCHK(dk::g_cov(b->dp, tl(T.dd), T.dd.n, s));
  for (int jb = 0; jb < T.max_nb; ++jb)
    BCHK(dk::g_chol_step(b->dp, tl(T.cdiag[jb]), T.cdiag[jb].n, tl(T.cpanel[jb]), T.cpanel[jb].n, tl(T.cupd[jb]),
                         T.cupd[jb].n, jb, s));
  BCHK(dk::g_adopt(b->dp, tl(T.dd), T.dd.n, s));
  BCHK(dk::g_sub_ref(b->dp, tl(T.dp), T.dp.n, b->P, s));
  BCHK(dk::g_tri_inv(b->dp, tl(T.triinv), T.triinv.n, s));
  for (int jb = 0; jb < T.max_nb; ++jb)
    BCHK(dk::g_trsm_step(b->dp, tl(T.tdiag[jb]), T.tdiag[jb].n, tl(T.tupd[jb]), T.tupd[jb].n, jb, b->P, s));
  BCHK(dk::g_colnorm(b->dp, tl(T.colnorm), T.colnorm.n, s));
  int any = 0;
  int r = retry_failed(b, jitter, &any);
  if (r) return r;
  BCHK(hipEventRecord(b->ev_out, b->cs));
  BCHK(hipStreamWaitEvent(b->user, b->ev_out, 0));
  if (any) return bfail(DIAM_E_NOT_PD, "a seeded covariance was not positive definite at any jitter level");
  return DIAM_OK;
}

extern "C" int diam_batch_set_tiles(diam_batch* b, int32_t choice) {
  if (!b) return bfail(DIAM_E_ARG, "null batch");
  if (choice < 0 || choice >= dk::G_TGT_CONFIGS) return bfail(DIAM_E_ARG, "tile choice %d out of range", choice);
  if (choice == b->tgt_cfg) return DIAM_OK;
  if (b->persistent) return bfail(DIAM_E_STATE, "the persistent loop runs its own tile shape");
  BCHK(hipStreamSynchronize(b->cs));
  b->tgt_cfg = choice;
  set_nrb(b);
  int r = upload_probs(b, b->cs);
  if (r) return r;
  drop_graph(b);
  return DIAM_OK;
}

extern "C" int diam_batch_set_persistent(diam_batch* b, int32_t on) {
  if (!b) return bfail(DIAM_E_ARG, "null batch");
  if (on) {
    for (int g = 0; g < b->G; ++g)
      if (b->dims[g] > 4096)
        return bfail(DIAM_E_ARG, "the persistent loop takes d <= 4096 (problem %d has d = %d)", g, b->dims[g]);
    if (b->tgt_cfg != dk::PERSIST_TGT_CFG) {
      BCHK(hipStreamSynchronize(b->cs));
      b->tgt_cfg = dk::PERSIST_TGT_CFG;
      set_nrb(b);
      int r = upload_probs(b, b->cs);
      if (r) return r;
    }
  }
  if ((on ? 1 : 0) != b->persistent) drop_graph(b);
  b->persistent = on ? 1 : 0;
  return DIAM_OK;
}

extern "C" int diam_batch_set_graph(diam_batch* b, int32_t on) {
  if (!b) return bfail(DIAM_E_ARG, "null batch");
  b->use_graph = on ? 1 : 0;
  if (!on) drop_graph(b);
  return DIAM_OK;
}

// Times every target tile shape on the batch's own problems (reps launches
// each, after two untimed ones) and keeps the fastest.  The launches only
// overwrite the target partial sums, which the next step recomputes.
extern "C" int diam_batch_autotune(diam_batch* b, int32_t reps, int32_t* choice, double* us) {
  if (!b) return bfail(DIAM_E_ARG, "null batch");
  if (reps < 1 || reps > 10000) return bfail(DIAM_E_ARG, "reps must lie in [1, 10000]");
  if (b->persistent) return bfail(DIAM_E_STATE, "the persistent loop runs its own tile shape");
  hipStream_t s = b->cs;
  BCHK(hipEventRecord(b->ev_in, b->user));
  BCHK(hipStreamWaitEvent(s, b->ev_in, 0));
  hipEvent_t e0, e1;
  BCHK(hipEventCreate(&e0));
  BCHK(hipEventCreate(&e1));
  const int saved = b->tgt_cfg;
  int best = saved;
  double best_us = 1e300;
  int rc = DIAM_OK;
  for (int c = 0; c < dk::G_TGT_CONFIGS && rc == DIAM_OK; ++c) {
    b->tgt_cfg = c;
    set_nrb(b);
    if ((rc = upload_probs(b, s))) break;
    const Seg& tg = b->T.tgt[c];
    const BTile* tl = b->dt + tg.off;
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = dk::g_tgt(c, b->dp, tl, tg.n, b->P, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = dk::g_tgt(c, b->dp, tl, tg.n, b->P, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      rc = bfail(DIAM_E_HIP, "autotune: %s", hipGetErrorString(e));
      break;
    }
    const double t = 1e3 * ms / reps;
    if (us) us[c] = t;
    if (t < best_us) {
      best_us = t;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->tgt_cfg = best;
  set_nrb(b);
  int r2 = upload_probs(b, s);
  if (rc) return rc;
  if (r2) return r2;
  if (best != saved) drop_graph(b);
  if (choice) *choice = best;
  return DIAM_OK;
}

static int bfield(diam_batch* b, int32_t g, int32_t f, const void** src, size_t* bytes) {
  if (g < 0 || g >= b->G) return bfail(DIAM_E_ARG, "problem %d out of range", g);
  const BProb& p = b->hp[g];
  const size_t d = p.d, P = b->P, n = b->n;
  switch (f) {
    case DIAM_F_X: *src = p.X; *bytes = d * P * 8; break;
    case DIAM_F_Z: *src = p.Z; *bytes = d * P * 8; break;
    case DIAM_F_LOGP: *src = p.lp; *bytes = P * 8; break;   // window boundaries: parity 0
    case DIAM_F_ZQ: *src = p.zq; *bytes = P * 8; break;
    case DIAM_F_XREF: *src = p.xr; *bytes = d * 8; break;
    case DIAM_F_L: *src = p.L; *bytes = d * d * 8; break;
    case DIAM_F_S: *src = p.S; *bytes = d * d * 8; break;
    case DIAM_F_M: *src = p.m; *bytes = d * 8; break;
    case DIAM_F_LA: *src = p.la; *bytes = n * P * 8; break;
    case DIAM_F_ACC: *src = p.acc; *bytes = n * P; break;
    case DIAM_F_NACC: *src = p.nacc; *bytes = P * 4; break;
    case DIAM_F_W: *src = p.W; *bytes = (size_t)p.ld * P * n * 4; break;  // rows padded to ld
    case DIAM_F_U: *src = b->U_all + (long)g * n * P; *bytes = n * P * 8; break;
    default: return bfail(DIAM_E_ARG, "field %d is not kept by the batched form", f);
  }
  return DIAM_OK;
}

extern "C" int diam_batch_field_bytes(diam_batch* b, int32_t g, int32_t field, size_t* bytes) {
  if (!b || !bytes) return bfail(DIAM_E_ARG, "null argument");
  const void* src;
  return bfield(b, g, field, &src, bytes);
}

extern "C" int diam_batch_get(diam_batch* b, int32_t g, int32_t field, void* dst, size_t bytes) {
  if (!b || !dst) return bfail(DIAM_E_ARG, "null argument");
  const void* src;
  size_t n;
  int r = bfield(b, g, field, &src, &n);
  if (r) return r;
  if (bytes != n) return bfail(DIAM_E_ARG, "field %d of problem %d has %zu bytes, got %zu", field, g, n, bytes);
  BCHK(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, b->user));
  return DIAM_OK;
}

extern "C" int diam_batch_get_stats(diam_batch* b, diam_stats* out) {
  if (!b || !out) return bfail(DIAM_E_ARG, "null argument");
  out->steps = b->steps;
  out->steps_in_window = 0;
  out->last_jitter = -1;
  out->n_samples = b->N;
  out->windows = b->windows;
  out->last_call_steps = b->n;
  out->beta = b->cfg.beta;
  return DIAM_OK;
}

extern "C" void diam_batch_destroy(diam_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->cs);
  drop_graph(b);
  (void)hipStreamDestroy(b->cs);
  (void)hipEventDestroy(b->ev_in);
  (void)hipEventDestroy(b->ev_out);
  delete b;
}
