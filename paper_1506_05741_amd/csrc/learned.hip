// Learned-part form: Bayesian logistic-regression target, the MLP surrogate
// of log pi (forward, backward, Adam; all on FP32 MFMA) and the kernels of
// two-stage delayed acceptance (Christen & Fox 2005): surrogate screen,
// survivor compaction, exact target on the survivors only.
#include <math.h>

#include "gemm.h"
#include "kernels.h"

using namespace gemm;

namespace dk {

// ============================================================================
// Logistic target: T = A X' (n_obs x d by d x P) on FP32 MFMA, then per
// element y t - softplus(t) and FP64 sums over 64-row blocks:
//   part[p][rb] = sum_{j in rb} [ y_j t_jp - softplus(t_jp) ]   (chain-major)
// Columns p >= *nact are skipped (their tiles exit at once).  Workgroup ids
// are dealt round-robin to the 8 XCDs; the column tiles of one row block are
// given consecutive ids on one XCD so that its rows of A are fetched once.
// ============================================================================
DEV float softplus_f(float t) { return fmaxf(t, 0.f) + log1pf(expf(-fabsf(t))); }

template <int BN>
__global__ __launch_bounds__(512) void k_tgt_logreg(const float* __restrict__ A, const float* __restrict__ y, int n_obs,
                                                    const float* __restrict__ V, int d, int P,
                                                    const int* __restrict__ nact_ptr, int nrb, int nct,
                                                    double* __restrict__ part) {
  constexpr int BM = 64, BK = 32, KG = 2;
  __shared__ float lds[KG * e_lds_elems<float, BM, BN, BK>()];
  __shared__ double red[2][BN];
  const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
  const int rb = (k / nct) * 8 + xcd, ct = k % nct;
  const int nact = nact_ptr ? *nact_ptr : P;
  const int i0 = rb * BM, j0 = ct * BN;
  if (rb >= nrb || j0 >= nact) return;  // uniform per workgroup, before any barrier
  EFrag<float, BM, BN> f;
  f.zero();
  // V always holds P columns (under delayed acceptance the survivors packed
  // first, the rest stale but readable), so the loads are bounded by P and a
  // partly filled last tile keeps the unguarded vector path; only columns
  // below nact are written
  e_gemm<float, BM, BN, BK, true, true, KG>(f, A, d, n_obs, V, d, P, i0, j0, 0, d, lds);
  const bool g0 = threadIdx.x < NT;
  const int lane = threadIdx.x & 63, w = (threadIdx.x & (NT - 1)) >> 6, wm = w & 1, wn = w >> 1;
  if (g0) {
#pragma unroll
    for (int n = 0; n < EFrag<float, BM, BN>::FN; ++n) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < EFrag<float, BM, BN>::FM; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int ti, tj;
          frag_coords<BM, BN>(m, n, r, ti, tj);
          const int i = i0 + ti;
          if (i < n_obs) {
            const float t = f.c[m][n][r];
            s += (double)(y[i] * t - softplus_f(t));
          }
        }
      s += lane_xor_f64<16>(s);
      s += lane_xor_f64<32>(s);
      if (lane < 16) red[wm][wn * (BN / 2) + n * 16 + lane] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < BN) {
    const int j = j0 + threadIdx.x;
    if (j < nact) part[(long)j * nrb + rb] = red[0][threadIdx.x] + red[1][threadIdx.x];
  }
}

int logreg_row_blocks(long n_obs) { return (int)((n_obs + 63) / 64); }

// Column tiles of 64 chains; under delayed acceptance (nact set) the tiles
// past the survivor count exit at once.  (32-chain tiles were measured 1.5x
// less efficient per chain, more than their finer granularity saves.)
hipError_t tgt_logreg(const float* A, const float* y, long n_obs, const float* V, int d, int P, const int* nact,
                      double* part, hipStream_t s) {
  const int nrb = logreg_row_blocks(n_obs), groups = (nrb + 7) / 8;
  const int nct = cdiv(P, 64);
  hipLaunchKernelGGL(k_tgt_logreg<64>, dim3(groups * 8 * nct), dim3(512), 0, s, A, y, (int)n_obs, V, d, P, nact, nrb,
                     nct, part);
  return hipGetLastError();
}

// ============================================================================
// MLP surrogate: s(x) = out_std * (W3 h2 + b3) + out_mean,
// h2 = gelu(W2 h1 + b2), h1 = gelu(W1 xs + b1), xs = (x - in_mean) * in_scale.
// Weights used in the forward pass are the bf16 roundings of the FP32 master
// weights (stored as FP32 values); Adam updates the masters.  Activations
// are column-major: column s is sample s.
// ============================================================================
DEV float gelu_f(float a) { return a * 0.5f * (1.f + erff(a * 0.70710678118654752f)); }
DEV float gelu_grad_f(float a) {
  return 0.5f * (1.f + erff(a * 0.70710678118654752f)) + a * 0.39894228040143268f * expf(-0.5f * a * a);
}

// C(m, n) = sum_k A(m, k) B(n, k) with the engine's (row, k) operand
// description, then one of three epilogues:
//   EPI 0: out[m * ldc + n] = C                       (weight gradients, row-major)
//   EPI 1: a[m + n * ldc] = C + bias[m]; h = gelu(a)    (forward layer)
//   EPI 2: out[m + n * ldc] = C * gelu'(aux[m + n*ldc]) (back through GELU)
template <bool AKC, bool BKC, int EPI>
__global__ __launch_bounds__(256) void k_mlp_gemm(const float* __restrict__ A, int lda, int M, const float* __restrict__ B,
                                                  int ldb, int N, int K, float* __restrict__ out, int ldc,
                                                  const float* __restrict__ bias, const float* __restrict__ aux,
                                                  float* __restrict__ out2) {
  constexpr int BM = 64, BN = 64, BK = 32;
  __shared__ float lds[e_lds_elems<float, BM, BN, BK>()];
  const int i0 = blockIdx.x * BM, j0 = blockIdx.y * BN;
  EFrag<float, BM, BN> f;
  f.zero();
  e_gemm<float, BM, BN, BK, AKC, BKC>(f, A, lda, M, B, ldb, N, i0, j0, 0, K, lds);
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ti, tj;
        frag_coords<BM, BN>(m, n, r, ti, tj);
        const int i = i0 + ti, j = j0 + tj;
        if (i >= M || j >= N) continue;
        const float c = f.c[m][n][r];
        if (EPI == 0) {
          out[(long)i * ldc + j] = c;
        } else if (EPI == 1) {
          const float a = c + bias[i];
          out[i + (long)j * ldc] = a;
          out2[i + (long)j * ldc] = gelu_f(a);
        } else {
          out[i + (long)j * ldc] = c * gelu_grad_f(aux[i + (long)j * ldc]);
        }
      }
}

// out[s] = sum_o w3[o] h2[o, s] + b3 (one wavefront per sample)
__global__ __launch_bounds__(256) void k_mlp_out(const float* __restrict__ w3, const float* __restrict__ b3,
                                                 const float* __restrict__ h2, int H, int n, float* __restrict__ out) {
  const int lane = threadIdx.x & 63, s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= n) return;
  float acc = 0.f;
  for (int o = lane; o < H; o += 64) acc = fmaf(w3[o], h2[o + (long)s * H], acc);
  acc = wave_sum_f32(acc);
  if (lane == 0) out[s] = acc + b3[0];
}

// xs[:, s] = (x_s - in_mean) * in_scale from FP64 (X64) or FP32 (X32) states
__global__ __launch_bounds__(256) void k_mlp_standardize(const double* __restrict__ X64, const float* __restrict__ X32,
                                                         const float* __restrict__ in_mean,
                                                         const float* __restrict__ in_scale, int D, long n,
                                                         float* __restrict__ xs) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)D * n) return;
  const int i = (int)(e % D);
  const float x = X64 ? (float)X64[e] : X32[e];
  xs[e] = (x - in_mean[i]) * in_scale[i];
}

// surrogate log density (FP64) from the FP32 network output
__global__ __launch_bounds__(256) void k_mlp_denorm(const float* __restrict__ out, const float* __restrict__ stats, int n,
                                                    double* __restrict__ s_out) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < n) s_out[e] = (double)out[e] * (double)stats[1] + (double)stats[0];
}

// per-coordinate mean and 1/std over n samples (FP64 inputs, column-major d x n)
__global__ __launch_bounds__(256) void k_mlp_in_stats(const double* __restrict__ X, int d, long n,
                                                      float* __restrict__ in_mean, float* __restrict__ in_scale) {
  __shared__ double red[2][256];
  const int i = blockIdx.x;
  double s = 0.0, q = 0.0;
  for (long k = threadIdx.x; k < n; k += 256) {
    const double x = X[i + k * d];
    s += x;
    q = __fma_rn(x, x, q);
  }
  red[0][threadIdx.x] = s;
  red[1][threadIdx.x] = q;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mean = red[0][0] / n;
    const double var = fmax(red[1][0] / n - mean * mean, 0.0);
    in_mean[i] = (float)mean;
    in_scale[i] = (float)(1.0 / fmax(sqrt(var), 1e-12));
  }
}

// stats[0] = mean, stats[1] = std of the n log densities; ts = standardised
__global__ __launch_bounds__(256) void k_mlp_out_stats(const double* __restrict__ lp, long n, float* __restrict__ stats,
                                                       float* __restrict__ ts) {
  __shared__ double red[2][256];
  __shared__ double mean_s, std_s;
  double s = 0.0, q = 0.0;
  for (long k = threadIdx.x; k < n; k += 256) {
    s += lp[k];
    q = __fma_rn(lp[k], lp[k], q);
  }
  red[0][threadIdx.x] = s;
  red[1][threadIdx.x] = q;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mean = red[0][0] / n;
    mean_s = mean;
    std_s = fmax(sqrt(fmax(red[1][0] / n - mean * mean, 0.0)), 1e-12);
    stats[0] = (float)mean;
    stats[1] = (float)std_s;
  }
  __syncthreads();
  for (long k = threadIdx.x; k < n; k += 256) ts[k] = (float)((lp[k] - mean_s) / std_s);
}

// He-normal init of the master weights from Philox (biases zero)
__global__ __launch_bounds__(256) void k_mlp_init(uint32_t k0, uint32_t k1, int D, int H, float* __restrict__ master,
                                                  float* __restrict__ eff, long nparam) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= nparam) return;
  const long oW1 = 0, ob1 = (long)H * D, oW2 = ob1 + H, ob2 = oW2 + (long)H * H, oW3 = ob2 + H, ob3 = oW3 + H;
  float scale = 0.f;
  if (e < ob1) scale = sqrtf(2.f / D);
  else if (e >= oW2 && e < ob2) scale = sqrtf(2.f / H);
  else if (e >= oW3 && e < ob3) scale = sqrtf(2.f / H);
  float v = 0.f;
  if (scale > 0.f) {
    const u4_t r = philox4x32_10({(uint32_t)e, (uint32_t)(e >> 32), 7u, 0u}, k0, k1);
    const float u1 = u01_f32(r.x), u2 = u01_f32(r.y);
    v = scale * sqrtf(-2.f * logf(u1)) * cosf(6.28318530717958647692f * u2);
  }
  master[e] = v;
  eff[e] = bf16_bits_to_f32(f32_to_bf16_bits(v));
}

// gather a minibatch: indices from Philox (with replacement), step tau
__global__ __launch_bounds__(256) void k_mlp_batch(uint32_t k0, uint32_t k1, long tau, const float* __restrict__ Xs,
                                                   const float* __restrict__ ts, int D, long n, int nb,
                                                   float* __restrict__ xb, float* __restrict__ tb,
                                                   int* __restrict__ idx) {
  const int j = blockIdx.x;
  __shared__ long src;
  if (threadIdx.x == 0) {
    const u4_t r = philox4x32_10({(uint32_t)tau, (uint32_t)(tau >> 32), 8u, (uint32_t)j}, k0, k1);
    const uint64_t bits = ((uint64_t)r.x << 32) | r.y;
    src = (long)(bits % (uint64_t)n);
    idx[j] = (int)src;
    tb[j] = ts[src];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < D; i += 256) xb[i + (long)j * D] = Xs[i + src * D];
}

// dL/dout for L = mean (out - t)^2, and the minibatch loss (one block)
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ out, const float* __restrict__ tb, int nb,
                                                  float* __restrict__ gout, float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int j = threadIdx.x; j < nb; j += 256) {
    const float r = out[j] - tb[j];
    gout[j] = 2.f * r / nb;
    s = fmaf(r, r, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / nb;
}

// output layer backward: gW3[o] = sum_s gout[s] h2[o,s] (one wave per o),
// gb3 = sum gout; ga2[o,s] = w3[o] gout[s] gelu'(a2[o,s])
__global__ __launch_bounds__(256) void k_mlp_out_bwd(const float* __restrict__ w3, const float* __restrict__ gout,
                                                     const float* __restrict__ h2, const float* __restrict__ a2, int H,
                                                     int nb, float* __restrict__ gW3, float* __restrict__ gb3,
                                                     float* __restrict__ ga2) {
  const int lane = threadIdx.x & 63, o = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (o < H) {
    float acc = 0.f;
    for (int s = lane; s < nb; s += 64) acc = fmaf(gout[s], h2[o + (long)s * H], acc);
    acc = wave_sum_f32(acc);
    if (lane == 0) gW3[o] = acc;
    for (int s = lane; s < nb; s += 64) ga2[o + (long)s * H] = w3[o] * gout[s] * gelu_grad_f(a2[o + (long)s * H]);
  }
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    float b = 0.f;
    for (int s = lane; s < nb; s += 64) b += gout[s];
    b = wave_sum_f32(b);
    if (lane == 0) gb3[0] = b;
  }
}

// bias gradient: gb[o] = sum_s g[o + s*H] (one wave per o)
__global__ __launch_bounds__(256) void k_mlp_bias_grad(const float* __restrict__ g, int H, int nb,
                                                       float* __restrict__ gb) {
  const int lane = threadIdx.x & 63, o = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (o >= H) return;
  float acc = 0.f;
  for (int s = lane; s < nb; s += 64) acc += g[o + (long)s * H];
  acc = wave_sum_f32(acc);
  if (lane == 0) gb[o] = acc;
}

// Adam (Kingma & Ba 2015), bias-corrected; eff = bf16 rounding of the master
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ master, float* __restrict__ eff,
                                                  const float* __restrict__ g, float* __restrict__ m,
                                                  float* __restrict__ v, long nparam, float lr, float b1, float b2,
                                                  float eps, float c1, float c2) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= nparam) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.f - b1) * gg;
  const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  const float w = master[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  master[e] = w;
  eff[e] = bf16_bits_to_f32(f32_to_bf16_bits(w));
}

__global__ void k_fill_f32(float* p, long n) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = 0.f;
}

static dim3 g2(int M, int N) { return dim3(cdiv(M, 64), cdiv(N, 64)); }

size_t mlp_nparam(int D, int H) { return (size_t)H * D + H + (size_t)H * H + H + H + 1; }

// Forward pass of n samples held in xs (D x n); writes a1, h1, a2, h2, out.
hipError_t mlp_forward(const MlpBufs& b, const float* xs, int n, hipStream_t s) {
  const int D = b.D, H = b.H;
  const float* W1 = b.eff;
  const float* b1 = W1 + (long)H * D;
  const float* W2 = b1 + H;
  const float* b2 = W2 + (long)H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + H;
  hipLaunchKernelGGL((k_mlp_gemm<true, true, 1>), g2(H, n), dim3(256), 0, s, W1, D, H, xs, D, n, D, b.a1, H, b1,
                     (const float*)nullptr, b.h1);
  hipLaunchKernelGGL((k_mlp_gemm<true, true, 1>), g2(H, n), dim3(256), 0, s, W2, H, H, (const float*)b.h1, H, n, H,
                     b.a2, H, b2, (const float*)nullptr, b.h2);
  hipLaunchKernelGGL(k_mlp_out, dim3(cdiv(n, 4)), dim3(256), 0, s, W3, b3, (const float*)b.h2, H, n, b.out);
  return hipGetLastError();
}

hipError_t mlp_eval(const MlpBufs& b, const double* X64, const float* X32, int n, double* s_out, hipStream_t s) {
  const long tot = (long)b.D * n;
  hipLaunchKernelGGL(k_mlp_standardize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X64, X32,
                     (const float*)b.in_mean, (const float*)b.in_scale, b.D, (long)n, b.xb);
  hipError_t e = mlp_forward(b, b.xb, n, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_denorm, dim3(cdiv(n, 256)), dim3(256), 0, s, (const float*)b.out, (const float*)b.stats, n,
                     s_out);
  return hipGetLastError();
}

hipError_t mlp_prepare(const MlpBufs& b, const double* X, const double* lp, long n, uint64_t seed, hipStream_t s) {
  const int D = b.D;
  hipLaunchKernelGGL(k_mlp_in_stats, dim3(D), dim3(256), 0, s, X, b.d_state, n, b.in_mean, b.in_scale);
  hipLaunchKernelGGL(k_mlp_out_stats, dim3(1), dim3(256), 0, s, lp, n, b.stats, b.ts);
  const long tot = (long)D * n;
  hipLaunchKernelGGL(k_mlp_standardize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, (const float*)nullptr,
                     (const float*)b.in_mean, (const float*)b.in_scale, D, n, b.Xs);
  const long np = (long)mlp_nparam(D, b.H);
  hipLaunchKernelGGL(k_mlp_init, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, (uint32_t)seed,
                     (uint32_t)(seed >> 32), D, b.H, b.master, b.eff, np);
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((2 * np + 255) / 256)), dim3(256), 0, s, b.m, 2 * np);
  return hipGetLastError();
}

// One Adam step on a Philox-drawn minibatch of nb training pairs.
hipError_t mlp_train_step(const MlpBufs& b, long n, int nb, long tau, uint64_t seed, float lr, hipStream_t s) {
  const int D = b.D, H = b.H;
  const long np = (long)mlp_nparam(D, H);
  float* gW1 = b.grad;
  float* gb1 = gW1 + (long)H * D;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (long)H * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + H;
  const float* W2 = b.eff + (long)H * D + H;
  const float* W3 = W2 + (long)H * H + H;
  hipLaunchKernelGGL(k_mlp_batch, dim3(nb), dim3(256), 0, s, (uint32_t)seed, (uint32_t)(seed >> 32), tau,
                     (const float*)b.Xs, (const float*)b.ts, D, n, nb, b.xb, b.tb, b.bidx);
  hipError_t e = mlp_forward(b, b.xb, nb, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s, (const float*)b.out, (const float*)b.tb, nb, b.gout, b.loss);
  hipLaunchKernelGGL(k_mlp_out_bwd, dim3(cdiv(H, 4)), dim3(256), 0, s, W3, (const float*)b.gout, (const float*)b.h2,
                     (const float*)b.a2, H, nb, gW3, gb3, b.ga2);
  // gW2 = ga2 h1^T ; gb2 = rowsum(ga2)
  hipLaunchKernelGGL((k_mlp_gemm<false, false, 0>), g2(H, H), dim3(256), 0, s, (const float*)b.ga2, H, H,
                     (const float*)b.h1, H, H, nb, gW2, H, (const float*)nullptr, (const float*)nullptr,
                     (float*)nullptr);
  hipLaunchKernelGGL(k_mlp_bias_grad, dim3(cdiv(H, 4)), dim3(256), 0, s, (const float*)b.ga2, H, nb, gb2);
  // ga1 = (W2^T ga2) * gelu'(a1)
  hipLaunchKernelGGL((k_mlp_gemm<false, true, 2>), g2(H, nb), dim3(256), 0, s, W2, H, H, (const float*)b.ga2, H, nb, H,
                     b.ga1, H, (const float*)nullptr, (const float*)b.a1, (float*)nullptr);
  // gW1 = ga1 xb^T ; gb1 = rowsum(ga1)
  hipLaunchKernelGGL((k_mlp_gemm<false, false, 0>), g2(H, D), dim3(256), 0, s, (const float*)b.ga1, H, H,
                     (const float*)b.xb, D, D, nb, gW1, D, (const float*)nullptr, (const float*)nullptr,
                     (float*)nullptr);
  hipLaunchKernelGGL(k_mlp_bias_grad, dim3(cdiv(H, 4)), dim3(256), 0, s, (const float*)b.ga1, H, nb, gb1);
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)(tau + 1)), c2 = 1.f - powf(b2, (float)(tau + 1));
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, b.master, b.eff,
                     (const float*)b.grad, b.m, b.m + np, np, lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

// ============================================================================
// Delayed acceptance, stage 1 (one workgroup of 16 waves):
//   s_new[p] = out_std * (w3 . h2[:, p] + b3) + out_mean       (network output)
//   log a1   = (s_new - s_cur) + [plain form only] (|z'|^2 - |z|^2) / (2 alpha^2)
// In the residual form the surrogate is r(x) - |z(x)|^2 / (2 alpha^2): its
// Gaussian part cancels the proposal's own correction, so stage 1 compares
// the network outputs alone.  Survivors get consecutive slots in chain
// order (wave ballots + prefix counts), so packing is deterministic.
// ============================================================================
__global__ __launch_bounds__(1024) void k_da_screen(const float* __restrict__ w3, const float* __restrict__ b3,
                                                    const float* __restrict__ h2, int H,
                                                    const float* __restrict__ stats, int P, int nch,
                                                    const double* __restrict__ s_cur,
                                                    const double* __restrict__ zq_part,
                                                    const double* __restrict__ zq, const double* __restrict__ u1,
                                                    double inv2a2, int resid, double* __restrict__ s_new,
                                                    uint8_t* __restrict__ pass, int* __restrict__ slot,
                                                    int* __restrict__ idx, int* __restrict__ nsurv,
                                                    int* __restrict__ npass) {
  __shared__ int wt[16];
  __shared__ int base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double om = (double)stats[0], os = (double)stats[1];
  for (int q = w; q < P; q += 16) {
    float acc = 0.f;
    for (int o = lane; o < H; o += 64) acc = fmaf(w3[o], h2[o + (long)q * H], acc);
    acc = wave_sum_f32(acc);
    if (lane == 0) s_new[q] = (double)(acc + b3[0]) * os + om;
  }
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int p0 = 0; p0 < P; p0 += 1024) {
    const int p = p0 + threadIdx.x;
    int ok = 0;
    if (p < P) {
      double la1 = s_new[p] - s_cur[p];
      if (!resid) {
        double zs = 0.0;
        for (int c = 0; c < nch; ++c) zs += zq_part[(long)p * nch + c];
        la1 += (zs - zq[p]) * inv2a2;
      }
      ok = log(u1[p]) < la1 ? 1 : 0;
      pass[p] = (uint8_t)ok;
      npass[p] += ok;
    }
    const unsigned long long m = __ballot(ok);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wt[w] = __popcll(m);
    __syncthreads();
    int off = base;
    for (int v = 0; v < w; ++v) off += wt[v];
    if (p < P) {
      slot[p] = ok ? off + below : -1;
      if (ok) idx[off + below] = p;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int v = 0; v < 16; ++v) t += wt[v];
      base += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *nsurv = base;
}

// survivors' proposals, packed: Vs[:, j] = V[:, idx[j]] for j < nsurv
__global__ __launch_bounds__(256) void k_da_gather(const float* __restrict__ V, const int* __restrict__ idx,
                                                   const int* __restrict__ nsurv, int d, int P,
                                                   float* __restrict__ Vs) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const int j = (int)(e / d), i = (int)(e % d);
  if (j >= P || j >= *nsurv) return;
  Vs[i + (long)j * d] = V[i + (long)idx[j] * d];
}

hipError_t da_screen(const MlpBufs& b, const float* V, int d, int P, int nch, const double* s_cur,
                     const double* zq_part, const double* zq, const double* u1, double inv2a2, int resid,
                     double* s_new, uint8_t* pass, int* slot, int* idx, int* nsurv, int* npass, float* Vs,
                     hipStream_t s) {
  const long tot = (long)b.D * P;
  hipLaunchKernelGGL(k_mlp_standardize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, (const double*)nullptr,
                     V, (const float*)b.in_mean, (const float*)b.in_scale, b.D, (long)P, b.xb);
  const int H = b.H;
  const float* W1 = b.eff;
  const float* b1 = W1 + (long)H * b.D;
  const float* W2 = b1 + H;
  const float* b2 = W2 + (long)H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + H;
  hipLaunchKernelGGL((k_mlp_gemm<true, true, 1>), g2(H, P), dim3(256), 0, s, W1, b.D, H, (const float*)b.xb, b.D, P,
                     b.D, b.a1, H, b1, (const float*)nullptr, b.h1);
  hipLaunchKernelGGL((k_mlp_gemm<true, true, 1>), g2(H, P), dim3(256), 0, s, W2, H, H, (const float*)b.h1, H, P, H,
                     b.a2, H, b2, (const float*)nullptr, b.h2);
  hipLaunchKernelGGL(k_da_screen, dim3(1), dim3(1024), 0, s, W3, b3, (const float*)b.h2, H, (const float*)b.stats, P,
                     nch, s_cur, zq_part, zq, u1, inv2a2, resid, s_new, pass, slot, idx, nsurv, npass);
  hipLaunchKernelGGL(k_da_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, V, (const int*)idx,
                     (const int*)nsurv, d, P, Vs);
  return hipGetLastError();
}

// t[k] = lp[k] + c zq[k]  (residual-form training targets)
__global__ __launch_bounds__(256) void k_axpy_f64(const double* __restrict__ lp, const double* __restrict__ zq,
                                                  double c, long n, double* __restrict__ t) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < n) t[e] = __fma_rn(c, zq[e], lp[e]);
}

hipError_t axpy_f64(const double* lp, const double* zq, double c, long n, double* t, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, lp, zq, c, n, t);
  return hipGetLastError();
}

}  // namespace dk
