// DIAM kernels for gfx950.  Every kernel is written for 64-wide wavefronts;
// dense contractions run on MFMA through the tile engines of gemm.h.
#include <math.h>

#include "gemm.h"
#include "kernels.h"

using namespace gemm;

namespace dk {

// x' = x_ref + rho (x - x_ref) + xi, one rounding sequence used everywhere
// the proposal of a state is formed (propose and accept must agree bitwise).
DEV double propose1(double xr, double x, double rho, double xi) { return __fma_rn(rho, x - xr, xr) + xi; }

// ============================================================================
// (b) target log-density: Gaussian, Y = R (x - mu) on MFMA, then column sums
// of Y^2 in FP64 per 64-row block (the caller adds the blocks in order).
// ============================================================================
// One output tile: rows [bx BM, +BM) of Y, chains [by BN, +BN); the tile's
// FP64 partial sums go to part[j * ldp + bx] (chain-major: a chain's ldp
// row-block partials are contiguous for the reader).
template <typename T, int BK, int BM, int BN, int KG>
DEV void tgt_gauss_tile(const T* __restrict__ R, const T* __restrict__ V, int d, int P, int bx, int by,
                        double* __restrict__ part, int ldp, const double* __restrict__ twist = nullptr) {
  __shared__ T lds[KG * e_lds_elems<T, BM, BN, BK>()];
  __shared__ double red[2][BN];
  const int i0 = bx * BM, j0 = by * BN;
  EFrag<T, BM, BN> f;
  f.zero();
  e_gemm<T, BM, BN, BK, true, true, KG>(f, R, d, d, V, d, P, i0, j0, 0, d, lds);
  const bool g0 = threadIdx.x < NT;
  const int lane = threadIdx.x & 63, w = (threadIdx.x & (NT - 1)) >> 6, wm = w & 1, wn = w >> 1;
  if (g0) {
#pragma unroll
    for (int n = 0; n < EFrag<T, BM, BN>::FN; ++n) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < EFrag<T, BM, BN>::FM; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double y = (double)f.c[m][n][r];
          if (twist) {
            // twisted target: row 2k+1 gets c y_{2k}^2 added before squaring.  Its
            // partner row sits in the same lane (FP32 layout: rows 4q + r) or in
            // lane ^ 16 (FP64 layout: rows 4r + q)
            const double yp = (sizeof(T) == 8) ? lane_xor_f64<16>(y) : (double)f.c[m][n][r & ~1];
            int ti, tj;
            frag_coords<BM, BN, T>(m, n, r, ti, tj);
            const int i = i0 + ti;
            if ((i & 1) && i < d) y = __fma_rn(twist[i], yp * yp, y);
          }
          s = __fma_rn(y, y, s);
        }
      s += lane_xor_f64<16>(s);
      s += lane_xor_f64<32>(s);
      if (lane < 16) red[wm][wn * (BN / 2) + n * 16 + lane] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < BN) {
    const int j = j0 + threadIdx.x;
    if (j < P) part[(long)j * ldp + bx] = -0.5 * (red[0][threadIdx.x] + red[1][threadIdx.x]);
  }
}

template <typename T, int BK>
__global__ __launch_bounds__(512) void k_tgt_gauss(const T* __restrict__ R, const T* __restrict__ V, int d, int P,
                                                   double* __restrict__ part, const double* __restrict__ twist) {
  tgt_gauss_tile<T, BK, 64, 64, 2>(R, V, d, P, blockIdx.x, blockIdx.y, part, gridDim.x, twist);
}

// ---- two-part half target (mixed form): Y = R V with both operands split
// into two IEEE half parts (products with the accuracy of FP32, see h2_gemm).
// Half precision needs operands in its range, so both are scaled by powers of
// two, exactly: coordinate k of x - mu by 2^s_k (vsc), chosen from the
// largest deviation of the current states and the current factor's row norm
// so that values up to 1024 times those stay finite (the step kernel flags
// any beyond); row i of R by
// 2^(a_i - s_k) so that its largest entry lies in [2^14, 2^15).  Then
// (R' V')_i = 2^a_i (R V)_i and the reduction multiplies by 2^-a_i (rsc).
// 64- or 128-wide tiles, K split in H2_KSPLIT ranges whose FP32 partial Y are
// summed in FP64 by the reduction, which squares and sums 64-row blocks
// (chain-major partials).
constexpr int H2_KSPLIT = 4;
// scaled V entries at or above this magnitude round to infinity in half
constexpr double H2_RANGE = 65520.0;

// vsc[k] = 2^(6 - e_k) with sigma_k < 2^e_k (frexp), sigma_k the larger of
// max_p |x_kp - mu_k| and the 2-norm of row k of the lower factor L
// (column-major; the spread of the proposals), or the former alone for an
// evaluation of the states themselves; e_k clamped to [-100, 100].  64 rows per block, one per
// lane; the 16 waves split the columns of L and the chains.
__global__ __launch_bounds__(1024) void k_h2_vscale(const double* __restrict__ X, const double* __restrict__ mu,
                                                    const double* __restrict__ L, int d, int P, int states_only,
                                                    float* __restrict__ vsc) {
  __shared__ double sdev[16][64], srn[16][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  double dev = 0.0, rn = 0.0;
  if (k < d) {
    const double mk = mu[k];
    for (int p = w; p < P; p += 16) dev = fmax(dev, fabs(X[k + (long)p * d] - mk));
    for (int j = w; j <= k; j += 16) {
      const double l = L[k + (long)j * d];
      rn = __fma_rn(l, l, rn);
    }
  }
  sdev[w][lane] = dev;
  srn[w][lane] = rn;
  __syncthreads();
  if (w != 0 || k >= d) return;
  for (int q = 1; q < 16; ++q) {
    dev = fmax(dev, sdev[q][lane]);
    rn += srn[q][lane];
  }
  // states_only (the evaluation of the states themselves): their spread
  // alone, the factor's row norm only where they do not spread
  const double sig = (states_only && dev > 0.0) ? dev : fmax(dev, sqrt(rn));
  int e = 0;
  if (sig > 0.0 && isfinite(sig)) {
    frexp(sig, &e);  // sig < 2^e
    e = 6 - e;
  }
  e = e < -100 ? -100 : (e > 100 ? 100 : e);
  vsc[k] = ldexpf(1.0f, e);
}

// Row i of R: a_i from the largest |R_ik / vsc[k]|, then both half parts of
// R_ik 2^a_i / vsc[k] into R2 (d x d each, in the tiled order h2_gemm reads,
// h2_tile_index) and rsc[i] = 2^-a_i.
__global__ __launch_bounds__(256) void k_h2_split_r(const float* __restrict__ R, const float* __restrict__ vsc, int d,
                                                    u16* __restrict__ R2, double* __restrict__ rsc) {
  __shared__ float red[4];
  const int i = blockIdx.x, t = threadIdx.x;
  const float* row = R + (long)i * d;
  float mx = 0.0f;
  for (int k = t; k < d; k += 256) mx = fmaxf(mx, fabsf(row[k] / vsc[k]));
  mx = wave_max_f32(mx);
  if ((t & 63) == 0) red[t >> 6] = mx;
  __syncthreads();
  mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  int e = 0;
  if (mx > 0.0f && isfinite(mx)) {
    frexpf(mx, &e);  // mx < 2^e
    e = 15 - e;
  }
  const long n = (long)d * d;
  const int arb = d / 16;
  for (int k = t; k < d; k += 256) {
    const double v = ldexp((double)row[k] / (double)vsc[k], e);
    u16 h, l;
    split_f16(v, h, l);
    const long q = h2_tile_index(i, k, arb);
    R2[q] = h;
    R2[n + q] = l;
  }
  if (t == 0) rsc[i] = ldexp(1.0, -e);
}

// Both half parts of (x - mu) vsc into V2 (d x P each, column-major).
__global__ __launch_bounds__(256) void k_h2_split_v(const double* __restrict__ X, const double* __restrict__ mu,
                                                    const float* __restrict__ vsc, int d, long n,
                                                    u16* __restrict__ V2) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int k = (int)(e % d);
  u16 h, l;
  split_f16((X[e] - mu[k]) * (double)vsc[k], h, l);
  V2[e] = h;
  V2[n + e] = l;
}

hipError_t h2_scales(const double* X, const double* mu, const double* L, const float* R, int d, int P, float* vsc,
                     uint16_t* R2, double* rsc, hipStream_t s, int states_only) {
  hipLaunchKernelGGL(k_h2_vscale, dim3((unsigned)((d + 63) / 64)), dim3(1024), 0, s, X, mu, L, d, P, states_only,
                     vsc);
  hipLaunchKernelGGL(k_h2_split_r, dim3(d), dim3(256), 0, s, R, (const float*)vsc, d, (u16*)R2, rsc);
  return hipGetLastError();
}

hipError_t h2_split_v(const double* X, const double* mu, const float* vsc, int d, int P, uint16_t* V2,
                      hipStream_t s) {
  const long n = (long)d * P;
  hipLaunchKernelGGL(k_h2_split_v, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, mu, vsc, d, n, (u16*)V2);
  return hipGetLastError();
}

template <int BM, int BN, int WGM, int WGN, int ST>
__global__ __launch_bounds__(64 * WGM * WGN) void k_tgt_h2(const u16* __restrict__ R2, const u16* __restrict__ V2,
                                                          int d, int P, float* __restrict__ Yp) {
  typedef W32Frag<BM, BN, WGM, WGN> F;
  __shared__ __attribute__((aligned(1024))) u16 lds[h2_lds_elems<BM, BN, ST>()];
  int i0 = blockIdx.x * BM, j0 = blockIdx.y * BN, ks = blockIdx.z;
  if (gridDim.y == 1 && gridDim.z == 1) {
    // one-dimensional grid: workgroups go round-robin to the eight XCDs, and
    // XCDs x and x + 4 take K range x mod 4, each half of the (row, chain)
    // tiles, a row block's chain tiles adjacent; an XCD then reads only its
    // quarter of x - mu and each tile of R once (requires the split into 4
    // and an even number of (row, chain) tiles, checked by the launcher)
    const int ncb = P / BN, half = (d / BM) * ncb / 2;
    const int xcd = blockIdx.x & 7, q = (xcd >> 2) * half + (blockIdx.x >> 3);
    ks = xcd & 3;
    i0 = (q / ncb) * BM;
    j0 = (q % ncb) * BN;
  }
  const int kl = d / H2_KSPLIT;
  // the output pointer is loaded before the loop: a scalar load left in
  // flight there would make every LDS wait of the pipelined loop a full one
  float* Y = Yp + (long)ks * P * d;
  asm volatile("" ::"s"(Y));
  F f;
  f.zero();
  h2_gemm<BM, BN, WGM, WGN, ST>(f, R2, (long)d * d, d / 16, V2, (long)d * P, d, i0, j0, ks * kl, (ks + 1) * kl,
                                lds);
#pragma unroll
  for (int m = 0; m < F::FM; ++m)
#pragma unroll
    for (int n = 0; n < F::FN; ++n)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        int ti, tj;
        w32_coords<BM, BN, WGM, WGN>(m, n, g, ti, tj);
        // four consecutive rows of one chain: one 16-byte store
        const f4_t v = {f.c[m][n][4 * g], f.c[m][n][4 * g + 1], f.c[m][n][4 * g + 2], f.c[m][n][4 * g + 3]};
        *(f4_t*)(Y + (long)(j0 + tj) * d + i0 + ti) = v;
      }
}

// part[j][rb] = -1/2 sum over rows of block rb of (rsc_i sum_s Yp[s])^2.  One
// wave per chain and four 64-row blocks: lane l takes rows 4l .. 4l + 3 of the
// wave's 256 (16-byte loads), sixteen lanes make one block (d is a multiple
// of 64, so a block is wholly inside or outside).
// Rows 256 q4 .. 256 q4 + 255 of chain j on one wavefront: the four row-block
// terms go to part; every lane returns its block's term.
DEV double h2_reduce_wave(const float* __restrict__ Yp, const double* __restrict__ rsc, int d, int P, int nrb,
                          double* __restrict__ part, const double* __restrict__ twist, int j, int q4) {
  const int lane = threadIdx.x & 63;
  const int i = q4 * 256 + 4 * lane;
  double q = 0.0;
  if (i < d) {
    double y[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < H2_KSPLIT; ++s) {
      const f4_t v = *(const f4_t*)(Yp + ((long)s * P + j) * d + i);
#pragma unroll
      for (int r = 0; r < 4; ++r) y[r] += (double)v[r];
    }
    const double2 r01 = *(const double2*)(rsc + i), r23 = *(const double2*)(rsc + i + 2);
    y[0] *= r01.x;
    y[1] *= r01.y;
    y[2] *= r23.x;
    y[3] *= r23.y;
    if (twist) {
      // twisted target: row 2k+1 gets c y_{2k}^2 (pairs lie within a lane)
      y[1] = __fma_rn(twist[i + 1], y[0] * y[0], y[1]);
      y[3] = __fma_rn(twist[i + 3], y[2] * y[2], y[3]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) q = __fma_rn(y[r], y[r], q);
  }
  q = row16_sum_f64(q);
  const int rb = q4 * 4 + (lane >> 4);
  if ((lane & 15) == 0 && i < d) part[(long)j * nrb + rb] = -0.5 * q;
  return -0.5 * q;
}

__global__ __launch_bounds__(256) void k_tgt_h2_reduce(const float* __restrict__ Yp, const double* __restrict__ rsc,
                                                       int d, int P, int nrb, double* __restrict__ part,
                                                       const double* __restrict__ twist) {
  const int nq = (nrb + 3) / 4;
  const long wid = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= (long)P * nq) return;
  h2_reduce_wave(Yp, rsc, d, P, nrb, part, twist, (int)(wid / nq), (int)(wid % nq));
}

#ifndef TGT_H2_XMAP
#define TGT_H2_XMAP 1
#endif
bool tgt_h2_ok(int d, int P) { return d % (H2_KSPLIT * 32) == 0 && d % 64 == 0 && P % 64 == 0; }

size_t tgt_h2_scratch_bytes(int d, int P) { return (size_t)H2_KSPLIT * d * P * sizeof(float); }

hipError_t tgt_gauss_h2(const uint16_t* R2, const uint16_t* V2, const double* rsc, int d, int P, float* Yp,
                        double* part, hipStream_t s, const double* twist) {
  // 128 x 128 tiles on 8 waves where they fit
  static_assert(H2_KSPLIT == 4, "the XCD mapping pairs the eight XCDs with four K ranges");
  if (d % 128 == 0 && P % 128 == 0 && (d / 128) * (P / 128) % 2 == 0 && TGT_H2_XMAP)
    hipLaunchKernelGGL((k_tgt_h2<128, 128, 4, 2, 4>), dim3((d / 128) * (P / 128) * H2_KSPLIT), dim3(512), 0, s,
                       (const u16*)R2, (const u16*)V2, d, P, Yp);
  else if (d % 128 == 0 && P % 128 == 0)
    hipLaunchKernelGGL((k_tgt_h2<128, 128, 4, 2, 4>), dim3(d / 128, P / 128, H2_KSPLIT), dim3(512), 0, s,
                       (const u16*)R2, (const u16*)V2, d, P, Yp);
  else
    hipLaunchKernelGGL((k_tgt_h2<64, 64, 2, 2, 4>), dim3(d / 64, P / 64, H2_KSPLIT), dim3(256), 0, s,
                       (const u16*)R2, (const u16*)V2, d, P, Yp);
  if (!part) return hipGetLastError();  // the reduction runs inside the step (step_h2)
  const int nrb = tgt_row_blocks(d);
  const long waves = (long)P * ((nrb + 3) / 4);
  hipLaunchKernelGGL(k_tgt_h2_reduce, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, (const float*)Yp, rsc, d,
                     P, nrb, part, twist);
  return hipGetLastError();
}

hipError_t tgt_gauss(Prec prec, const void* R, const void* V, int d, int P, double* part, hipStream_t s,
                     const double* twist) {
  dim3 grid(cdiv(d, TGT_BM), cdiv(P, 64));
  if (prec == P64)
    hipLaunchKernelGGL((k_tgt_gauss<double, 16>), grid, dim3(512), 0, s, (const double*)R, (const double*)V, d, P, part,
                       twist);
  else
    hipLaunchKernelGGL((k_tgt_gauss<float, 32>), grid, dim3(512), 0, s, (const float*)R, (const float*)V, d, P, part,
                       twist);
  return hipGetLastError();
}

// ============================================================================
// (a) proposal contraction Xi = c L W, L lower triangular: the K range of a
// row tile stops at its last row.
// ============================================================================
template <typename T, int BK>
DEV void trigemm_tile(const T* __restrict__ L, const T* __restrict__ W, T* __restrict__ Xi, int d, int ncols, double c,
                      int bx, int by) {
  constexpr int BM = 64, BN = 64;
  __shared__ T lds[e_lds_elems<T, BM, BN, BK>()];
  const int i0 = bx * BM, j0 = by * BN;
  const int kend = min(d, i0 + BM);
  EFrag<T, BM, BN> f;
  f.zero();
  e_gemm<T, BM, BN, BK, false, true>(f, L, d, d, W, d, ncols, i0, j0, 0, kend, lds);
#pragma unroll
  for (int m = 0; m < EFrag<T, BM, BN>::FM; ++m)
#pragma unroll
    for (int n = 0; n < EFrag<T, BM, BN>::FN; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ti, tj;
        frag_coords<BM, BN, T>(m, n, r, ti, tj);
        const int i = i0 + ti, j = j0 + tj;
        if (i < d && j < ncols) Xi[i + (long)j * d] = (T)(c * (double)f.c[m][n][r]);
      }
}

template <typename T, int BK>
__global__ __launch_bounds__(256) void k_trigemm_e(const T* __restrict__ L, const T* __restrict__ W, T* __restrict__ Xi,
                                                   int d, int ncols, double c) {
  trigemm_tile<T, BK>(L, W, Xi, d, ncols, c, blockIdx.x, blockIdx.y);
}

// bf16: Xi^T = W~^T L~^T with the roles swapped so that lanes run along the
// rows i of Xi (coalesced stores): A operand = W (rows = columns j of W,
// k-contiguous), B operand = L~ (rows i, k-contiguous, row-major factor).
// W~ = W_hi + W_lo and L~ = L_hi + L_lo; the four bf16 products run as one
// segmented, pipelined K loop into the same fp32 registers.
// Tile order: workgroup ids are dealt round-robin to the 8 XCDs, so ids
// xcd + 8 k on one XCD take the ni row blocks of one column block of W
// (longest K range first): that slice of W is fetched into the XCD's L2 once.
// Wide variant: TBM (j) x TBN (i) tiles, WGM x WGN wavefronts, 64-deep K slices.
template <int TBM, int TBN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void k_trigemm_bf16w(const u16* __restrict__ Lhi,
                                                                 const u16* __restrict__ Whi, long dW,
                                                                 float* __restrict__ Xi, int d, int ncols, float c,
                                                                 int vec_ok, int nj, int ni) {
  typedef WFrag<TBM, TBN, WGM, WGN> F;
  __shared__ u16 lds[w_lds_elems<TBM, TBN>()];
  const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
  const int jb = (k / ni) * 8 + xcd;
  if (jb >= nj) return;
  const int ib = ni - 1 - (k % ni);
  const int j0 = jb * TBM, i0 = ib * TBN;
  const int kend = min(d, i0 + TBN);
  F f;
  f.zero();
  w_gemm_seg<TBM, TBN, WGM, WGN>(f, Whi, dW, d, ncols, Lhi, (long)d * d, d, d, vec_ok, j0, i0, 0, kend, 4, lds);
#pragma unroll
  for (int m = 0; m < F::FM; ++m)
#pragma unroll
    for (int n = 0; n < F::FN; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int tj, ti;
        w_coords<TBM, TBN, WGM, WGN>(m, n, r, tj, ti);
        const int i = i0 + ti, j = j0 + tj;
        if (i < d && j < ncols) Xi[i + (long)j * d] = c * f.c[m][n][r];
      }
}
// Direct-to-LDS hi/lo variant for operands that fill whole tiles (d a
// multiple of 2 TBN, ncols of TBM; 256 x 128 tiles on 8 waves, 3-stage ring): the K range of a row tile ends at its
// last row, so row tiles ib and ni - 1 - ib together cost the same for every
// pair; each workgroup takes one such pair of one column block of W (the
// pairs of a column block run on one XCD, which keeps that block of W in its
// L2).  The four products accumulate per 32-deep slice.
template <int TBM, int TBN, int WGM, int WGN, int ST>
__global__ __launch_bounds__(64 * WGM * WGN) void k_trigemm_hl(const u16* __restrict__ Lhi, const u16* __restrict__ Whi,
                                                              long dW, float* __restrict__ Xi, int d, int ncols, float c,
                                                              int nj, int ni) {
  typedef WFrag<TBM, TBN, WGM, WGN> F;
  __shared__ __attribute__((aligned(1024))) u16 lds[h_lds_elems<TBM, TBN, ST>()];
  const int npair = ni / 2;
  const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
  const int jb = (k / npair) * 8 + xcd;
  if (jb >= nj) return;
  const int q = k % npair;
  const int j0 = jb * TBM;
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    const int ib = h ? q : ni - 1 - q;
    const int i0 = ib * TBN;
    const int kend = min(d, i0 + TBN);
    F f;
    f.zero();
    h_gemm<TBM, TBN, WGM, WGN, ST>(f, Whi, dW, d, Lhi, (long)d * d, d, j0, i0, kend, lds);
#pragma unroll
    for (int m = 0; m < F::FM; ++m)
#pragma unroll
      for (int n = 0; n < F::FN; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int tj, ti;
          w_coords<TBM, TBN, WGM, WGN>(m, n, r, tj, ti);
          Xi[(i0 + ti) + (long)(j0 + tj) * d] = c * f.c[m][n][r];
        }
  }
}

// tile shape of the wide proposal kernel
constexpr int TW_BM = 256, TW_BN = 128, TW_WGM = 4, TW_WGN = 2;

hipError_t trigemm(Prec prec, const void* L, const void* W, const void* Wlo, void* Xi, int d, long ncols, double c,
                   hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  dim3 grid(cdiv(d, 64), cdiv(ncols, 64));
  if (prec == P64)
    hipLaunchKernelGGL((k_trigemm_e<double, 16>), grid, dim3(256), 0, s, (const double*)L, (const double*)W,
                       (double*)Xi, d, (int)ncols, c);
  else if (prec == P32)
    hipLaunchKernelGGL((k_trigemm_e<float, 32>), grid, dim3(256), 0, s, (const float*)L, (const float*)W, (float*)Xi,
                       d, (int)ncols, c);
  else {
    const u16* Lhi = (const u16*)L;
    const long dW = (const u16*)Wlo - (const u16*)W;
    const int vec_ok = (d % 8 == 0) && ((uintptr_t)L % 16 == 0) && ((uintptr_t)W % 16 == 0) && ((uintptr_t)Wlo % 16 == 0);
    const bool whole = vec_ok && (ncols % 256 == 0);
    if (whole && d % 512 == 0) {
      const int nj = ncols / 256, ni = d / 256, groups = (nj + 7) / 8;
      hipLaunchKernelGGL((k_trigemm_hl<256, 256, 2, 4, 2>), dim3(groups * 8 * (ni / 2)), dim3(512), 0, s, Lhi,
                         (const u16*)W, dW, (float*)Xi, d, (int)ncols, (float)c, nj, ni);
      return hipGetLastError();
    }
    if (whole && d % 256 == 0) {
      const int nj = ncols / 256, ni = d / 128, groups = (nj + 7) / 8;
      hipLaunchKernelGGL((k_trigemm_hl<256, 128, 4, 2, 3>), dim3(groups * 8 * (ni / 2)), dim3(512), 0, s, Lhi,
                         (const u16*)W, dW, (float*)Xi, d, (int)ncols, (float)c, nj, ni);
      return hipGetLastError();
    }
    const int nj = cdiv(ncols, TW_BM), ni = cdiv(d, TW_BN), groups = (nj + 7) / 8;
    hipLaunchKernelGGL((k_trigemm_bf16w<TW_BM, TW_BN, TW_WGM, TW_WGN>), dim3(groups * 8 * ni),
                       dim3(64 * TW_WGM * TW_WGN), 0, s, Lhi, (const u16*)W, dW, (float*)Xi, d, (int)ncols, (float)c,
                       vec_ok, nj, ni);
  }
  return hipGetLastError();
}

// ============================================================================
// (d) window scatter G = sum_k xs_k xs_k^T (lower tiles) and row sums h.
// ============================================================================
DEV void tile_pair(int t, int& bi, int& bj) {
  // t enumerates (bi >= bj) row by row: t = bi (bi + 1)/2 + bj
  int b = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((b + 1) * (b + 2) / 2 <= t) ++b;
  while (b * (b + 1) / 2 > t) --b;
  bi = b;
  bj = t - b * (b + 1) / 2;
}

constexpr int FOLD_K = 4096;  // fp32 accumulation span before folding into fp64

// lower tile t (row-by-row enumeration) of the scatter over K split ksp
template <typename T, int BK>
DEV void syrk_tile(const T* __restrict__ Xs, int d, int K, int kchunk, int t, int ksp, double* __restrict__ Gpart) {
  constexpr int BM = 64, BN = 64;
  __shared__ T lds[e_lds_elems<T, BM, BN, BK>()];
  int bi, bj;
  tile_pair(t, bi, bj);
  const int i0 = bi * BM, j0 = bj * BN;
  const int kb = ksp * kchunk, ke = min(K, kb + kchunk);
  double acc[EFrag<T, BM, BN>::FM][EFrag<T, BM, BN>::FN][4];
#pragma unroll
  for (int m = 0; m < EFrag<T, BM, BN>::FM; ++m)
#pragma unroll
    for (int n = 0; n < EFrag<T, BM, BN>::FN; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[m][n][r] = 0.0;
  const int span = (sizeof(T) == 8) ? kchunk : FOLD_K;
  for (int k0 = kb; k0 < ke; k0 += span) {
    EFrag<T, BM, BN> f;
    f.zero();
    e_gemm<T, BM, BN, BK, false, false>(f, Xs, d, d, Xs, d, d, i0, j0, k0, min(ke, k0 + span), lds);
#pragma unroll
    for (int m = 0; m < EFrag<T, BM, BN>::FM; ++m)
#pragma unroll
      for (int n = 0; n < EFrag<T, BM, BN>::FN; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[m][n][r] += (double)f.c[m][n][r];
  }
  double* G = Gpart + (long)ksp * d * d;
#pragma unroll
  for (int m = 0; m < EFrag<T, BM, BN>::FM; ++m)
#pragma unroll
    for (int n = 0; n < EFrag<T, BM, BN>::FN; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ti, tj;
        frag_coords<BM, BN, T>(m, n, r, ti, tj);
        const int i = i0 + ti, j = j0 + tj;
        if (i < d && j < d) G[j + (long)i * d] = acc[m][n][r];  // G(i,j) at (row j, col i): upper
      }
}

template <typename T, int BK>
__global__ __launch_bounds__(256) void k_syrk_e(const T* __restrict__ Xs, int d, int K, int kchunk,
                                                double* __restrict__ Gpart) {
  syrk_tile<T, BK>(Xs, d, K, kchunk, blockIdx.x, blockIdx.y, Gpart);
}

// bf16: Xt is the transposed window (d x K row-major, ld = K).  Tiles are
// 128 rows (i) x 64 columns (j) covering the lower triangle: in row block bi
// the column blocks bj < 2 (bi + 1).  fp32 accumulation is folded into fp64
// every FOLD_BF16 columns of K.
constexpr int FOLD_BF16 = 2048;

DEV void syrk_tile_128x64(int t, int nbj, int& bi, int& bj) {
  int b = 0, c0 = 0;
  for (;;) {
    const int n = min(2 * b + 2, nbj);
    if (t < c0 + n) break;
    c0 += n;
    ++b;
  }
  bi = b;
  bj = t - c0;
}

__global__ __launch_bounds__(256) void k_syrk_bf16(const u16* __restrict__ Xt, int d, int K, int kchunk, int vec_ok,
                                                   double* __restrict__ Gpart) {
  constexpr int BM = 128, BN = 64;
  __shared__ u16 lds[b_lds_elems<BM, BN>()];
  int bi, bj;
  syrk_tile_128x64(blockIdx.x, (d + 63) / 64, bi, bj);
  const int i0 = bi * BM, j0 = bj * BN;
  const int kb = blockIdx.y * kchunk, ke = min(K, kb + kchunk);
  double acc[BFrag<BM, BN>::FM][BFrag<BM, BN>::FN][4];
#pragma unroll
  for (int m = 0; m < BFrag<BM, BN>::FM; ++m)
#pragma unroll
    for (int n = 0; n < BFrag<BM, BN>::FN; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[m][n][r] = 0.0;
  for (int k0 = kb; k0 < ke; k0 += FOLD_BF16) {
    BFrag<BM, BN> f;
    f.zero();
    b_gemm<BM, BN>(f, Xt, K, d, vec_ok, Xt, K, d, vec_ok, i0, j0, k0, min(ke, k0 + FOLD_BF16), lds);
#pragma unroll
    for (int m = 0; m < BFrag<BM, BN>::FM; ++m)
#pragma unroll
      for (int n = 0; n < BFrag<BM, BN>::FN; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[m][n][r] += (double)f.c[m][n][r];
  }
  double* G = Gpart + (long)blockIdx.y * d * d;
#pragma unroll
  for (int m = 0; m < BFrag<BM, BN>::FM; ++m)
#pragma unroll
    for (int n = 0; n < BFrag<BM, BN>::FN; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ti, tj;
        frag_coords<BM, BN>(m, n, r, ti, tj);
        const int i = i0 + ti, j = j0 + tj;
        if (i < d && j < d) G[j + (long)i * d] = acc[m][n][r];  // G(i,j) at (row j, col i): upper
      }
}

// Direct-to-LDS variant for whole tiles (d a multiple of 256, K chunks of
// 64): 256 (i) x 128 (j) tiles covering the lower triangle (bj < 2 (bi + 1)),
// fp32 accumulation folded into fp64 every FOLD_BF16 columns.
DEV void syrk_tile_256x128(int t, int nbj, int& bi, int& bj) {
  int b = 0, c0 = 0;
  for (;;) {
    const int n = min(2 * b + 2, nbj);
    if (t < c0 + n) break;
    c0 += n;
    ++b;
  }
  bi = b;
  bj = t - c0;
}

__global__ __launch_bounds__(512) void k_syrk_pl(const u16* __restrict__ Xt, int d, int K, int kchunk,
                                                 double* __restrict__ Gpart) {
  constexpr int BM = 256, BN = 128, WGM = 4, WGN = 2, ST = 3;
  typedef WFrag<BM, BN, WGM, WGN> F;
  __shared__ __attribute__((aligned(1024))) u16 lds[p_lds_elems<BM, BN, ST>()];
  int bi, bj;
  syrk_tile_256x128(blockIdx.x, d / 128, bi, bj);
  const int i0 = bi * BM, j0 = bj * BN;
  const int kb = blockIdx.y * kchunk, ke = min(K, kb + kchunk);
  double acc[F::FM][F::FN][4];
#pragma unroll
  for (int m = 0; m < F::FM; ++m)
#pragma unroll
    for (int n = 0; n < F::FN; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[m][n][r] = 0.0;
  for (int k0 = kb; k0 < ke; k0 += FOLD_BF16) {
    F f;
    f.zero();
    p_gemm<BM, BN, WGM, WGN, ST>(f, Xt, K, Xt, K, i0, j0, k0, min(ke, k0 + FOLD_BF16), lds);
#pragma unroll
    for (int m = 0; m < F::FM; ++m)
#pragma unroll
      for (int n = 0; n < F::FN; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[m][n][r] += (double)f.c[m][n][r];
  }
  double* G = Gpart + (long)blockIdx.y * d * d;
#pragma unroll
  for (int m = 0; m < F::FM; ++m)
#pragma unroll
    for (int n = 0; n < F::FN; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ti, tj;
        w_coords<BM, BN, WGM, WGN>(m, n, r, ti, tj);
        G[(j0 + tj) + (long)(i0 + ti) * d] = acc[m][n][r];  // G(i,j) at (row j, col i): upper
      }
}

// Row sums over K of the window.  COLMAJOR: element (i, k) at X[i + k d];
// otherwise at X[i K + k] (bf16 transposed window).
template <typename T, bool COLMAJOR>
DEV void rowsum_block(const T* __restrict__ X, int d, int K, int kchunk, int bx, int by, double* __restrict__ hpart) {
  __shared__ double red[4][64];
  const int kb = by * kchunk, ke = min(K, kb + kchunk);
  if (COLMAJOR) {
    const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int i = bx * 64 + r;
    double s = 0.0;
    if (i < d)
      for (int k = kb + q; k < ke; k += 4) s += (double)X[i + (long)k * d];
    red[q][r] = s;
    __syncthreads();
    if (threadIdx.x < 64 && i < d)
      hpart[(long)by * d + i] = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
  } else {
    // one row per wavefront, 4 rows per block
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = bx * 4 + w;
    if (i >= d) return;
    double s = 0.0;
    for (int k = kb + lane; k < ke; k += 64) s += (double)bf16_bits_to_f32(((const u16*)X)[(long)i * K + k]);
    s = wave_sum_f64(s);
    if (lane == 0) hpart[(long)by * d + i] = s;
  }
}

template <typename T, bool COLMAJOR>
__global__ __launch_bounds__(256) void k_rowsum(const T* __restrict__ X, int d, int K, int kchunk,
                                                double* __restrict__ hpart) {
  rowsum_block<T, COLMAJOR>(X, d, K, kchunk, blockIdx.x, blockIdx.y, hpart);
}

// col-major d x K bf16 -> row-major d x K (ld K)
__global__ __launch_bounds__(256) void k_transpose_bf16(const u16* __restrict__ in, u16* __restrict__ out, int d,
                                                        long K) {
  __shared__ u16 tile[64][66];
  const long k0 = (long)blockIdx.x * 64;
  const int i0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int kk = ty; kk < 64; kk += 4) {
    const long k = k0 + kk;
    const int i = i0 + tx;
    tile[kk][tx] = (k < K && i < d) ? in[i + k * d] : (u16)0;
  }
  __syncthreads();
  for (int ii = ty; ii < 64; ii += 4) {
    const int i = i0 + ii;
    const long k = k0 + tx;
    if (i < d && k < K) out[(long)i * K + k] = tile[tx][ii];
  }
}

// Transposition of the col-major d x K bf16 window into row-major (ld K) with
// the row sums over K taken on the way (whole 64 x 64 tiles: d and K multiples
// of 64).  Workgroup (bx, by) owns rows 64 bx .. 64 bx + 63 and the K range of
// chunk by; its four wavefronts take the chunk's 64-column tiles in turn.  In
// a tile, lane (g, q) = (lane % 8, lane / 8) reads columns 8 q .. 8 q + 7 of
// rows 8 g .. 8 g + 7 as eight 16-byte loads, transposes the 8 x 8 block in
// registers and writes it as eight 16-byte row pieces.  The bf16 values are
// summed in FP64 in a fixed order (exact while a row's values span less than
// 2^29 in magnitude: each has 8 significant bits).
DEV uint32_t pack_lo16(uint32_t a, uint32_t b) { return (a & 0xffffu) | (b << 16); }
DEV uint32_t pack_hi16(uint32_t a, uint32_t b) { return (a >> 16) | (b & 0xffff0000u); }

__global__ __launch_bounds__(256) void k_transpose_rowsum_bf16(const u16* __restrict__ in, u16* __restrict__ out,
                                                               int d, long K, long kchunk,
                                                               double* __restrict__ hpart) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane & 7, q = lane >> 3;
  const int i0 = blockIdx.x * 64 + 8 * g;
  const long kb = (long)blockIdx.y * kchunk, ke = kb + kchunk < K ? kb + kchunk : K;
  double hs[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) hs[r] = 0.0;
  for (long k0 = kb + 64 * w; k0 < ke; k0 += 256) {
    uint32_t v[8][4];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint4 x = *(const uint4*)(in + i0 + (k0 + 8 * q + j) * d);
      v[j][0] = x.x; v[j][1] = x.y; v[j][2] = x.z; v[j][3] = x.w;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int c = r >> 1;
      uint32_t o[4];
#pragma unroll
      for (int m = 0; m < 4; ++m)
        o[m] = (r & 1) ? pack_hi16(v[2 * m][c], v[2 * m + 1][c]) : pack_lo16(v[2 * m][c], v[2 * m + 1][c]);
      *(uint4*)(out + (long)(i0 + r) * K + k0 + 8 * q) = make_uint4(o[0], o[1], o[2], o[3]);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        hs[r] += (double)__uint_as_float((r & 1) ? (v[j][c] & 0xffff0000u) : (v[j][c] << 16));
    }
  }
  // lanes of one row group (same g) hold the sums of its eight column groups
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    double s = hs[r];
    s += lane_xor_f64<8>(s);
    s += lane_xor_f64<16>(s);
    s += lane_xor_f64<32>(s);
    if (q == 0) red[w][8 * g + r] = s;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    hpart[(long)blockIdx.y * d + i] = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                      (red[2][threadIdx.x] + red[3][threadIdx.x]);
  }
}

__global__ __launch_bounds__(256) void k_reduce_splits(const double* __restrict__ Gpart, int ns,
                                                       const double* __restrict__ hpart, int nh, int d,
                                                       double* __restrict__ G, double* __restrict__ h) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const long dd = (long)d * d;
  if (e < dd) {
    const int r = (int)(e % d), c = (int)(e / d);
    if (r <= c) {  // the scatter is stored in the upper triangle
      double g = 0.0;
      for (int q = 0; q < ns; ++q) g += Gpart[q * dd + e];
      G[e] = g;
    }
  }
  if (e < d) {
    double s = 0.0;
    for (int q = 0; q < nh; ++q) s += hpart[(long)q * d + e];
    h[e] = s;
  }
}

// Output tiles of the scatter: 64 x 64 lower pairs (f64/f32) or 128 x 64
// lower-covering tiles (bf16).
// bf16 windows whose tiles are whole take the direct-to-LDS kernel
static bool syrk_pl(int prec, int d, long K) { return prec == PMIX && d % 256 == 0 && K % 64 == 0; }

static int syrk_tiles(int prec, int d, long K) {
  if (prec != PMIX) return cdiv(d, 64) * (cdiv(d, 64) + 1) / 2;
  const int bi_rows = syrk_pl(prec, d, K) ? 256 : 128, bj_cols = bi_rows / 2;
  const int nbi = cdiv(d, bi_rows), nbj = cdiv(d, bj_cols);
  int n = 0;
  for (int b = 0; b < nbi; ++b) n += min(2 * b + 2, nbj);
  return n;
}

// K is split so that at least ~512 workgroups run; chunks are whole
// multiples of 64 columns (keeps the bf16 vector loads 16-byte aligned).
// FP32 chunks are whole multiples of the FP32 span FOLD_K: a window of at
// most FOLD_K samples is then one chunk, accumulated exactly as the grouped
// scatter of the batched form accumulates it (same FP32 sums, same FP64 fold).
static long syrk_kchunk(int prec, int d, long K) {
  const int nt = syrk_tiles(prec, d, K);
  int ns = cdiv(512, nt);
  const int maxs = (int)((K + 2047) / 2048);
  if (ns > maxs) ns = maxs;
  if (ns < 1) ns = 1;
  long kc = (K + ns - 1) / ns;
  if (prec == P32) return ((kc + FOLD_K - 1) / FOLD_K) * FOLD_K;
  return ((kc + 63) / 64) * 64;
}
static int syrk_splits(int prec, int d, long K) {
  const long kc = syrk_kchunk(prec, d, K);
  const long ns = (K + kc - 1) / kc;
  return ns < 1 ? 1 : (int)ns;
}

size_t syrk_scratch_bytes(int prec, int d, long K) {
  const int ns = syrk_splits(prec, d, K);
  return (size_t)ns * d * d * sizeof(double) + (size_t)64 * d * sizeof(double);
}

hipError_t syrk_window(Prec prec, const void* Xw, void* Xt, int d, long K, double* G, double* h, void* scratch,
                       hipStream_t s) {
  const int ns = syrk_splits(prec, d, K);
  const int kchunk = (int)syrk_kchunk(prec, d, K);
  double* Gpart = (double*)scratch;
  double* hpart = Gpart + (size_t)ns * d * d;
  // row sums: at most 64 K-chunks
  int nh = (int)((K + 4095) / 4096) < 64 ? (int)((K + 4095) / 4096) : 64;
  int hchunk = (int)((K + nh - 1) / nh);
  // the bf16 window is scattered from its row-major copy (K contiguous per
  // coordinate); whole tiles take the transposition with the row sums fused
  const void* Xs = Xw;
  bool h_done = false;
  if (prec == PMIX) {
    if (d % 64 == 0 && K % 64 == 0 && (uintptr_t)Xw % 16 == 0 && (uintptr_t)Xt % 16 == 0) {
      const long hc = (K / 64 + nh - 1) / nh * 64;
      nh = (int)((K + hc - 1) / hc);
      hchunk = (int)hc;
      hipLaunchKernelGGL(k_transpose_rowsum_bf16, dim3(d / 64, nh), dim3(256), 0, s, (const u16*)Xw, (u16*)Xt, d, K,
                         hc, hpart);
      h_done = true;
    } else {
      hipLaunchKernelGGL(k_transpose_bf16, dim3((unsigned)((K + 63) / 64), cdiv(d, 64)), dim3(256), 0, s,
                         (const u16*)Xw, (u16*)Xt, d, K);
    }
    Xs = Xt;
  }
  const int nt = syrk_tiles(prec, d, K);
  dim3 grid(nt, ns);
  if (syrk_pl(prec, d, K) && (uintptr_t)Xs % 16 == 0)
    hipLaunchKernelGGL(k_syrk_pl, grid, dim3(512), 0, s, (const u16*)Xs, d, (int)K, kchunk, Gpart);
  else if (prec == P64)
    hipLaunchKernelGGL((k_syrk_e<double, 16>), grid, dim3(256), 0, s, (const double*)Xs, d, (int)K, kchunk, Gpart);
  else if (prec == P32)
    hipLaunchKernelGGL((k_syrk_e<float, 32>), grid, dim3(256), 0, s, (const float*)Xs, d, (int)K, kchunk, Gpart);
  else {
    const int vec_ok = (K % 8 == 0) && ((uintptr_t)Xs % 16 == 0);
    hipLaunchKernelGGL(k_syrk_bf16, grid, dim3(256), 0, s, (const u16*)Xs, d, (int)K, kchunk, vec_ok, Gpart);
  }
  if (prec == P64)
    hipLaunchKernelGGL((k_rowsum<double, true>), dim3(cdiv(d, 64), nh), dim3(256), 0, s, (const double*)Xs, d, (int)K,
                       hchunk, hpart);
  else if (prec == P32)
    hipLaunchKernelGGL((k_rowsum<float, true>), dim3(cdiv(d, 64), nh), dim3(256), 0, s, (const float*)Xs, d, (int)K,
                       hchunk, hpart);
  else if (!h_done)
    hipLaunchKernelGGL((k_rowsum<u16, false>), dim3(cdiv(d, 4), nh), dim3(256), 0, s, (const u16*)Xs, d, (int)K,
                       hchunk, hpart);
  // reduce the splits in order into G (lower) and h
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_splits, dim3(cdiv((long)d * d, 256)), dim3(256), 0, s, Gpart, ns, hpart, nh, d, G, h);
  return hipGetLastError();
}

// ============================================================================
// moment fold (eqs. mom2g / mom1g with sample counts), covariance assembly
// ============================================================================
DEV void fold_mean_elem(const double* __restrict__ h, const double* __restrict__ sft, double N, double n,
                        double* __restrict__ m, int i) {
  m[i] = (N * m[i] + (h[i] + n * sft[i])) / (N + n);
}

DEV void fold_S_elem(const double* __restrict__ G, const double* __restrict__ h, const double* __restrict__ sft,
                     double N, double n, double* __restrict__ S, int d, long e) {
  const int i = (int)(e % d), j = (int)(e / d);
  const int a = i > j ? i : j, b = i > j ? j : i;
  const double g = G[b + (long)a * d];  // upper storage
  const double sxx = g + sft[a] * h[b] + h[a] * sft[b] + n * sft[a] * sft[b];
  S[e] = (N * S[e] + sxx) / (N + n);
}

__global__ __launch_bounds__(256) void k_fold_mean(const double* __restrict__ h, const double* __restrict__ sft, double N,
                                                   double n, double* __restrict__ m, int d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < d) fold_mean_elem(h, sft, N, n, m, i);
}

// fold_S_elem by 64 x 64 tiles of S: the scatter's upper-storage tile that
// holds the tile's values, G(min(i, j), max(i, j)), is read along its columns
// into LDS first, so the tiles below the diagonal do not read G at a stride
// of d (each element's arithmetic is fold_S_elem's).
__global__ __launch_bounds__(256) void k_fold_S(const double* __restrict__ G, const double* __restrict__ h,
                                                const double* __restrict__ sft, double N, double n,
                                                double* __restrict__ S, int d) {
  __shared__ double T[64][65];
  const int bx = blockIdx.x, by = blockIdx.y;
  const int r0 = 64 * min(bx, by), c0 = 64 * max(bx, by);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int c = ty; c < 64; c += 4) {
    const int r = r0 + tx, cc = c0 + c;
    T[tx][c] = (r < d && cc < d) ? G[r + (long)cc * d] : 0.0;
  }
  __syncthreads();
  for (int jj = ty; jj < 64; jj += 4) {
    const int i = 64 * bx + tx, j = 64 * by + jj;
    if (i < d && j < d) {
      const int a = i > j ? i : j, b = i > j ? j : i;
      const double g = T[b - r0][a - c0];
      const long e = i + (long)j * d;
      const double sxx = g + sft[a] * h[b] + h[a] * sft[b] + n * sft[a] * sft[b];
      S[e] = (N * S[e] + sxx) / (N + n);
    }
  }
}

hipError_t fold_moments(const double* G, const double* h, const double* sft, double N, long K, double* S, double* m,
                        int d, hipStream_t s) {
  hipLaunchKernelGGL(k_fold_S, dim3(cdiv(d, 64), cdiv(d, 64)), dim3(256), 0, s, G, h, sft, N, (double)K, S, d);
  hipLaunchKernelGGL(k_fold_mean, dim3(cdiv(d, 256)), dim3(256), 0, s, h, sft, N, (double)K, m, d);
  return hipGetLastError();
}

DEV void cov_elem(const double* __restrict__ S, const double* __restrict__ m, double eps, double* __restrict__ C,
                  int d, long e) {
  const int i = (int)(e % d), j = (int)(e / d);
  double v = 0.0;
  if (i >= j) {
    v = S[e] - m[i] * m[j];
    if (i == j) v += eps;
  }
  C[e] = v;
}

__global__ __launch_bounds__(256) void k_cov(const double* __restrict__ S, const double* __restrict__ m, double eps,
                                             double* __restrict__ C, int d) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < (long)d * d) cov_elem(S, m, eps, C, d, e);
}

DEV void trace_block(const double* __restrict__ S, const double* __restrict__ m, int d, double* __restrict__ tr) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) s += S[i + (long)i * d] - m[i] * m[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *tr = red[0];
}

__global__ __launch_bounds__(256) void k_trace(const double* __restrict__ S, const double* __restrict__ m, int d,
                                               double* __restrict__ tr) {
  trace_block(S, m, d, tr);
}

hipError_t cov_assemble(const double* S, const double* m, double eps, double* C, double* tr, int d, hipStream_t s) {
  hipLaunchKernelGGL(k_cov, dim3(cdiv((long)d * d, 256)), dim3(256), 0, s, S, m, eps, C, d);
  if (tr) hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, s, S, m, d, tr);
  return hipGetLastError();
}

// ============================================================================
// (e) blocked right-looking Cholesky, FP64, block 64.  Per block column:
//   k_chol_diag   one wavefront factors the 64 x 64 diagonal block with its
//                 rows in registers and forms the block's inverse;
//   k_chol_panel  MFMA: A_ij <- A_ij L_jj^-T as a product with that inverse;
//   k_chol_update_diag MFMA: trailing lower tiles A_ik -= A_ij A_kj^T, and
//                 the next diagonal block factored by the workgroup that
//                 updated it.
// ============================================================================

// Inverse of the lower-triangular 64 x 64 block held in Ls (row-major, LDS):
// lane c forms column c of L^-1 by forward substitution; x[] stays in
// registers (the loops are fully unrolled), Ls reads are broadcasts.
// rdiag[q] = 1 / Ls[q][q]; four partial sums break the dependency chain of
// each substitution step.
DEV void tri_inverse_col(const double (*Ls)[CHOL_NB + 1], const double* rdiag, double* x, int c) {
#pragma unroll
  for (int rr = 0; rr < CHOL_NB; ++rr) {
    double s[4] = {(rr == c) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < rr; ++q) s[q & 3] = __fma_rn(-Ls[rr][q], x[q], s[q & 3]);
    x[rr] = ((s[0] + s[1]) + (s[2] + s[3])) * rdiag[rr];
  }
}

// lane's value v broadcast from lane `src` (a compile-time lane after unrolling)
DEV double readlane_f64(double v, int src) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The diagonal block on a workgroup of four wavefronts.  Lane r of every
// wavefront holds row r; wavefront w holds columns 16 w .. 16 w + 15 of it.
// Column c is published through a double-buffered LDS vector; after one
// workgroup barrier every wavefront that owns columns right of c applies the
// rank-1 update to its part of each row, without per-element masks (entries
// right of the diagonal collect values that are never read).  Blocks of
// CHOL_CB columns with look-ahead: the wavefront owning the next block
// applies the block just published to that block first, factors its CB
// columns in turn (each updating the later ones of the block from its own
// registers and the pivot row's value by readlane) and publishes them before
// its other updates, so one barrier per CB columns separates consecutive
// blocks (per column in the earlier design: 20 to 9 us per 64 x 64 core,
// the factor bitwise unchanged).  The pivot step forms
// y ~ 1/sqrt(pivot) by the hardware reciprocal square root refined with two
// Newton-Raphson steps, then L(c, c) = pivot y and L(r, c) = a(r, c) y; a
// pivot that is not > 0 (or NaN) gives a diagonal that is not > 0.  Each
// entry of the lower triangle sees the updates in the same order as a
// right-looking factorisation.  The block inverse is formed as
// [[A, 0], [B, C]]^-1 = [[A^-1, 0], [-C^-1 B A^-1, C^-1]] twice: each
// wavefront inverts one 16 x 16 diagonal block by substitution (lane c a
// column), two wavefronts per 32 x 32 half combine two of them with two
// 16 x 16 products, then all four combine the halves (32 x 32 products).
// LDS: two buffers of CB columns, the factored block (whose zero upper
// triangle then holds the products' intermediate terms), the reciprocal
// diagonal, A^-1 and C^-1 of the 32 x 32 halves, the four 16 x 16 inverses.
constexpr int CHOL_DIAG_THREADS = 256;
constexpr int CHOL_CB = 4;  // columns factored per workgroup barrier
static_assert((CHOL_NB / 4) % CHOL_CB == 0, "a column block lies within one wavefront's columns");
constexpr int CHOL_DIAG_LDS =
    2 * CHOL_CB * CHOL_NB + CHOL_NB * (CHOL_NB + 1) + CHOL_NB + 2 * 32 * 33 + 4 * 16 * 17;  // doubles

// 1/sqrt(x): hardware estimate, then two Newton-Raphson steps
// y <- y + y (1 - x y^2) / 2 (NaN for x < 0 or NaN, +inf for x = 0)
DEV double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = __fma_rn(-x * y, y, 1.0);
    y = __fma_rn(0.5 * y, e, y);
  }
  return y;
}

// Column c (0 .. 15) of the inverse of the lower-triangular 16 x 16 block of
// Ls starting at (o, o), by forward substitution (four partial sums).
DEV void tri_inverse_col16(const double (*Ls)[CHOL_NB + 1], const double* rdiag, int o, double* x, int c) {
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    double s[4] = {(rr == c) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < rr; ++q) s[q & 3] = __fma_rn(-Ls[o + rr][o + q], x[q], s[q & 3]);
    x[rr] = ((s[0] + s[1]) + (s[2] + s[3])) * rdiag[o + rr];
  }
}

DEV void chol_diag_core(double* __restrict__ A, int d, int j0, int jn, double* __restrict__ Linv,
                        int* __restrict__ info, double* sh) {
  constexpr int H = CHOL_NB / 4;  // columns per wavefront
  double (*colp)[CHOL_CB][CHOL_NB] = (double (*)[CHOL_CB][CHOL_NB])sh;  // [parity][column of block][row]
  double (*Ls)[CHOL_NB + 1] = (double (*)[CHOL_NB + 1])(sh + 2 * CHOL_CB * CHOL_NB);
  double* rdiag = sh + 2 * CHOL_CB * CHOL_NB + CHOL_NB * (CHOL_NB + 1);
  double (*Ai)[33] = (double (*)[33])(rdiag + CHOL_NB);
  double (*Ci)[33] = Ai + 32;
  double (*Di)[16][17] = (double (*)[16][17])(Ai + 64);
  const int t = threadIdx.x, r = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  double a[H];
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const int c = w * H + k;
    double v = 0.0;
    if (r < jn && c < jn) {
      if (c <= r) v = A[(j0 + r) + (long)(j0 + c) * d];
    } else if (c == r) {
      v = 1.0;  // identity padding beyond the matrix edge
    }
    a[k] = v;
  }
  // pivot step of column c by the wavefront holding it (its local column kc)
  auto pivot = [&](int c, int kc, double* dst) {
    const double piv = readlane_f64(a[kc], c);
    const double y = rsqrt_nr(piv);
    const double l = (r == c) ? piv * y : a[kc] * y;
    a[kc] = l;
    dst[r] = (r >= c) ? l : 0.0;
  };
  // the owner of block (n .. n + CB - 1) factors its columns in turn, each
  // updating the later ones of the block from its own registers and the
  // pivot row's value (readlane), and publishes them
  auto own_block = [&](int n, int buf) {
    const int k0 = n % H;
#pragma unroll
    for (int t = 0; t < CHOL_CB; ++t) {
      pivot(n + t, k0 + t, colp[buf][t]);
      const double lt = (r >= n + t) ? a[k0 + t] : 0.0;
#pragma unroll
      for (int u = t + 1; u < CHOL_CB; ++u) a[k0 + u] = __fma_rn(-lt, readlane_f64(a[k0 + t], n + u), a[k0 + u]);
    }
  };
  if (w == 0) own_block(0, 0);
#pragma unroll
  for (int q = 0; q < CHOL_NB / CHOL_CB; ++q) {
    const int c0 = CHOL_CB * q, wc = c0 / H, n0 = c0 + CHOL_CB, wn = n0 / H;
    const int buf = q & 1;
    __syncthreads();
    if (n0 < CHOL_NB && w == wn) {
      // owner of the next block: the published block applied to its columns,
      // that block factored and published, then the rest of its columns
      double lb[CHOL_CB];
#pragma unroll
      for (int t = 0; t < CHOL_CB; ++t) lb[t] = colp[buf][t][r];
      const int k0 = n0 % H;
#pragma unroll
      for (int u = 0; u < CHOL_CB; ++u)
#pragma unroll
        for (int t = 0; t < CHOL_CB; ++t) a[k0 + u] = __fma_rn(-lb[t], colp[buf][t][n0 + u], a[k0 + u]);
      own_block(n0, buf ^ 1);
#pragma unroll
      for (int k = (wn == wc) ? k0 + CHOL_CB : CHOL_CB; k < H; ++k)
#pragma unroll
        for (int t = 0; t < CHOL_CB; ++t) a[k] = __fma_rn(-lb[t], colp[buf][t][w * H + k], a[k]);
    } else if (w > wc) {
      double lb[CHOL_CB];
#pragma unroll
      for (int t = 0; t < CHOL_CB; ++t) lb[t] = colp[buf][t][r];
#pragma unroll
      for (int k = 0; k < H; ++k)
#pragma unroll
        for (int t = 0; t < CHOL_CB; ++t) a[k] = __fma_rn(-lb[t], colp[buf][t][w * H + k], a[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const int c = w * H + k;
    if (r < jn && c < jn) A[(j0 + r) + (long)(j0 + c) * d] = (c <= r) ? a[k] : 0.0;
    Ls[r][c] = (c <= r) ? a[k] : 0.0;
  }
  __syncthreads();
  if (w == 0) {
    // a pivot that is not > 0 (or NaN) leaves a diagonal root that is not > 0,
    // and every later pivot inherits the failure: the first bad column is the
    // lowest such lane
    const double diag = Ls[r][r];
    const unsigned long long bad = __ballot(r < jn && !(diag > 0.0));
    if (r == 0 && bad && *info == 0) *info = j0 + __ffsll((long long)bad);
    rdiag[r] = 1.0 / diag;
  }
  __syncthreads();
  // the inverses of the four 16 x 16 diagonal blocks, one per wavefront
  // (lane c < 16: column c, by substitution; zeros above the diagonal)
  if (r < 16) {
    double x[16];
    tri_inverse_col16(Ls, rdiag, 16 * w, x, r);
#pragma unroll
    for (int q = 0; q < 16; ++q) Di[w][q][r] = x[q];
  }
  __syncthreads();
  // the two 32 x 32 halves, [[D0, 0], [E, D1]]^-1 = [[D0^-1, 0], [-D1^-1 E
  // D0^-1, D1^-1]], half hh on wavefronts 2 hh and 2 hh + 1: thread u forms
  // row u / 8, columns 2 (u % 8) .. + 1 of T = E D0^-1 into the factor's zero
  // block Ls[o + i][o + 16 + j], then of -D1^-1 T, and copies its share of
  // the diagonal blocks and the zero block into A^-1 (hh = 0) or C^-1
  {
    const int hh = w >> 1, u = t & 127, o = 32 * hh;
    const int ui = u >> 3, uj = (u & 7) * 2;
    double (*Dst)[33] = hh ? Ci : Ai;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double e = Ls[o + 16 + ui][o + k];
      s0 = __fma_rn(e, Di[2 * hh][k][uj], s0);
      s1 = __fma_rn(e, Di[2 * hh][k][uj + 1], s1);
    }
    Ls[o + ui][o + 16 + uj] = s0;
    Ls[o + ui][o + 16 + uj + 1] = s1;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      Dst[ui][uj + e] = Di[2 * hh][ui][uj + e];
      Dst[16 + ui][16 + uj + e] = Di[2 * hh + 1][ui][uj + e];
      Dst[ui][16 + uj + e] = 0.0;
    }
  }
  __syncthreads();
  {
    const int hh = w >> 1, u = t & 127, o = 32 * hh;
    const int ui = u >> 3, uj = (u & 7) * 2;
    double (*Dst)[33] = hh ? Ci : Ai;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double g = Di[2 * hh + 1][ui][k];
      s0 = __fma_rn(-g, Ls[o + k][o + 16 + uj], s0);
      s1 = __fma_rn(-g, Ls[o + k][o + 16 + uj + 1], s1);
    }
    Dst[16 + ui][uj] = s0;
    Dst[16 + ui][uj + 1] = s1;
  }
  __syncthreads();
  // T = B A^-1 (B = rows 32 .. 63, columns 0 .. 31 of L; A^-1 lower) into
  // Ls[i][32 + j] (rows 0 .. 31 of the factor's zero columns 32 .. 63):
  // thread t forms row t / 8, columns 4 (t % 8) .. 4 (t % 8) + 3
  const int ti = t >> 3, tj = (t & 7) * 4;
  {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const double bq = Ls[32 + ti][q];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] = __fma_rn(bq, Ai[q][tj + e], acc[e]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) Ls[ti][32 + tj + e] = acc[e];
  }
  __syncthreads();
  // lower-left block of the inverse: -C^-1 T (C^-1 lower)
  double xl[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    const double cq = Ci[ti][q];
#pragma unroll
    for (int e = 0; e < 4; ++e) xl[e] = __fma_rn(-cq, Ls[q][32 + tj + e], xl[e]);
  }
  // inverse out, column-major: Linv[q + c 64] = (L^-1)(q, c).  Thread t
  // writes its lower-left entries from registers, then the other three blocks
  // (A^-1, the zero block, C^-1) from LDS in coalesced column runs
#pragma unroll
  for (int e = 0; e < 4; ++e) Linv[(32 + ti) + (tj + e) * CHOL_NB] = xl[e];
#pragma unroll
  for (int k = 0; k < CHOL_NB * CHOL_NB / CHOL_DIAG_THREADS; ++k) {
    const int e = t + k * CHOL_DIAG_THREADS;
    const int q = e & (CHOL_NB - 1), c = e >> 6;
    if (c < 32) {
      if (q < 32) Linv[e] = Ai[q][c];
    } else {
      Linv[e] = (q < 32) ? 0.0 : Ci[q - 32][c - 32];
    }
  }
}

DEV void chol_diag_block(double* __restrict__ A, int d, int j0, int jn, double* __restrict__ Linv,
                         int* __restrict__ info) {
  __shared__ double sh[CHOL_DIAG_LDS];
  chol_diag_core(A, d, j0, jn, Linv, info, sh);
}

__global__ __launch_bounds__(CHOL_DIAG_THREADS) void k_chol_diag(double* __restrict__ A, int d, int j0, int jn,
                                                                 double* __restrict__ Linv, int* __restrict__ info) {
  chol_diag_block(A, d, j0, jn, Linv, info);
}

// Inverses of all (already factored) diagonal blocks of L, one wave per block.
DEV void tri_inv_block(const double* __restrict__ L, int d, double* __restrict__ Linv, int bx) {
  __shared__ double Ls[CHOL_NB][CHOL_NB + 1];
  __shared__ double rdiag[CHOL_NB];
  const int r = threadIdx.x, j0 = bx * CHOL_NB, jn = min(CHOL_NB, d - j0);
#pragma unroll
  for (int c = 0; c < CHOL_NB; ++c) {
    double v = (c == r) ? 1.0 : 0.0;
    if (r < jn && c < jn) v = (c <= r) ? L[(j0 + r) + (long)(j0 + c) * d] : 0.0;
    Ls[r][c] = v;
  }
  __syncthreads();
  rdiag[r] = 1.0 / Ls[r][r];
  __syncthreads();
  double x[CHOL_NB];
  tri_inverse_col(Ls, rdiag, x, r);
  double* out = Linv + (long)bx * CHOL_NB * CHOL_NB;
#pragma unroll
  for (int q = 0; q < CHOL_NB; ++q) out[q + r * CHOL_NB] = x[q];
}

__global__ __launch_bounds__(64) void k_tri_inv(const double* __restrict__ L, int d, double* __restrict__ Linv) {
  tri_inv_block(L, d, Linv, blockIdx.x);
}

// Panel rows below the diagonal block: A(i, j0 + c) <- sum_q A(i, j0 + q) Linv(c, q)
DEV void chol_panel_tile(double* __restrict__ A, int d, int j0, int jn, const double* __restrict__ Linv, int bx) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ double lds[e_lds_elems<double, BM, BN, BK>()];
  const int i0 = j0 + jn + bx * BM;
  EFrag<double, BM, BN> f;
  f.zero();
  e_gemm<double, BM, BN, BK, false, false>(f, A + (long)j0 * d, d, d, Linv, CHOL_NB, jn, i0, 0, 0, jn, lds);
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ti, tj;
        frag_coords<BM, BN, double>(m, n, r, ti, tj);
        const int i = i0 + ti;
        if (i < d && tj < jn) A[i + (long)(j0 + tj) * d] = f.c[m][n][r];
      }
}

__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ A, int d, int j0, int jn,
                                                    const double* __restrict__ Linv) {
  chol_panel_tile(A, d, j0, jn, Linv, blockIdx.x);
}

// Trailing update A(i, k) -= sum_c A(i, c) A(k, c) over the panel columns,
// for the lower tiles of block rows/cols >= t0.
constexpr int CHOL_UPD_LDS = e_lds_elems<double, 64, 64, 16>();  // doubles

DEV void chol_update_core(double* __restrict__ A, int d, int j0, int jn, int t0, int t, double* lds) {
  constexpr int BM = 64, BN = 64, BK = 16;
  int bi, bk;
  tile_pair(t, bi, bk);
  const int i0 = (t0 + bi) * BM, k0 = (t0 + bk) * BN;
  const double* Pc = A + (long)j0 * d;
  EFrag<double, BM, BN> f;
  f.zero();
  e_gemm<double, BM, BN, BK, false, false>(f, Pc, d, d, Pc, d, d, i0, k0, 0, jn, lds);
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ti, tj;
        frag_coords<BM, BN, double>(m, n, r, ti, tj);
        const int i = i0 + ti, k = k0 + tj;
        if (i < d && k < d) A[i + (long)k * d] -= f.c[m][n][r];
      }
}

DEV void chol_update_tile(double* __restrict__ A, int d, int j0, int jn, int t0, int t) {
  __shared__ double lds[CHOL_UPD_LDS];
  chol_update_core(A, d, j0, jn, t0, t, lds);
}

size_t chol_scratch_bytes(int d) { return (size_t)cdiv(d, CHOL_NB) * CHOL_NB * CHOL_NB * sizeof(double); }

// Trailing update of block column j0 fused with the factorisation of the
// next diagonal block: workgroup 0 updates tile (t0, t0), the first of the
// row-by-row enumeration, which is that diagonal block, and then factors it
// while the other workgroups finish the update.  The barrier at the start of
// the factorisation orders the tile's stores before its loads (one
// workgroup); nothing else reads the block before the next launch.
// Both phases use the same LDS buffer.
__global__ __launch_bounds__(256) void k_chol_update_diag(double* __restrict__ A, int d, int j0, int jn, int t0,
                                                          double* __restrict__ Linv_next, int* __restrict__ info) {
  constexpr int NLDS = CHOL_UPD_LDS > CHOL_DIAG_LDS ? CHOL_UPD_LDS : CHOL_DIAG_LDS;
  __shared__ double lds[NLDS];
  chol_update_core(A, d, j0, jn, t0, blockIdx.x, lds);
  if (blockIdx.x == 0) {
    __syncthreads();
    const int j1 = t0 * CHOL_NB;
    chol_diag_core(A, d, j1, min(CHOL_NB, d - j1), Linv_next, info, lds);
  }
}

hipError_t potrf(double* A, int d, int* info, double* Linv, hipStream_t s) {
  const int nb = cdiv(d, CHOL_NB);
  hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(CHOL_DIAG_THREADS), 0, s, A, d, 0, min(CHOL_NB, d), Linv, info);
  for (int jb = 0; jb + 1 < nb; ++jb) {
    const int j0 = jb * CHOL_NB, jn = CHOL_NB;
    const double* Li = Linv + (long)jb * CHOL_NB * CHOL_NB;
    const int m = nb - jb - 1;
    hipLaunchKernelGGL(k_chol_panel, dim3(m), dim3(256), 0, s, A, d, j0, jn, Li);
    hipLaunchKernelGGL(k_chol_update_diag, dim3(m * (m + 1) / 2), dim3(256), 0, s, A, d, j0, jn, jb + 1,
                       Linv + (long)(jb + 1) * CHOL_NB * CHOL_NB, info);
  }
  return hipGetLastError();
}

DEV void round_factor_elem(int prec, double* __restrict__ L, void* __restrict__ Llow, int d, long e) {
  const int i = (int)(e % d), j = (int)(e / d);
  const double v = (i >= j) ? L[e] : 0.0;
  if (prec == P32) {
    const float f = (float)v;
    L[e] = (double)f;
    ((float*)Llow)[e] = f;
  } else {
    // L~ = hi + lo, both bf16, row-major copies (k-contiguous for the MFMA)
    const u16 hi = f32_to_bf16_bits((float)v);
    const double rem = v - (double)bf16_bits_to_f32(hi);
    const u16 lo = f32_to_bf16_bits((float)rem);
    L[e] = (double)bf16_bits_to_f32(hi) + (double)bf16_bits_to_f32(lo);
    ((u16*)Llow)[(long)i * d + j] = hi;
    ((u16*)Llow)[(long)d * d + (long)i * d + j] = lo;
  }
}

__global__ __launch_bounds__(256) void k_round_factor(int prec, double* __restrict__ L, void* __restrict__ Llow, int d) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < (long)d * d) round_factor_elem(prec, L, Llow, d, e);
}

// The mixed form's rounding by 64 x 64 tiles: the column-major factor is
// read and written back along its columns, and the row-major hi and lo
// copies leave through an LDS transpose along their rows (each element's
// arithmetic is round_factor_elem's).
__global__ __launch_bounds__(256) void k_round_factor_hl(double* __restrict__ L, u16* __restrict__ Llow, int d) {
  __shared__ u16 th[64][66], tl[64][66];  // [column][row] of the tile
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int jj = ty; jj < 64; jj += 4) {
    const int i = i0 + tx, j = j0 + jj;
    u16 hi = 0, lo = 0;
    if (i < d && j < d) {
      const long e = i + (long)j * d;
      const double v = (i >= j) ? L[e] : 0.0;
      hi = f32_to_bf16_bits((float)v);
      const double rem = v - (double)bf16_bits_to_f32(hi);
      lo = f32_to_bf16_bits((float)rem);
      L[e] = (double)bf16_bits_to_f32(hi) + (double)bf16_bits_to_f32(lo);
    }
    th[jj][tx] = hi;
    tl[jj][tx] = lo;
  }
  __syncthreads();
  for (int ii = ty; ii < 64; ii += 4) {
    const int i = i0 + ii, j = j0 + tx;
    if (i < d && j < d) {
      Llow[(long)i * d + j] = th[tx][ii];
      Llow[(long)d * d + (long)i * d + j] = tl[tx][ii];
    }
  }
}

hipError_t round_factor(Prec prec, double* L, void* Llow, int d, hipStream_t s) {
  if (prec == P64) return hipSuccess;
  if (prec == PMIX)
    hipLaunchKernelGGL(k_round_factor_hl, dim3(cdiv(d, 64), cdiv(d, 64)), dim3(256), 0, s, L, (u16*)Llow, d);
  else
    hipLaunchKernelGGL(k_round_factor, dim3(cdiv((long)d * d, 256)), dim3(256), 0, s, (int)prec, L, Llow, d);
  return hipGetLastError();
}

// ============================================================================
// Potential scale reduction factor (Section 2.4.2, eqs. winco, btwco, psrf,
// M = 1).  Per chain p and coordinate i the running mean and the sum of
// squared deviations of the visited states, merged window by window from the
// window store (state = pivot of the window + stored shift, in the store's
// precision) with the pairwise update of Chan, Golub and LeVeque (1979), so
// no raw second moment is ever formed.
// ============================================================================
// V consecutive stored values from element e (e a multiple of V; V = 1, 2 or 4)
template <int PR, int V>
DEV void load_win_v(const void* win, long e, double* v) {
  if (V == 1) {
    if (PR == P64) v[0] = ((const double*)win)[e];
    else if (PR == P32) v[0] = (double)((const float*)win)[e];
    else v[0] = (double)bf16_bits_to_f32(((const u16*)win)[e]);
  } else if (V == 2) {
    if (PR == P64) {
      const double2 a = *(const double2*)((const double*)win + e);
      v[0] = a.x; v[1] = a.y;
    } else if (PR == P32) {
      const float2 a = *(const float2*)((const float*)win + e);
      v[0] = a.x; v[1] = a.y;
    } else {
      const uint32_t a = *(const uint32_t*)((const u16*)win + e);
      v[0] = (double)bf16_bits_to_f32((u16)(a & 0xffff));
      v[1] = (double)bf16_bits_to_f32((u16)(a >> 16));
    }
  } else if (PR == P64) {
    const double2 a = *(const double2*)((const double*)win + e), b = *(const double2*)((const double*)win + e + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  } else if (PR == P32) {
    const float4 a = *(const float4*)((const float*)win + e);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  } else {
    const uint2 a = *(const uint2*)((const u16*)win + e);
    v[0] = (double)bf16_bits_to_f32((u16)(a.x & 0xffff));
    v[1] = (double)bf16_bits_to_f32((u16)(a.x >> 16));
    v[2] = (double)bf16_bits_to_f32((u16)(a.y & 0xffff));
    v[3] = (double)bf16_bits_to_f32((u16)(a.y >> 16));
  }
}

// elements e = i + d p, V consecutive coordinates of one chain per thread
// (V = 4 needs d % 4 == 0); window column of chain p at step t: p + P t
template <int PR, int V>
__global__ __launch_bounds__(256) void k_psrf_acc(const void* __restrict__ win, int d, int P, int nw,
                                                  const double* __restrict__ xr, double n0, double* __restrict__ mean,
                                                  double* __restrict__ m2) {
  const long e0 = ((long)blockIdx.x * 256 + threadIdx.x) * V;
  if (e0 >= (long)d * P) return;
  const int i0 = (int)(e0 % d), p = (int)(e0 / d);
  double s1[V], s2[V];
#pragma unroll
  for (int k = 0; k < V; ++k) s1[k] = s2[k] = 0.0;
  // loads of 16 steps in flight per thread for 4-wide rows (measured best at
  // d = 4096, P = 256: 71 % of the HBM peak), 4 for single coordinates
  constexpr int UNR = V == 4 ? 16 : 4;
#pragma unroll UNR
  for (int t = 0; t < nw; ++t) {
    double v[V];
    load_win_v<PR, V>(win, i0 + (long)(p + (long)P * t) * d, v);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      s1[k] += v[k];
      s2[k] = __fma_rn(v[k], v[k], s2[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const long e = e0 + k;
    const double mw = s1[k] / nw;
    const double qw = __fma_rn(-s1[k], mw, s2[k]);  // sum over the window of (v - mw)^2
    const double xm = xr[i0 + k] + mw;              // the window's mean state
    if (n0 == 0.0) {
      mean[e] = xm;
      m2[e] = qw;
    } else {
      const double nt = n0 + (double)nw;
      const double delta = xm - mean[e];
      mean[e] = __fma_rn(delta, (double)nw / nt, mean[e]);
      m2[e] = m2[e] + qw + delta * delta * (n0 * (double)nw / nt);
    }
  }
}

template <int PR>
static void psrf_acc_launch(const void* win, int d, int P, int nw, const double* xr, double n0, double* mean,
                            double* m2, hipStream_t s) {
  const long n = (long)d * P;
  if (d % 4 == 0 && (uintptr_t)win % 16 == 0)
    hipLaunchKernelGGL((k_psrf_acc<PR, 4>), dim3(cdiv(n / 4, 256)), dim3(256), 0, s, win, d, P, nw, xr, n0, mean, m2);
  else
    hipLaunchKernelGGL((k_psrf_acc<PR, 1>), dim3(cdiv(n, 256)), dim3(256), 0, s, win, d, P, nw, xr, n0, mean, m2);
}

hipError_t psrf_accumulate(Prec prec, const void* win, int d, int P, int nw, const double* xr, double n0, double* mean,
                           double* m2, hipStream_t s) {
  if (prec == P64) psrf_acc_launch<P64>(win, d, P, nw, xr, n0, mean, m2, s);
  else if (prec == P32) psrf_acc_launch<P32>(win, d, P, nw, xr, n0, mean, m2, s);
  else psrf_acc_launch<PMIX>(win, d, P, nw, xr, n0, mean, m2, s);
  return hipGetLastError();
}

// out[i] = sqrt(R_i): B_i = n/(P-1) sum_p (m^p - mbar)_i^2 with mbar the mean
// of the chain means, W_i = sum_p m2[i, p] / ((n - 1) P) (the average of the
// chains' 1/n variances times n/(n-1)), R_i = (n-1)/n + (P+1)/(P n) B_i/W_i.
__global__ __launch_bounds__(256) void k_psrf_final(const double* __restrict__ mean, const double* __restrict__ m2,
                                                    int d, int P, double n, double* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= d) return;
  double sm = 0.0, sq = 0.0;
  for (int p = 0; p < P; ++p) {
    sm += mean[i + (long)p * d];
    sq += m2[i + (long)p * d];
  }
  const double mbar = sm / P;
  double sb = 0.0;
  for (int p = 0; p < P; ++p) {
    const double u = mean[i + (long)p * d] - mbar;
    sb = __fma_rn(u, u, sb);
  }
  const double B = n / (double)(P - 1) * sb;
  const double W = sq / ((n - 1.0) * (double)P);
  const double R = (n - 1.0) / n + (double)(P + 1) / ((double)P * n) * (B / W);
  out[i] = sqrt(R);
}

hipError_t psrf_finalize(const double* mean, const double* m2, int d, int P, double n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_psrf_final, dim3(cdiv(d, 256)), dim3(256), 0, s, mean, m2, d, P, n, out);
  return hipGetLastError();
}

// ---- whitening Z = L^-1 (X - xr) ------------------------------------------
DEV void sub_ref_elem(const double* __restrict__ X, const double* __restrict__ xr, double* __restrict__ Z, int d,
                      long e) {
  Z[e] = X[e] - xr[e % d];
}

__global__ __launch_bounds__(256) void k_sub_ref(const double* __restrict__ X, const double* __restrict__ xr,
                                                 double* __restrict__ Z, int d, int P) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < (long)d * P) sub_ref_elem(X, xr, Z, d, e);
}

// Z_j <- Linv_jj Z_j (in place: each workgroup reads its 64 x 64 column
// block completely before writing it back)
DEV void trsm_diag_tile(const double* __restrict__ Linv, double* __restrict__ Z, int d, int P, int j0, int jn, int bx) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ double lds[e_lds_elems<double, BM, BN, BK>()];
  const int p0 = bx * BN;
  EFrag<double, BM, BN> f;
  f.zero();
  e_gemm<double, BM, BN, BK, false, true>(f, Linv, CHOL_NB, jn, Z + j0, d, P, 0, p0, 0, jn, lds);
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ti, tj;
        frag_coords<BM, BN, double>(m, n, r, ti, tj);
        const int p = p0 + tj;
        if (ti < jn && p < P) Z[(j0 + ti) + (long)p * d] = f.c[m][n][r];
      }
}

__global__ __launch_bounds__(256) void k_trsm_diag(const double* __restrict__ Linv, double* __restrict__ Z, int d, int P,
                                                   int j0, int jn) {
  trsm_diag_tile(Linv, Z, d, P, j0, jn, blockIdx.x);
}

// Z_i -= L_ij Z_j for row blocks below j
DEV void trsm_update_tile(const double* __restrict__ L, double* __restrict__ Z, int d, int P, int j0, int jn, int bx,
                          int by) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ double lds[e_lds_elems<double, BM, BN, BK>()];
  const int i0 = j0 + jn + bx * BM, p0 = by * BN;
  EFrag<double, BM, BN> f;
  f.zero();
  e_gemm<double, BM, BN, BK, false, true>(f, L + (long)j0 * d, d, d, Z + j0, d, P, i0, p0, 0, jn, lds);
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ti, tj;
        frag_coords<BM, BN, double>(m, n, r, ti, tj);
        const int i = i0 + ti, p = p0 + tj;
        if (i < d && p < P) Z[i + (long)p * d] -= f.c[m][n][r];
      }
}

// The update of block column j fused with the diagonal solve of block j + 1:
// the first row tile of the update is that block, so the workgroup that
// finishes it applies Linv_{j+1} to its own column tile at once (the barrier
// orders the tile's stores before the solve's loads in one workgroup; no
// other workgroup touches that tile before the next launch).
__global__ __launch_bounds__(256) void k_trsm_update_diag(const double* __restrict__ L, double* __restrict__ Z, int d,
                                                          int P, int j0, int jn, const double* __restrict__ Linv_next) {
  trsm_update_tile(L, Z, d, P, j0, jn, blockIdx.x, blockIdx.y);
  if (blockIdx.x == 0) {
    __syncthreads();
    const int j1 = j0 + jn;
    trsm_diag_tile(Linv_next, Z, d, P, j1, min(CHOL_NB, d - j1), blockIdx.y);
  }
}

DEV void colnorm_block(const double* __restrict__ Z, int d, double* __restrict__ zq, int p) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    const double z = Z[i + (long)p * d];
    s = __fma_rn(z, z, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) zq[p] = red[0];
}

__global__ __launch_bounds__(256) void k_colnorm(const double* __restrict__ Z, int d, double* __restrict__ zq) {
  colnorm_block(Z, d, zq, blockIdx.x);
}

hipError_t trsm_whiten(const double* L, const double* X, const double* xr, double* Z, double* zq, double* Linv, int d,
                       int P, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_ref, dim3(cdiv((long)d * P, 256)), dim3(256), 0, s, X, xr, Z, d, P);
  const int nb = cdiv(d, CHOL_NB);
  hipLaunchKernelGGL(k_tri_inv, dim3(nb), dim3(64), 0, s, L, d, Linv);
  // block 0's solve, then per block column the update fused with the next block's solve
  hipLaunchKernelGGL(k_trsm_diag, dim3(cdiv(P, 64)), dim3(256), 0, s, (const double*)Linv, Z, d, P, 0,
                     min(CHOL_NB, d));
  for (int jb = 0; jb < nb; ++jb) {
    const int j0 = jb * CHOL_NB, jn = min(CHOL_NB, d - j0);
    const int rem = d - (j0 + jn);
    if (rem > 0)
      hipLaunchKernelGGL(k_trsm_update_diag, dim3(cdiv(rem, 64), cdiv(P, 64)), dim3(256), 0, s, L, Z, d, P, j0, jn,
                         (const double*)(Linv + (long)(jb + 1) * CHOL_NB * CHOL_NB));
  }
  if (zq) hipLaunchKernelGGL(k_colnorm, dim3(P), dim3(256), 0, s, Z, d, zq);
  return hipGetLastError();
}

// ---- batches of independent factorisations and whitenings -------------------
// One problem per blockIdx.z (the per-chain pairs of the local-global
// logistics), through the same device cores as potrf / trsm_whiten, so every
// problem's arithmetic is bitwise that of a separate call.  Problem z owns A
// + z sA, Linv + z sL, info[z]; the whitening works on column z of X and Z.
// skip (whitening): problem z is left untouched when skip[z] != 0.
__global__ __launch_bounds__(CHOL_DIAG_THREADS) void kb_chol_diag(double* __restrict__ A, long sA, int d, int j0, int jn,
                                                   double* __restrict__ Linv, long sL, int* __restrict__ info) {
  const int z = blockIdx.z;
  chol_diag_block(A + z * sA, d, j0, jn, Linv + z * sL, info + z);
}

__global__ __launch_bounds__(256) void kb_chol_panel(double* __restrict__ A, long sA, int d, int j0, int jn,
                                                     const double* __restrict__ Linv, long sL) {
  const int z = blockIdx.z;
  chol_panel_tile(A + z * sA, d, j0, jn, Linv + z * sL, blockIdx.x);
}

__global__ __launch_bounds__(256) void kb_chol_update_diag(double* __restrict__ A, long sA, int d, int j0, int jn,
                                                           int t0, double* __restrict__ Linv_next, long sL,
                                                           int* __restrict__ info) {
  constexpr int NLDS = CHOL_UPD_LDS > CHOL_DIAG_LDS ? CHOL_UPD_LDS : CHOL_DIAG_LDS;
  __shared__ double lds[NLDS];
  const int z = blockIdx.z;
  double* Az = A + z * sA;
  chol_update_core(Az, d, j0, jn, t0, blockIdx.x, lds);
  if (blockIdx.x == 0) {
    __syncthreads();
    const int j1 = t0 * CHOL_NB;
    chol_diag_core(Az, d, j1, min(CHOL_NB, d - j1), Linv_next + z * sL, info + z, lds);
  }
}

hipError_t potrf_batched(double* A, long sA, int d, int* info, double* Linv, long sL, int nprob, hipStream_t s) {
  if (nprob < 1 || nprob > 65535) return hipErrorInvalidValue;
  const int nb = cdiv(d, CHOL_NB);
  hipLaunchKernelGGL(kb_chol_diag, dim3(1, 1, nprob), dim3(CHOL_DIAG_THREADS), 0, s, A, sA, d, 0, min(CHOL_NB, d),
                     Linv, sL, info);
  for (int jb = 0; jb + 1 < nb; ++jb) {
    const int j0 = jb * CHOL_NB, jn = CHOL_NB;
    const int m = nb - jb - 1;
    hipLaunchKernelGGL(kb_chol_panel, dim3(m, 1, nprob), dim3(256), 0, s, A, sA, d, j0, jn,
                       (const double*)(Linv + (long)jb * CHOL_NB * CHOL_NB), sL);
    hipLaunchKernelGGL(kb_chol_update_diag, dim3(m * (m + 1) / 2, 1, nprob), dim3(256), 0, s, A, sA, d, j0, jn,
                       jb + 1, Linv + (long)(jb + 1) * CHOL_NB * CHOL_NB, sL, info);
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void kb_sub_ref(const double* __restrict__ X, const double* __restrict__ xrp,
                                                  double* __restrict__ Z, int d, int P, const int* __restrict__ skip) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < (long)d * P && !skip[e / d]) Z[e] = X[e] - xrp[e];
}

__global__ __launch_bounds__(64) void kb_tri_inv(const double* __restrict__ L, long sA, int d,
                                                 double* __restrict__ Linv, long sL, const int* __restrict__ skip) {
  const int z = blockIdx.z;
  if (skip[z]) return;
  tri_inv_block(L + z * sA, d, Linv + z * sL, blockIdx.x);
}

__global__ __launch_bounds__(256) void kb_trsm_diag(const double* __restrict__ Linv, long sL, double* __restrict__ Z,
                                                    int d, int j0, int jn, const int* __restrict__ skip) {
  const int z = blockIdx.z;
  if (skip[z]) return;
  trsm_diag_tile(Linv + z * sL, Z + (long)z * d, d, 1, j0, jn, 0);
}

__global__ __launch_bounds__(256) void kb_trsm_update(const double* __restrict__ L, long sA, double* __restrict__ Z,
                                                      int d, int j0, int jn, const int* __restrict__ skip) {
  const int z = blockIdx.z;
  if (skip[z]) return;
  trsm_update_tile(L + z * sA, Z + (long)z * d, d, 1, j0, jn, blockIdx.x, 0);
}

__global__ __launch_bounds__(256) void kb_colnorm(const double* __restrict__ Z, int d, double* __restrict__ zq,
                                                  const int* __restrict__ skip) {
  if (skip[blockIdx.x]) return;
  colnorm_block(Z, d, zq, blockIdx.x);
}

hipError_t trsm_whiten_batched(const double* L, long sA, const double* X, const double* xrp, double* Z, double* zq,
                               double* Linv, long sL, int d, int P, const int* skip, hipStream_t s) {
  if (P < 1 || P > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kb_sub_ref, dim3(cdiv((long)d * P, 256)), dim3(256), 0, s, X, xrp, Z, d, P, skip);
  const int nb = cdiv(d, CHOL_NB);
  hipLaunchKernelGGL(kb_tri_inv, dim3(nb, 1, P), dim3(64), 0, s, L, sA, d, Linv, sL, skip);
  for (int jb = 0; jb < nb; ++jb) {
    const int j0 = jb * CHOL_NB, jn = min(CHOL_NB, d - j0);
    hipLaunchKernelGGL(kb_trsm_diag, dim3(1, 1, P), dim3(256), 0, s,
                       (const double*)(Linv + (long)jb * CHOL_NB * CHOL_NB), sL, Z, d, j0, jn, skip);
    const int rem = d - (j0 + jn);
    if (rem > 0) hipLaunchKernelGGL(kb_trsm_update, dim3(cdiv(rem, 64), 1, P), dim3(256), 0, s, L, sA, Z, d, j0, jn, skip);
  }
  hipLaunchKernelGGL(kb_colnorm, dim3(P), dim3(256), 0, s, Z, d, zq, skip);
  return hipGetLastError();
}

// ============================================================================
// random numbers: Philox4x32-10 counters (stream 0 = W, 1 + g = U stage g)
// ============================================================================
// Four FP32 normals from counter ctr of the stream (Box-Muller on the four
// 24-bit uniforms of one Philox block).
DEV void normals4_f32(uint32_t k0, uint32_t k1, uint64_t ctr, float* v) {
  const u4_t r = philox4x32_10({(uint32_t)ctr, (uint32_t)(ctr >> 32), 0u, 0u}, k0, k1);
  const float ua = u01_f32(r.x), ub = u01_f32(r.y), uc = u01_f32(r.z), ud = u01_f32(r.w);
  const float ra = sqrtf(-2.0f * logf(ua)), rc = sqrtf(-2.0f * logf(uc));
  float s1, c1, s2, c2;
  sincosf(6.28318530717958647692f * ub, &s1, &c1);
  sincosf(6.28318530717958647692f * ud, &s2, &c2);
  v[0] = ra * c1;
  v[1] = ra * s1;
  v[2] = rc * c2;
  v[3] = rc * s2;
}

__global__ __launch_bounds__(256) void k_normals(int prec, uint32_t k0, uint32_t k1, long g0, long total,
                                                 void* __restrict__ W, void* __restrict__ Wlo) {
  const long stride = (long)gridDim.x * 256;
  const long gid = (long)blockIdx.x * 256 + threadIdx.x;
  if (prec == P64) {
    for (long q = gid; 2 * q < total; q += stride) {
      const uint64_t ctr = (uint64_t)(g0 + 2 * q);
      const u4_t r = philox4x32_10({(uint32_t)ctr, (uint32_t)(ctr >> 32), 0u, 0u}, k0, k1);
      const double u1 = u01_f64(r.x, r.y), u2 = u01_f64(r.z, r.w);
      const double rad = sqrt(-2.0 * log(u1));
      double sn, cs;
      sincos(6.283185307179586476925286766559 * u2, &sn, &cs);
      double* w = (double*)W;
      w[2 * q] = rad * cs;
      if (2 * q + 1 < total) w[2 * q + 1] = rad * sn;
    }
  } else {
    const bool vec = (uintptr_t)W % 16 == 0 && (prec == P32 || (uintptr_t)Wlo % 8 == 0);
    for (long q = gid; 4 * q < total; q += stride) {
      float v[4];
      normals4_f32(k0, k1, (uint64_t)(g0 + 4 * q), v);
      if (4 * q + 3 < total && vec) {
        // the thread's four values as one 16-byte (FP32) or two 8-byte stores
        if (prec == P32) {
          *(float4*)((float*)W + 4 * q) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
          u16 hi[4], lo[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) split_bf16(v[e], hi[e], lo[e]);
          *(uint2*)((u16*)W + 4 * q) = make_uint2(hi[0] | ((uint32_t)hi[1] << 16), hi[2] | ((uint32_t)hi[3] << 16));
          *(uint2*)((u16*)Wlo + 4 * q) = make_uint2(lo[0] | ((uint32_t)lo[1] << 16), lo[2] | ((uint32_t)lo[3] << 16));
        }
        continue;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long idx = 4 * q + e;
        if (idx < total) {
          if (prec == P32) {
            ((float*)W)[idx] = v[e];
          } else {
            u16 hi, lo;
            split_bf16(v[e], hi, lo);
            ((u16*)W)[idx] = hi;
            ((u16*)Wlo)[idx] = lo;
          }
        }
      }
    }
  }
}

hipError_t normals(Prec prec, uint64_t seed, long s0, int n, int d, int P, void* W, void* Wlo, hipStream_t s) {
  const long total = (long)n * P * d;
  if (total <= 0) return hipSuccess;
  const long per = (prec == P64) ? 2 : 4;
  long nq = (total + per - 1) / per;
  int blocks = (int)((nq + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_normals, dim3(blocks), dim3(256), 0, s, (int)prec, (uint32_t)seed, (uint32_t)(seed >> 32),
                     s0 * (long)P * d, total, W, Wlo);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_uniforms(uint32_t k0, uint32_t k1, long s0, int n, int P, int stages,
                                                  double* __restrict__ U) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const long total = (long)n * stages * P;
  if (e >= total) return;
  const int p = (int)(e % P);
  const long tg = e / P;
  const int g = (int)(tg % stages);
  const long t = tg / stages;
  const uint64_t st = (uint64_t)(s0 + t);
  const u4_t r = philox4x32_10({(uint32_t)st, (uint32_t)(st >> 32), 1u + (uint32_t)g, (uint32_t)(p >> 1)}, k0, k1);
  U[e] = (p & 1) ? u01_f64(r.z, r.w) : u01_f64(r.x, r.y);
}

hipError_t uniforms(uint64_t seed, long s0, int n, int P, int stages, double* U, hipStream_t s) {
  const long total = (long)n * stages * P;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_uniforms, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (uint32_t)seed,
                     (uint32_t)(seed >> 32), s0, n, P, stages, U);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_convert_normals(int prec, const double* __restrict__ W64, long count,
                                                         void* __restrict__ W, void* __restrict__ Wlo) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  const float f = (float)W64[e];
  if (prec == P32) {
    ((float*)W)[e] = f;
  } else {
    u16 hi, lo;
    split_bf16(f, hi, lo);
    ((u16*)W)[e] = hi;
    ((u16*)Wlo)[e] = lo;
  }
}

hipError_t convert_normals(Prec prec, const double* W64, long count, void* W, void* Wlo, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert_normals, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, (int)prec, W64, count,
                     W, Wlo);
  return hipGetLastError();
}

// ============================================================================
// (c) accept / reject of step t fused with the proposal of step t+1.
// One wavefront per (chain, 512-row chunk); the chain's decision is formed
// redundantly by every wavefront of that chain from the same partial sums in
// the same order, so all of them agree bitwise.
// ============================================================================
template <int PR> struct StepT;
template <> struct StepT<P64> { typedef double XI; typedef double WT; typedef double VT; typedef double WIN; };
template <> struct StepT<P32> { typedef float XI; typedef float WT; typedef float VT; typedef float WIN; };
template <> struct StepT<PMIX> { typedef float XI; typedef u16 WT; typedef float VT; typedef u16 WIN; };

template <int PR>
DEV double load_w(const void* w, const void* wlo, long e) {
  if (PR == P64) return ((const double*)w)[e];
  if (PR == P32) return (double)((const float*)w)[e];
  return (double)bf16_bits_to_f32(((const u16*)w)[e]) + (double)bf16_bits_to_f32(((const u16*)wlo)[e]);
}

template <int PR>
DEV void store_win(void* win, long e, double v) {
  if (PR == P64) ((double*)win)[e] = v;
  else if (PR == P32) ((float*)win)[e] = (float)v;
  else ((u16*)win)[e] = f32_to_bf16_bits((float)v);
}

constexpr int MAXPROJ = 4;

// chunk ch of nch (STEP_RCH rows each) of chains 4 pq .. 4 pq + 3, one wave each.
// MODE 0: decision and state update in one pass (every chunk's wave
// recomputes its chain's decision); MODE 1: decision only (one wave per
// chain, ch = 0), written to acc_out and the per-chain scalars; MODE 2: state
// update and next proposal only, reading the decision from acc_out.
template <int PR, int MODE = 0>
DEV void step_body(const StepArgs& a, int ch, int nch, int pq) {
  typedef typename StepT<PR>::XI XI;
  typedef typename StepT<PR>::VT VT;
  constexpr int RPL = STEP_RCH / 64;  // rows per lane
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p = pq * 4 + w;
  if (p >= a.P) return;
  const int d = a.d, P = a.P;
  const int r0 = ch * STEP_RCH;
  const XI* xi_cur = (const XI*)a.xi_cur;
  const XI* xi_nxt = (const XI*)a.xi_nxt;
  VT* V = (VT*)a.V;
  // issue every row load of this lane first; the chain's decision (which
  // needs two reductions and a log) overlaps their latency
  double x[RPL], z[RPL], xr[RPL], xc[RPL], wc[RPL], xn[RPL], wn[RPL], mu[RPL];
  bool in[RPL];
#pragma unroll
  for (int q = 0; q < RPL && MODE != 1; ++q) {
    const int i = r0 + q * 64 + lane;
    in[q] = i < d;
    const long e = i + (long)p * d;
    x[q] = z[q] = xr[q] = xc[q] = wc[q] = xn[q] = wn[q] = mu[q] = 0.0;
    if (in[q]) {
      x[q] = a.X[e];
      z[q] = a.Z[e];
      xr[q] = a.xr[i];
      const long ew = i + (long)p * (a.ldw ? a.ldw : d);
      if (a.do_accept) {
        xc[q] = (double)xi_cur[ew];
        wc[q] = load_w<PR>(a.w_cur, a.wlo_cur, ew);
      }
      if (a.do_propose) {
        xn[q] = (double)xi_nxt[ew];
        wn[q] = load_w<PR>(a.w_nxt, a.wlo_nxt, ew);
        mu[q] = a.mu ? a.mu[i] : 0.0;
      }
    }
  }
  bool acc = false;
  if (MODE == 2 && a.do_accept) acc = a.acc_out[p] != 0;
  if (MODE != 2 && a.do_accept) {
    // exact log density of the proposal: target partials (of this chain, or
    // of its survivor slot under delayed acceptance) plus the prior
    const bool live = !a.da || a.pass1[p];
    const int col = a.da ? a.slot[p] : p;
    double s = 0.0;
    if (live)
      for (int q = lane; q < a.nrb; q += 64) s += a.lpp_part[(long)col * a.nrb + q];
    s = wave_sum_f64(s);
    if (a.prior_w > 0.0) {
      double pq = 0.0;
      for (int q = lane; q < nch; q += 64) pq += a.pq_part_cur[(long)p * nch + q];
      pq = wave_sum_f64(pq);
      s = __fma_rn(-a.prior_w, pq, s);
    }
    const double lpp = s;
    double zs = 0.0;
    for (int q = lane; q < nch; q += 64) zs += a.zq_part_cur[(long)p * nch + q];
    zs = wave_sum_f64(zs);
    const double lp = a.lp_cur[p], zq = a.zq_cur[p];
    double la;
    if (!a.da) {
      la = (lpp + zs * a.inv2a2) - (lp + zq * a.inv2a2);
      acc = log(a.u[p]) < la;  // NaN compares false: rejected
    } else {
      // second stage: log alpha_2 = (log pi(x') - log pi(x)) - (s(x') - s(x)),
      // with s = r - |z|^2/(2 alpha^2) in the residual form (r = network)
      double l2 = (lpp - lp) - (a.s_new[p] - a.s_in[p]);
      if (a.da_resid) l2 += (zs - zq) * a.inv2a2;
      la = live ? l2 : -INFINITY;
      acc = live && (log(a.u2[p]) < la);
    }
    if (ch == 0 && lane == 0) {
      a.lp_nxt[p] = acc ? lpp : lp;
      a.zq_nxt[p] = acc ? zs : zq;
      a.nacc[p] += acc ? 1 : 0;
      if (a.wacc) a.wacc[p] += acc ? 1 : 0;
      a.la_out[p] = la;
      a.acc_out[p] = acc ? 1 : 0;
      if (a.da) a.s_out[p] = acc ? a.s_new[p] : a.s_in[p];
      if (a.trace_lp) a.trace_lp[p] = acc ? lpp : lp;
      if (live && isinf(lpp) && lpp > 0.0) atomicOr(a.err, 1);
    }
  }
  if (MODE == 1) return;
  double zacc = 0.0, xacc = 0.0;
  double pacc[MAXPROJ] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    if (!in[q]) continue;
    const int i = r0 + q * 64 + lane;
    const long e = i + (long)p * d;
    double xv = x[q], zv = z[q];
    if (a.do_accept) {
      if (acc) {
        xv = propose1(xr[q], xv, a.rho, xc[q]);
        zv = __fma_rn(a.c, wc[q], a.rho * zv);
        a.X[e] = xv;
        a.Z[e] = zv;
      }
      store_win<PR>(a.win, i + (a.win_col0 + p) * (long)d, xv - xr[q]);
      for (int k = 0; k < a.nproj; ++k) pacc[k] = __fma_rn(a.proj[i + (long)k * d], xv, pacc[k]);
    }
    if (a.do_propose) {
      const double xp = propose1(xr[q], xv, a.rho, xn[q]);
      if (a.vh) {
        u16 h, l;
        const double sv = (xp - mu[q]) * (double)a.vsc[i];
        if (fabs(sv) >= H2_RANGE) atomicOr(a.err, 2);
        split_f16(sv, h, l);
        a.vh[e] = h;
        a.vh[(long)d * P + e] = l;
      } else {
        const long ev = i + (long)p * (a.ldv ? a.ldv : d);
        if (a.v32) ((float*)a.V)[ev] = (float)(xp - mu[q]);
        else V[ev] = (VT)(xp - mu[q]);
      }
      const double zp = __fma_rn(a.c, wn[q], a.rho * zv);
      zacc = __fma_rn(zp, zp, zacc);
      xacc = __fma_rn(xp, xp, xacc);
    }
  }
  if (a.do_propose) {
    zacc = wave_sum_f64(zacc);
    if (lane == 0) a.zq_part_nxt[(long)p * nch + ch] = zacc;
    if (a.prior_w > 0.0) {
      xacc = wave_sum_f64(xacc);
      if (lane == 0) a.pq_part_nxt[(long)p * nch + ch] = xacc;
    }
  }
  if (a.do_accept && a.nproj > 0) {
    for (int k = 0; k < a.nproj; ++k) {
      const double v = wave_sum_f64(pacc[k]);
      if (lane == 0) a.proj_part[((long)ch * a.nproj + k) * P + p] = v;
    }
  }
}

// Sum over the 256 threads of a workgroup in a fixed order (every thread
// gets the result).  red: 4 doubles of LDS.
DEV double block_sum_f64(double v, double* red) {
  v = wave_sum_f64(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Stopping errors of the experiments (Section 3.3): |S - m m^T - Sigma|_F^2,
// |Sigma|_F^2 and |m - mu|^2, as per-block FP64 partial sums (fixed order)
// reduced by one more block: deterministic (MERR_BLOCKS in kernels.h).

__global__ __launch_bounds__(256) void k_moment_err(const double* __restrict__ S, const double* __restrict__ m,
                                                    const double* __restrict__ Sigma, const double* __restrict__ mu,
                                                    int d, double* __restrict__ part) {
  __shared__ double red[4];
  const long n = (long)d * d;
  double a = 0.0, b = 0.0, c = 0.0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const int i = (int)(e % d), j = (int)(e / d);
    const double sg = Sigma[e];
    const double u = (S[e] - m[i] * m[j]) - sg;
    a = __fma_rn(u, u, a);
    b = __fma_rn(sg, sg, b);
  }
  if (mu)
    for (int i = blockIdx.x * 256 + threadIdx.x; i < d; i += gridDim.x * 256) {
      const double u = m[i] - mu[i];
      c = __fma_rn(u, u, c);
    }
  a = block_sum_f64(a, red);
  b = block_sum_f64(b, red);
  c = block_sum_f64(c, red);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = a;
    part[3 * blockIdx.x + 1] = b;
    part[3 * blockIdx.x + 2] = c;
  }
}

__global__ __launch_bounds__(256) void k_moment_err_final(const double* __restrict__ part, int nb,
                                                          double* __restrict__ out) {
  __shared__ double red[4];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) {
    a += part[3 * k];
    b += part[3 * k + 1];
    c += part[3 * k + 2];
  }
  a = block_sum_f64(a, red);
  b = block_sum_f64(b, red);
  c = block_sum_f64(c, red);
  if (threadIdx.x == 0) {
    out[0] = sqrt(a / b);
    out[1] = sqrt(c);
  }
}

size_t moment_err_scratch_bytes() { return MERR_SCRATCH_DOUBLES * sizeof(double); }

hipError_t moment_error(const double* S, const double* m, const double* Sigma, const double* mu, int d, double* scratch,
                        hipStream_t s) {
  const int nb = min(MERR_BLOCKS, cdiv((long)d * d, 256));
  hipLaunchKernelGGL(k_moment_err, dim3(nb), dim3(256), 0, s, S, m, Sigma, mu, d, scratch + 2);
  hipLaunchKernelGGL(k_moment_err_final, dim3(1), dim3(256), 0, s, (const double*)(scratch + 2), nb, scratch);
  return hipGetLastError();
}


// Decision of chain p by one workgroup of 256 threads: the target partials
// (thousands of row blocks for the logistic target) are summed by all
// threads, then MH (or the second stage of delayed acceptance) decides.
DEV void decide_block(const StepArgs& a, int nch, int p) {
  __shared__ double red[4];
  const int t = threadIdx.x;
  const bool live = !a.da || a.pass1[p];
  const int col = a.da ? a.slot[p] : p;
  double s = 0.0;
  if (live)
    for (int q = t; q < a.nrb; q += 256) s += a.lpp_part[(long)col * a.nrb + q];
  s = block_sum_f64(s, red);
  if (a.prior_w > 0.0) {
    double pq = 0.0;
    for (int q = t; q < nch; q += 256) pq += a.pq_part_cur[(long)p * nch + q];
    pq = block_sum_f64(pq, red);
    s = __fma_rn(-a.prior_w, pq, s);
  }
  const double lpp = s;
  double zs = 0.0;
  for (int q = t; q < nch; q += 256) zs += a.zq_part_cur[(long)p * nch + q];
  zs = block_sum_f64(zs, red);
  if (t != 0) return;
  const double lp = a.lp_cur[p], zq = a.zq_cur[p];
  double la;
  bool acc;
  if (!a.da) {
    la = (lpp + zs * a.inv2a2) - (lp + zq * a.inv2a2);
    acc = log(a.u[p]) < la;  // NaN compares false: rejected
  } else {
    // second stage: log alpha_2 = (log pi(x') - log pi(x)) - (s(x') - s(x)),
    // with s = r - |z|^2/(2 alpha^2) in the residual form (r = network)
    double l2 = (lpp - lp) - (a.s_new[p] - a.s_in[p]);
    if (a.da_resid) l2 += (zs - zq) * a.inv2a2;
    la = live ? l2 : -INFINITY;
    acc = live && (log(a.u2[p]) < la);
  }
  a.lp_nxt[p] = acc ? lpp : lp;
  a.zq_nxt[p] = acc ? zs : zq;
  a.nacc[p] += acc ? 1 : 0;
  if (a.wacc) a.wacc[p] += acc ? 1 : 0;
  a.la_out[p] = la;
  a.acc_out[p] = acc ? 1 : 0;
  if (a.da) a.s_out[p] = acc ? a.s_new[p] : a.s_in[p];
  if (a.trace_lp) a.trace_lp[p] = acc ? lpp : lp;
  if (live && isinf(lpp) && lpp > 0.0) atomicOr(a.err, 1);
}

__global__ __launch_bounds__(256) void k_decide(StepArgs a, int nch) { decide_block(a, nch, blockIdx.x); }

// The decision of chain p taken by one wavefront inside the update launch
// (no delayed acceptance; at most 64 target row blocks and 64 row chunks).
// With that many partials decide_block's block sums reduce to wave 0's
// shuffle sum plus exact zeros, so these sums, log alpha and the verdict are
// bitwise decide_block's.  Every row-chunk workgroup of the chain takes the
// (cheap, L2-resident) decision; only `write` stores its outputs.
// parts: the chain's nrb target partials (global memory or LDS).
// The decision's inputs other than the target's row-block terms, all written
// by earlier launches: this lane's z-norm (and prior) partial of the
// proposal, the current state's log pi and z-norm, and the uniform.  A kernel
// that waits for the target's terms can load these first.
struct DecIn {
  double zs, pq, lp, zq, u;
};

DEV DecIn decide_inputs(const StepArgs& a, int nch, int p) {
  const int lane = threadIdx.x & 63;
  DecIn in;
  in.zs = lane < nch ? 0.0 + a.zq_part_cur[(long)p * nch + lane] : 0.0;
  in.pq = (a.prior_w > 0.0 && lane < nch) ? 0.0 + a.pq_part_cur[(long)p * nch + lane] : 0.0;
  in.lp = a.lp_cur[p];
  in.zq = a.zq_cur[p];
  in.u = a.u[p];
  return in;
}

DEV bool decide_wave(const StepArgs& a, int nch, int p, bool write, const double* parts, const DecIn& in) {
  const int lane = threadIdx.x & 63;
  double s = lane < a.nrb ? 0.0 + parts[lane] : 0.0;
  s = wave_sum_f64(s);
  if (a.prior_w > 0.0) {
    const double pq = wave_sum_f64(in.pq);
    s = __fma_rn(-a.prior_w, pq, s);
  }
  const double lpp = s;
  const double zs = wave_sum_f64(in.zs);
  const double lp = in.lp, zq = in.zq;
  const double la = (lpp + zs * a.inv2a2) - (lp + zq * a.inv2a2);
  const bool acc = log(in.u) < la;  // NaN compares false: rejected
  if (write && lane == 0) {
    a.lp_nxt[p] = acc ? lpp : lp;
    a.zq_nxt[p] = acc ? zs : zq;
    a.nacc[p] += acc ? 1 : 0;
    if (a.wacc) a.wacc[p] += acc ? 1 : 0;
    a.la_out[p] = la;
    a.acc_out[p] = acc ? 1 : 0;
    if (a.trace_lp) a.trace_lp[p] = acc ? lpp : lp;
    if (isinf(lpp) && lpp > 0.0) atomicOr(a.err, 1);
  }
  return acc;
}

DEV bool decide_wave(const StepArgs& a, int nch, int p, bool write, const double* parts) {
  return decide_wave(a, nch, p, write, parts, decide_inputs(a, nch, p));
}

// Paired-row loads and stores for the update half (d even, so that every
// chain's column starts on an even element): lane l owns rows 2l, 2l + 1 of
// its 128-row chunk and moves them with 16-, 8- or 4-byte accesses.
// 128-row chunks per wavefront of the update (two: half the wavefronts take
// the same decision; one or four ran slower at d = 4096, P = 256)
#ifndef STEP_CPW
#define STEP_CPW 2
#endif
template <int PR> struct Pair2;
template <> struct Pair2<P64> { typedef double2 XI; typedef double2 W; };
template <> struct Pair2<P32> { typedef float2 XI; typedef float2 W; };
template <> struct Pair2<PMIX> { typedef float2 XI; typedef uint32_t W; };

template <int PR>
DEV void store_win2(void* win, long e, double v0, double v1) {
  if (PR == P64) {
    *(double2*)((double*)win + e) = make_double2(v0, v1);
  } else if (PR == P32) {
    *(float2*)((float*)win + e) = make_float2((float)v0, (float)v1);
  } else {
    *(uint32_t*)((u16*)win + e) = (uint32_t)f32_to_bf16_bits((float)v0) | ((uint32_t)f32_to_bf16_bits((float)v1) << 16);
  }
}

// The update of chain p over row chunks CPW cb .. CPW cb + CPW - 1 (STEP_RCH
// rows each; chunks past nch are skipped), one wavefront, in two phases:
// upd_load issues every load that does not depend on the chain's decision
// (keeping the raw bits, so nothing waits for them there), upd_finish takes
// the decision, loads the accepted proposal's Xi and W for every chunk
// before it converts any, and stores.  One partial per chunk, so the partials are those of one chunk
// per wavefront whatever CPW is.
// A row pair of a proposal's Xi and W as loaded (both bf16 parts of W in the
// mixed form); the conversion to double (raw_xi, raw_w; W = hi + lo in the
// mixed form) is left to where the values are used, so that the loads stay
// in flight until then instead of being waited for at once.
template <int PR> struct Raw2;
template <> struct Raw2<P64> { double2 xi, w; };
template <> struct Raw2<P32> { float2 xi, w; };
template <> struct Raw2<PMIX> { float2 xi; uint32_t wh, wl; };

DEV void raw_zero(Raw2<P64>& r) { r.xi = make_double2(0.0, 0.0); r.w = make_double2(0.0, 0.0); }
DEV void raw_zero(Raw2<P32>& r) { r.xi = make_float2(0.f, 0.f); r.w = make_float2(0.f, 0.f); }
DEV void raw_zero(Raw2<PMIX>& r) { r.xi = make_float2(0.f, 0.f); r.wh = r.wl = 0u; }

DEV void raw_load(Raw2<P64>& r, const void* xi, const void* w, const void*, long e) {
  r.xi = *(const double2*)((const double*)xi + e);
  r.w = *(const double2*)((const double*)w + e);
}
DEV void raw_load(Raw2<P32>& r, const void* xi, const void* w, const void*, long e) {
  r.xi = *(const float2*)((const float*)xi + e);
  r.w = *(const float2*)((const float*)w + e);
}
DEV void raw_load(Raw2<PMIX>& r, const void* xi, const void* w, const void* wlo, long e) {
  r.xi = *(const float2*)((const float*)xi + e);
  r.wh = *(const uint32_t*)((const u16*)w + e);
  r.wl = *(const uint32_t*)((const u16*)wlo + e);
}

DEV void raw_xi(const Raw2<P64>& r, double& v0, double& v1) { v0 = r.xi.x; v1 = r.xi.y; }
DEV void raw_xi(const Raw2<P32>& r, double& v0, double& v1) { v0 = r.xi.x; v1 = r.xi.y; }
DEV void raw_xi(const Raw2<PMIX>& r, double& v0, double& v1) { v0 = r.xi.x; v1 = r.xi.y; }
DEV void raw_w(const Raw2<P64>& r, double& w0, double& w1) { w0 = r.w.x; w1 = r.w.y; }
DEV void raw_w(const Raw2<P32>& r, double& w0, double& w1) { w0 = r.w.x; w1 = r.w.y; }
DEV void raw_w(const Raw2<PMIX>& r, double& w0, double& w1) {
  w0 = (double)bf16_bits_to_f32((u16)(r.wh & 0xffff)) + (double)bf16_bits_to_f32((u16)(r.wl & 0xffff));
  w1 = (double)bf16_bits_to_f32((u16)(r.wh >> 16)) + (double)bf16_bits_to_f32((u16)(r.wl >> 16));
}

template <int PR, int CPW>
struct UpdRegs {
  int ii[CPW];
  bool in[CPW];
  double x0[CPW], x1[CPW], z0[CPW], z1[CPW], r0[CPW], r1[CPW];
  double m0[CPW], m1[CPW];
  Raw2<PR> nw[CPW];  // the next proposal's Xi and W
  float2 sv[CPW];
};

template <int PR, int CPW>
DEV void upd_load(const StepArgs& a, int p, int cb, int nch, UpdRegs<PR, CPW>& g) {
  const int lane = threadIdx.x & 63;
  const int d = a.d;
  const long ldw = a.ldw ? a.ldw : d;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int ch = cb * CPW + c;
    g.ii[c] = ch * STEP_RCH + 2 * lane;
    g.in[c] = ch < nch && g.ii[c] < d;  // d even: the pair lies wholly inside or outside
    g.x0[c] = g.x1[c] = g.z0[c] = g.z1[c] = g.r0[c] = g.r1[c] = 0.0;
    g.m0[c] = g.m1[c] = 0.0;
    raw_zero(g.nw[c]);
    g.sv[c] = make_float2(0.f, 0.f);
    if (g.in[c]) {
      const int i = g.ii[c];
      const long e = i + (long)p * d, ew = i + (long)p * ldw;
      const double2 xv = *(const double2*)(a.X + e), zv = *(const double2*)(a.Z + e);
      const double2 rv = *(const double2*)(a.xr + i);
      g.x0[c] = xv.x; g.x1[c] = xv.y; g.z0[c] = zv.x; g.z1[c] = zv.y; g.r0[c] = rv.x; g.r1[c] = rv.y;
      if (a.do_propose) {
        raw_load(g.nw[c], a.xi_nxt, a.w_nxt, a.wlo_nxt, ew);
        if (a.mu) {
          const double2 mv = *(const double2*)(a.mu + i);
          g.m0[c] = mv.x; g.m1[c] = mv.y;
        }
        if (a.vh) g.sv[c] = *(const float2*)(a.vsc + i);
      }
    }
  }
}

template <int PR, int CPW>
DEV void upd_finish(const StepArgs& a, int p, int cb, int nch, bool acc, const UpdRegs<PR, CPW>& g) {
  const int lane = threadIdx.x & 63;
  const int d = a.d, P = a.P;
  const long ldw = a.ldw ? a.ldw : d;
  Raw2<PR> cw[CPW];  // the accepted proposal's Xi and W
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    raw_zero(cw[c]);
    if (g.in[c] && acc) raw_load(cw[c], a.xi_cur, a.w_cur, a.wlo_cur, g.ii[c] + (long)p * ldw);
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int ch = cb * CPW + c;
    if (ch >= nch) break;
    const int i = g.ii[c];
    const long e = i + (long)p * d;
    double zacc = 0.0, xacc = 0.0;
    double pacc[MAXPROJ] = {0.0, 0.0, 0.0, 0.0};
    if (g.in[c]) {
      double xa = g.x0[c], xb = g.x1[c], za = g.z0[c], zb = g.z1[c];
      const double ra = g.r0[c], rb = g.r1[c];
      if (a.do_accept) {
        if (acc) {
          double c0, c1, wc0, wc1;
          raw_xi(cw[c], c0, c1);
          raw_w(cw[c], wc0, wc1);
          xa = propose1(ra, xa, a.rho, c0);
          xb = propose1(rb, xb, a.rho, c1);
          za = __fma_rn(a.c, wc0, a.rho * za);
          zb = __fma_rn(a.c, wc1, a.rho * zb);
          *(double2*)(a.X + e) = make_double2(xa, xb);
          *(double2*)(a.Z + e) = make_double2(za, zb);
        }
        store_win2<PR>(a.win, i + (a.win_col0 + p) * (long)d, xa - ra, xb - rb);
        for (int k = 0; k < a.nproj; ++k) {
          const double2 pv = *(const double2*)(a.proj + i + (long)k * d);
          pacc[k] = __fma_rn(pv.y, xb, __fma_rn(pv.x, xa, pacc[k]));
        }
      }
      if (a.do_propose) {
        double n0, n1, wn0, wn1;
        raw_xi(g.nw[c], n0, n1);
        raw_w(g.nw[c], wn0, wn1);
        const double xp0 = propose1(ra, xa, a.rho, n0), xp1 = propose1(rb, xb, a.rho, n1);
        if (a.vh) {
          u16 h0, l0, h1, l1;
          const double s0 = (xp0 - g.m0[c]) * (double)g.sv[c].x, s1 = (xp1 - g.m1[c]) * (double)g.sv[c].y;
          if (fmax(fabs(s0), fabs(s1)) >= H2_RANGE) atomicOr(a.err, 2);
          split_f16(s0, h0, l0);
          split_f16(s1, h1, l1);
          *(uint32_t*)(a.vh + e) = (uint32_t)h0 | ((uint32_t)h1 << 16);
          *(uint32_t*)(a.vh + (long)d * P + e) = (uint32_t)l0 | ((uint32_t)l1 << 16);
        } else {
          const long ev = i + (long)p * (a.ldv ? a.ldv : d);
          if (a.v32 || PR != P64)
            *(float2*)((float*)a.V + ev) = make_float2((float)(xp0 - g.m0[c]), (float)(xp1 - g.m1[c]));
          else *(double2*)((double*)a.V + ev) = make_double2(xp0 - g.m0[c], xp1 - g.m1[c]);
        }
        const double zp0 = __fma_rn(a.c, wn0, a.rho * za), zp1 = __fma_rn(a.c, wn1, a.rho * zb);
        zacc = __fma_rn(zp1, zp1, __fma_rn(zp0, zp0, 0.0));
        xacc = __fma_rn(xp1, xp1, __fma_rn(xp0, xp0, 0.0));
      }
    }
    if (a.do_propose) {
      zacc = wave_sum_f64(zacc);
      if (lane == 0) a.zq_part_nxt[(long)p * nch + ch] = zacc;
      if (a.prior_w > 0.0) {
        xacc = wave_sum_f64(xacc);
        if (lane == 0) a.pq_part_nxt[(long)p * nch + ch] = xacc;
      }
    }
    if (a.do_accept && a.nproj > 0) {
      for (int k = 0; k < a.nproj; ++k) {
        const double v = wave_sum_f64(pacc[k]);
        if (lane == 0) a.proj_part[((long)ch * a.nproj + k) * P + p] = v;
      }
    }
  }
}

// The update of chain 4 pq + (wave) over the chunks of cb.
template <int PR, int CPW = 1>
DEV void step_update2(const StepArgs& a, int cb, int nch, int pq) {
  const int w = threadIdx.x >> 6;
  const int p = pq * 4 + w;
  if (p >= a.P) return;
  UpdRegs<PR, CPW> g;
  upd_load<PR, CPW>(a, p, cb, nch, g);
  const bool acc =
      a.do_accept && (a.fuse_dec ? decide_wave(a, nch, p, cb == 0, a.lpp_part + (long)p * a.nrb) : a.acc_out[p] != 0);
  upd_finish<PR, CPW>(a, p, cb, nch, acc, g);
}

// The update half of k_step_h2, where every 128-row chunk lies inside d (d a
// multiple of 256, two chunks per wavefront), the target's mean and the
// proposal's scales are set, and PROP tells whether the step proposes.  Its
// loads are issued without branches and kept raw, so the compiler keeps them
// in flight until their first use (the shared upd_load and upd_finish wait
// for each chunk's loads at the branches that guard them); the arithmetic and
// the stores are those of upd_finish.
template <bool PROP>
DEV void upd_load_h2(const StepArgs& a, int p, int cb, UpdRegs<PMIX, 2>& g) {
  const int lane = threadIdx.x & 63;
  const int d = a.d;
  const long ldw = a.ldw ? a.ldw : d;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int i = (cb * 2 + c) * STEP_RCH + 2 * lane;
    g.ii[c] = i;
    g.in[c] = true;
    const long e = i + (long)p * d, ew = i + (long)p * ldw;
    const double2 xv = *(const double2*)(a.X + e), zv = *(const double2*)(a.Z + e);
    const double2 rv = *(const double2*)(a.xr + i);
    g.x0[c] = xv.x; g.x1[c] = xv.y; g.z0[c] = zv.x; g.z1[c] = zv.y; g.r0[c] = rv.x; g.r1[c] = rv.y;
    if (PROP) {
      raw_load(g.nw[c], a.xi_nxt, a.w_nxt, a.wlo_nxt, ew);
      const double2 mv = *(const double2*)(a.mu + i);
      g.m0[c] = mv.x; g.m1[c] = mv.y;
      g.sv[c] = *(const float2*)(a.vsc + i);
    } else {
      raw_zero(g.nw[c]);
      g.m0[c] = g.m1[c] = 0.0;
      g.sv[c] = make_float2(0.f, 0.f);
    }
  }
}

template <bool PROP>
DEV void upd_finish_h2(const StepArgs& a, int p, int cb, int nch, bool acc, const UpdRegs<PMIX, 2>& g) {
  const int lane = threadIdx.x & 63;
  const int d = a.d, P = a.P;
  const long ldw = a.ldw ? a.ldw : d;
  double xa[2], xb[2], za[2], zb[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    xa[c] = g.x0[c]; xb[c] = g.x1[c]; za[c] = g.z0[c]; zb[c] = g.z1[c];
  }
  if (acc) {
    // both chunks' accepted Xi and W in flight before either is converted
    Raw2<PMIX> cw[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) raw_load(cw[c], a.xi_cur, a.w_cur, a.wlo_cur, g.ii[c] + (long)p * ldw);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double c0, c1, wc0, wc1;
      raw_xi(cw[c], c0, c1);
      raw_w(cw[c], wc0, wc1);
      xa[c] = propose1(g.r0[c], xa[c], a.rho, c0);
      xb[c] = propose1(g.r1[c], xb[c], a.rho, c1);
      za[c] = __fma_rn(a.c, wc0, a.rho * za[c]);
      zb[c] = __fma_rn(a.c, wc1, a.rho * zb[c]);
      const long e = g.ii[c] + (long)p * d;
      *(double2*)(a.X + e) = make_double2(xa[c], xb[c]);
      *(double2*)(a.Z + e) = make_double2(za[c], zb[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int ch = cb * 2 + c;
    const int i = g.ii[c];
    const long e = i + (long)p * d;
    const double ra = g.r0[c], rb = g.r1[c];
    store_win2<PMIX>(a.win, i + (a.win_col0 + p) * (long)d, xa[c] - ra, xb[c] - rb);
    double pacc[MAXPROJ] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < a.nproj; ++k) {
      const double2 pv = *(const double2*)(a.proj + i + (long)k * d);
      pacc[k] = __fma_rn(pv.y, xb[c], __fma_rn(pv.x, xa[c], pacc[k]));
    }
    if (PROP) {
      double n0, n1, wn0, wn1;
      raw_xi(g.nw[c], n0, n1);
      raw_w(g.nw[c], wn0, wn1);
      const double xp0 = propose1(ra, xa[c], a.rho, n0), xp1 = propose1(rb, xb[c], a.rho, n1);
      u16 h0, l0, h1, l1;
      const double s0 = (xp0 - g.m0[c]) * (double)g.sv[c].x, s1 = (xp1 - g.m1[c]) * (double)g.sv[c].y;
      if (fmax(fabs(s0), fabs(s1)) >= H2_RANGE) atomicOr(a.err, 2);
      split_f16(s0, h0, l0);
      split_f16(s1, h1, l1);
      *(uint32_t*)(a.vh + e) = (uint32_t)h0 | ((uint32_t)h1 << 16);
      *(uint32_t*)(a.vh + (long)d * P + e) = (uint32_t)l0 | ((uint32_t)l1 << 16);
      const double zp0 = __fma_rn(a.c, wn0, a.rho * za[c]), zp1 = __fma_rn(a.c, wn1, a.rho * zb[c]);
      double zacc = __fma_rn(zp1, zp1, __fma_rn(zp0, zp0, 0.0));
      double xacc = __fma_rn(xp1, xp1, __fma_rn(xp0, xp0, 0.0));
      zacc = wave_sum_f64(zacc);
      if (lane == 0) a.zq_part_nxt[(long)p * nch + ch] = zacc;
      if (a.prior_w > 0.0) {
        xacc = wave_sum_f64(xacc);
        if (lane == 0) a.pq_part_nxt[(long)p * nch + ch] = xacc;
      }
    }
    if (a.nproj > 0) {
      for (int k = 0; k < a.nproj; ++k) {
        const double v = wave_sum_f64(pacc[k]);
        if (lane == 0) a.proj_part[((long)ch * a.nproj + k) * P + p] = v;
      }
    }
  }
}

// One step of the mixed form with the half target's reduction folded in:
// workgroup p (d / 256 wavefronts) issues its update loads, reduces the
// K-split partial products of its rows into the row-block terms of log pi
// (stored to part as the separate reduction does, and kept in LDS), then
// every wavefront takes the chain's decision from the LDS terms (bitwise the
// sums of the separate path) and updates its two 128-row chunks; wavefront 0
// writes the decision's outputs.
template <bool PROP>
__global__ __launch_bounds__(1024) void k_step_h2(StepArgs a, int nch, const float* __restrict__ Yp,
                                                  const double* __restrict__ rsc, double* __restrict__ part,
                                                  const double* __restrict__ twist) {
  __shared__ double lpp[64];
  const int p = blockIdx.x, v = threadIdx.x >> 6, lane = threadIdx.x & 63;
  UpdRegs<PMIX, 2> g;
  upd_load_h2<PROP>(a, p, v, g);
  const DecIn din = decide_inputs(a, nch, p);
  const double q = h2_reduce_wave(Yp, rsc, a.d, a.P, a.nrb, part, twist, p, v);
  if ((lane & 15) == 0) lpp[v * 4 + (lane >> 4)] = q;
  __syncthreads();
  const bool acc = decide_wave(a, nch, p, v == 0, lpp, din);
  upd_finish_h2<PROP>(a, p, v, nch, acc, g);
}

// STEP_CPW chunks per wavefront and 8 / STEP_CPW waves per SIMD: the
// P * d / (128 STEP_CPW) wavefronts of a step at P = 256, d = 4096 fit the
// chip in one round (the argument block alone would hold it below that)
template <int PR, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8 / STEP_CPW))) void k_step(StepArgs a, int nch) {
  if (MODE == 2 && (a.d & 1) == 0) step_update2<PR, STEP_CPW>(a, blockIdx.x, nch, blockIdx.y);
  else step_body<PR, MODE>(a, blockIdx.x, nch, blockIdx.y);
}

// A step with an accept half runs as a decision launch (one wave per chain)
// followed by the streaming update; the first proposal of a call has no
// decision.
hipError_t step(const StepArgs& a, hipStream_t s) {
  const int nch = step_chunks(a.d);
  const dim3 gupd((a.d & 1) == 0 ? cdiv(nch, STEP_CPW) : nch, cdiv(a.P, 4));
  // the decision moves into the update launch where one wavefront can take it
  StepArgs b = a;
  b.fuse_dec = a.do_accept && !a.da && a.nrb <= 64 && nch <= 64 && (a.d & 1) == 0;
  if (a.do_accept && !b.fuse_dec) hipLaunchKernelGGL(k_decide, dim3(a.P), dim3(256), 0, s, b, nch);
  if (a.prec == P64) hipLaunchKernelGGL((k_step<P64, 2>), gupd, dim3(256), 0, s, b, nch);
  else if (a.prec == P32) hipLaunchKernelGGL((k_step<P32, 2>), gupd, dim3(256), 0, s, b, nch);
  else hipLaunchKernelGGL((k_step<PMIX, 2>), gupd, dim3(256), 0, s, b, nch);
  return hipGetLastError();
}

bool step_h2_ok(int d, int P, int nrb) {
  return d % 256 == 0 && d <= 4096 && nrb == d / 64 && step_chunks(d) <= 64 && tgt_h2_ok(d, P);
}

hipError_t step_h2(const StepArgs& a, const float* Yp, const double* rsc, double* part, const double* twist,
                   hipStream_t s) {
  if (a.prec != PMIX || !a.vh || !a.mu || !a.vsc || !a.do_accept || a.da || !step_h2_ok(a.d, a.P, a.nrb))
    return hipErrorInvalidValue;
  StepArgs b = a;
  b.fuse_dec = 1;
  if (a.do_propose)
    hipLaunchKernelGGL(k_step_h2<true>, dim3(a.P), dim3(64 * (a.d / 256)), 0, s, b, step_chunks(a.d), Yp, rsc, part,
                       twist);
  else
    hipLaunchKernelGGL(k_step_h2<false>, dim3(a.P), dim3(64 * (a.d / 256)), 0, s, b, step_chunks(a.d), Yp, rsc,
                       part, twist);
  return hipGetLastError();
}

DEV void init_eval_elem(int v64, const double* __restrict__ X, const double* __restrict__ mu, void* __restrict__ V,
                        double* __restrict__ Z, int d, long e) {
  const double x = X[e];
  const double v = x - (mu ? mu[e % d] : 0.0);
  if (v64) ((double*)V)[e] = v;
  else ((float*)V)[e] = (float)v;
  Z[e] = x;
}

__global__ __launch_bounds__(256) void k_init_eval(int v64, const double* __restrict__ X, const double* __restrict__ mu,
                                                   void* __restrict__ V, double* __restrict__ Z, int d, long n) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < n) init_eval_elem(v64, X, mu, V, Z, d, e);
}

hipError_t init_eval(int v64, const double* X, const double* mu, void* V, double* Z, int d, int P, hipStream_t s) {
  const long n = (long)d * P;
  hipLaunchKernelGGL(k_init_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v64, X, mu, V, Z, d, n);
  return hipGetLastError();
}

// lp[p] = sum_rb part[rb][p] - prior_w |x_p|^2 (one block per chain)
DEV void init_finish_block(const double* __restrict__ part, int nrb, int P, const double* __restrict__ X, int d,
                           double prior_w, double* __restrict__ lp, int p) {
  __shared__ double red[2][256];
  double s = 0.0, q = 0.0;
  for (int k = threadIdx.x; k < nrb; k += 256) s += part[(long)p * nrb + k];
  if (prior_w > 0.0)
    for (int i = threadIdx.x; i < d; i += 256) {
      const double x = X[i + (long)p * d];
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
  if (threadIdx.x == 0) lp[p] = (prior_w > 0.0) ? __fma_rn(-prior_w, red[1][0], red[0][0]) : red[0][0];
}

__global__ __launch_bounds__(256) void k_init_finish(const double* __restrict__ part, int nrb, int P,
                                                     const double* __restrict__ X, int d, double prior_w,
                                                     double* __restrict__ lp) {
  init_finish_block(part, nrb, P, X, d, prior_w, lp, blockIdx.x);
}

hipError_t init_finish(const double* part, int nrb, const double* Z, const double* X, double prior_w, double* lp,
                       double* zq, int d, int P, hipStream_t s) {
  hipLaunchKernelGGL(k_init_finish, dim3(P), dim3(256), 0, s, part, nrb, P, X, d, prior_w, lp);
  hipLaunchKernelGGL(k_colnorm, dim3(P), dim3(256), 0, s, Z, d, zq);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_proj_reduce(const double* __restrict__ proj_part, int n, int nch, int nproj,
                                                     int P, double* __restrict__ trace, int nfun) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)n * nproj * P) return;
  const int p = (int)(e % P);
  const int k = (int)((e / P) % nproj);
  const long t = e / ((long)P * nproj);
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += proj_part[((t * nch + c) * nproj + k) * P + p];
  trace[(t * nfun + 1 + k) * P + p] = s;
}

hipError_t proj_reduce(const double* proj_part, int n, int nch, int nproj, int P, double* trace, int nfun,
                       hipStream_t s) {
  const long total = (long)n * nproj * P;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_proj_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, proj_part, n, nch, nproj, P,
                     trace, nfun);
  return hipGetLastError();
}

// ============================================================================
// Batched form: G independent Gaussian problems of uneven d with P chains
// each (FP32 path, FP64 state and Cholesky).  Every launch below serves all
// problems at once: a host-built tile list maps blockIdx.x to (problem, tile),
// and the tile runs the same body as the single-problem kernel, so results
// are bitwise those of separate runs with the same tile shapes.
// ============================================================================
__global__ __launch_bounds__(256) void gk_normals(uint32_t k0, uint32_t k1, const long* __restrict__ win,
                                                  long per_window, long total, float* __restrict__ W) {
  const long g0 = *win * per_window;
  const long stride = (long)gridDim.x * 256;
  const bool vec = (uintptr_t)W % 16 == 0;
  for (long q = (long)blockIdx.x * 256 + threadIdx.x; 4 * q < total; q += stride) {
    float v[4];
    normals4_f32(k0, k1, (uint64_t)(g0 + 4 * q), v);
    if (vec && 4 * q + 3 < total) {
      *(float4*)(W + 4 * q) = make_float4(v[0], v[1], v[2], v[3]);
      continue;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (4 * q + e < total) W[4 * q + e] = v[e];
  }
}

// U[e], e = (g n + t) P + p: Philox stream 1, counter (window, problem-step, p/2)
__global__ __launch_bounds__(256) void gk_uniforms(uint32_t k0, uint32_t k1, const long* __restrict__ win, long total,
                                                   int P, double* __restrict__ U) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int p = (int)(e % P);
  const long gt = e / P;
  const uint64_t w = (uint64_t)*win;
  const u4_t r = philox4x32_10({(uint32_t)w, (uint32_t)gt, 1u, (uint32_t)(p >> 1)}, k0, k1);
  U[e] = (p & 1) ? u01_f64(r.z, r.w) : u01_f64(r.x, r.y);
}

__global__ void gk_bump(long* win, double* N, double K) {
  if (threadIdx.x == 0) {
    *win += 1;
    *N += K;
  }
}

template <int BM, int KG>
__global__ __launch_bounds__(256 * KG) void gk_tgt(const BProb* __restrict__ pr, const BTile* __restrict__ tl, int P) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  tgt_gauss_tile<float, 32, BM, 32, KG>(b.Rp, b.Vp, b.ld, P, t.a, t.b, b.lpp_part, b.nrb);
}

hipError_t g_tgt(int cfg, const BProb* pr, const BTile* tl, int ntiles, int P, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (cfg) {
    case 0: hipLaunchKernelGGL((gk_tgt<32, 2>), dim3(ntiles), dim3(512), 0, s, pr, tl, P); break;
    case 1: hipLaunchKernelGGL((gk_tgt<64, 1>), dim3(ntiles), dim3(256), 0, s, pr, tl, P); break;
    case 2: hipLaunchKernelGGL((gk_tgt<64, 2>), dim3(ntiles), dim3(512), 0, s, pr, tl, P); break;
    case 3: hipLaunchKernelGGL((gk_tgt<128, 2>), dim3(ntiles), dim3(512), 0, s, pr, tl, P); break;
    default: hipLaunchKernelGGL((gk_tgt<32, 4>), dim3(ntiles), dim3(1024), 0, s, pr, tl, P); break;
  }
  return hipGetLastError();
}
int g_tgt_bm(int cfg) {
  static const int bm[G_TGT_CONFIGS] = {32, 64, 64, 128, 32};
  return bm[cfg];
}

// Step arguments of problem b for step st.t (accept step t, propose step
// t + 1; t = -1: the first proposal only).
DEV StepArgs g_step_args(const BProb& b, const BStep& st, int g) {
  const int P = st.P, d = b.d, cu = st.t & 1, nx = cu ^ 1;
  const long dP = (long)b.ld * P;  // one step's slice of W and Xi (padded rows)
  StepArgs a{};
  a.d = d;
  a.P = P;
  a.prec = P32;
  a.rho = st.rho;
  a.c = st.c;
  a.inv2a2 = st.inv2a2;
  a.xr = b.xr;
  a.mu = b.mu;
  a.X = b.X;
  a.Z = b.Z;
  a.V = b.Vp;
  a.ldv = b.ld;
  a.ldw = b.ld;
  a.nrb = b.nrb;
  a.lpp_part = b.lpp_part;
  a.nacc = b.nacc;
  a.win = b.win;
  a.err = st.err;
  if (st.t >= 0) {
    a.do_accept = 1;
    a.xi_cur = b.Xi + st.t * dP;
    a.w_cur = b.W + st.t * dP;
    a.wlo_cur = nullptr;
    a.zq_part_cur = b.zq_part + (long)cu * b.nch * P;
    a.lp_cur = b.lp + (long)cu * P;
    a.zq_cur = b.zq + (long)cu * P;
    a.lp_nxt = b.lp + (long)nx * P;
    a.zq_nxt = b.zq + (long)nx * P;
    a.u = st.U + ((long)g * st.n + st.t) * P;
    a.la_out = b.la + (long)st.t * P;
    a.acc_out = b.acc + (long)st.t * P;
    a.win_col0 = (long)st.t * P;
  }
  const int tn = st.t + 1;
  if (tn < st.n) {
    // the proposal of step tn is judged with the scalars of parity tn & 1
    a.do_propose = 1;
    a.xi_nxt = b.Xi + tn * dP;
    a.w_nxt = b.W + tn * dP;
    a.wlo_nxt = nullptr;
    a.zq_part_nxt = b.zq_part + (long)(tn & 1) * b.nch * P;
  }
  return a;
}

template <int MODE>
__global__ __launch_bounds__(256) void gk_step(const BProb* __restrict__ pr, const BTile* __restrict__ tl, BStep st) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  const StepArgs a = g_step_args(b, st, t.g);
  if (MODE == 1) decide_block(a, b.nch, t.b);
  else if ((b.d & 1) == 0) step_update2<P32>(a, t.a, b.nch, t.b);
  else step_body<P32, 2>(a, t.a, b.nch, t.b);
}

// decision launch over (problem, 0, chain) tiles (a workgroup per chain),
// then the update over (problem, chunk, chain quad) tiles; the first
// proposal has no decision
hipError_t g_step(const BProb* pr, const BTile* dec_tl, int ndec, const BTile* tl, int ntiles, const BStep& st,
                  hipStream_t s) {
  if (st.t >= 0) hipLaunchKernelGGL((gk_step<1>), dim3(ndec), dim3(256), 0, s, pr, dec_tl, st);
  hipLaunchKernelGGL((gk_step<2>), dim3(ntiles), dim3(256), 0, s, pr, tl, st);
  return hipGetLastError();
}

// The n_lag steps of a window for every problem in one launch (see PItem).
// Items are taken in queue order, so every item an item waits for was taken
// earlier by a running workgroup: the earliest unfinished item can always
// proceed, whatever the grid size.  A wait is bounded: after spin_max polls it
// sets bit 1 of the error word, and every workgroup then stops taking items.
// Thread 0 publishes a finished item (agent-scope release, after the
// workgroup barrier that ends the item) when it takes the next one; a waiter
// polls relaxed and then fences with an agent-scope acquire.  Every loop exit
// tests a value read back as wavefront-uniform, so all wavefronts leave (and
// pass every barrier) together.  The bodies are those of gk_tgt (64 x 2
// tiles), decide_wave (bitwise decide_block at these sizes: at most 64 row
// blocks and 64 chunks) and the update half of gk_step, so results are
// bitwise those of the per-phase launches with the default tile shape.
__global__ __launch_bounds__(PERSIST_THREADS) void gk_persist(const BProb* __restrict__ pr,
                                                              const PItem* __restrict__ items, int nitems, BStep st,
                                                              PCtl c) {
  __shared__ int s_q, s_ok;
  const int total = nitems * st.n;
  int prev_g = -1;  // problem of the item finished in the previous pass (thread 0 publishes it)
  for (;;) {
    if (threadIdx.x == 0) {
      if (prev_g >= 0) __hip_atomic_fetch_add(c.done + prev_g, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      int q = -1;
      if ((__hip_atomic_load(c.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2) == 0)
        q = __hip_atomic_fetch_add(c.qctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_q = q;
    }
    __syncthreads();
    const int q = __builtin_amdgcn_readfirstlane(s_q);
    if (q < 0 || q >= total) break;
    const int t = q / nitems;
    const PItem it = items[q - t * nitems];
    if (threadIdx.x == 0) {
      const int need = t * c.per_step[it.g] + it.need;
      int ok = 1, spins = 0;
      while (__hip_atomic_load(c.done + it.g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (++spins > c.spin_max || (__hip_atomic_load(c.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2)) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (!ok) __hip_atomic_fetch_or(c.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_ok = ok;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_ok) == 0) break;
    const int kind = __builtin_amdgcn_readfirstlane(it.kind), g = __builtin_amdgcn_readfirstlane(it.g);
    const BProb& b = pr[g];
    if (kind == 0) {
      tgt_gauss_tile<float, 32, 64, 32, 2>(b.Rp, b.Vp, b.ld, st.P, it.a, it.b, b.lpp_part, b.nrb);
    } else {
      BStep sp = st;
      sp.t = t;
      StepArgs a = g_step_args(b, sp, g);
      // the update items take the decision themselves where no decision item
      // was queued (the same predicate as the queue's construction)
      a.fuse_dec = kind == 2 && persist_fused_decision(b.d, b.nrb, b.nch) ? 1 : 0;
      const int w = threadIdx.x >> 6;
      if (kind == 1) {
        for (int p = w; p < st.P; p += PERSIST_THREADS / 64)
          decide_wave(a, b.nch, p, true, a.lpp_part + (long)p * a.nrb);
      } else {
        // eight waves: chains 8k .. 8k + 7 per pass (the bodies take chain 4 pq + wave)
        for (int pq = 0; pq * 4 < st.P; pq += PERSIST_THREADS / 256) {
          if ((b.d & 1) == 0) step_update2<P32>(a, it.a, b.nch, pq);
          else step_body<P32, 2>(a, it.a, b.nch, pq);
        }
      }
    }
    // the item's stores, in every wavefront, complete (a workgroup barrier
    // alone does not wait for other wavefronts' stores) before thread 0
    // publishes the item with its agent-scope release
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    prev_g = g;
  }
}

hipError_t g_persist(const BProb* pr, const PItem* items, int nitems, const BStep& st, const PCtl& ctl, int grid,
                     hipStream_t s) {
  if (nitems <= 0 || st.n <= 0 || grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(gk_persist, dim3(grid), dim3(PERSIST_THREADS), 0, s, pr, items, nitems, st, ctl);
  return hipGetLastError();
}

int g_persist_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gk_persist, PERSIST_THREADS, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

__global__ __launch_bounds__(256) void gk_trigemm(const BProb* __restrict__ pr, const BTile* __restrict__ tl, int ncols,
                                                  double c) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  trigemm_tile<float, 32>(b.Lp, b.W, b.Xi, b.ld, ncols, c, t.a, t.b);
}

hipError_t g_trigemm(const BProb* pr, const BTile* tl, int ntiles, int ncols, double c, hipStream_t s) {
  hipLaunchKernelGGL(gk_trigemm, dim3(ntiles), dim3(256), 0, s, pr, tl, ncols, c);
  return hipGetLastError();
}

// window scatter (one K split) and row sums
__global__ __launch_bounds__(256) void gk_syrk(const BProb* __restrict__ pr, const BTile* __restrict__ tl, int K) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  syrk_tile<float, 32>(b.win, b.d, K, K, t.a, 0, b.G);
}
__global__ __launch_bounds__(256) void gk_rowsum(const BProb* __restrict__ pr, const BTile* __restrict__ tl, int K) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  rowsum_block<float, true>(b.win, b.d, K, K, t.a, 0, b.h);
}

hipError_t g_scatter(const BProb* pr, const BTile* syrk_tl, int nsyrk, const BTile* row_tl, int nrow, int K,
                     hipStream_t s) {
  hipLaunchKernelGGL(gk_syrk, dim3(nsyrk), dim3(256), 0, s, pr, syrk_tl, K);
  hipLaunchKernelGGL(gk_rowsum, dim3(nrow), dim3(256), 0, s, pr, row_tl, K);
  return hipGetLastError();
}

// Element-wise phases over per-problem index spaces: tile (g, block) covers
// elements [256 block, 256 block + 256) of problem g.
__global__ __launch_bounds__(256) void gk_fold(const BProb* __restrict__ pr, const BTile* __restrict__ dd_tl,
                                               const double* __restrict__ N, double K) {
  const BTile t = dd_tl[blockIdx.x];
  const BProb& b = pr[t.g];
  const long e = (long)t.a * 256 + threadIdx.x;
  const double n0 = *N;
  if (e < (long)b.d * b.d) fold_S_elem(b.G, b.h, b.xr, n0, K, b.S, b.d, e);
}
__global__ __launch_bounds__(256) void gk_fold_mean(const BProb* __restrict__ pr, const BTile* __restrict__ d_tl,
                                                    const double* __restrict__ N, double K) {
  const BTile t = d_tl[blockIdx.x];
  const BProb& b = pr[t.g];
  const int i = t.a * 256 + threadIdx.x;
  if (i < b.d) fold_mean_elem(b.h, b.xr, *N, K, b.m, i);
}

hipError_t g_fold(const BProb* pr, const BTile* dd_tl, int ndd, const BTile* d_tl, int nd, const double* N, double K,
                  hipStream_t s) {
  hipLaunchKernelGGL(gk_fold, dim3(ndd), dim3(256), 0, s, pr, dd_tl, N, K);
  hipLaunchKernelGGL(gk_fold_mean, dim3(nd), dim3(256), 0, s, pr, d_tl, N, K);
  return hipGetLastError();
}

// covariance (no jitter) into C; clears the problem's Cholesky status
__global__ __launch_bounds__(256) void gk_cov(const BProb* __restrict__ pr, const BTile* __restrict__ dd_tl) {
  const BTile t = dd_tl[blockIdx.x];
  const BProb& b = pr[t.g];
  const long e = (long)t.a * 256 + threadIdx.x;
  if (e < (long)b.d * b.d) cov_elem(b.S, b.m, 0.0, b.C, b.d, e);
  if (t.a == 0 && threadIdx.x == 0) *b.info = 0;
}

hipError_t g_cov(const BProb* pr, const BTile* dd_tl, int ndd, hipStream_t s) {
  hipLaunchKernelGGL(gk_cov, dim3(ndd), dim3(256), 0, s, pr, dd_tl);
  return hipGetLastError();
}

// blocked Cholesky, block column jb of every problem with more than jb blocks
__global__ __launch_bounds__(CHOL_DIAG_THREADS) void gk_chol_diag(const BProb* __restrict__ pr, const BTile* __restrict__ tl, int jb) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  const int j0 = jb * CHOL_NB, jn = min(CHOL_NB, b.d - j0);
  chol_diag_block(b.C, b.d, j0, jn, b.Linv + (long)jb * CHOL_NB * CHOL_NB, b.info);
}
__global__ __launch_bounds__(256) void gk_chol_panel(const BProb* __restrict__ pr, const BTile* __restrict__ tl, int jb) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  const int j0 = jb * CHOL_NB, jn = min(CHOL_NB, b.d - j0);
  chol_panel_tile(b.C, b.d, j0, jn, b.Linv + (long)jb * CHOL_NB * CHOL_NB, t.a);
}
__global__ __launch_bounds__(256) void gk_chol_update(const BProb* __restrict__ pr, const BTile* __restrict__ tl,
                                                      int jb) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  const int j0 = jb * CHOL_NB, jn = min(CHOL_NB, b.d - j0);
  chol_update_tile(b.C, b.d, j0, jn, jb + 1, t.a);
}

hipError_t g_chol_step(const BProb* pr, const BTile* diag, int ndiag, const BTile* panel, int npanel,
                       const BTile* upd, int nupd, int jb, hipStream_t s) {
  if (ndiag) hipLaunchKernelGGL(gk_chol_diag, dim3(ndiag), dim3(CHOL_DIAG_THREADS), 0, s, pr, diag, jb);
  if (npanel) hipLaunchKernelGGL(gk_chol_panel, dim3(npanel), dim3(256), 0, s, pr, panel, jb);
  if (nupd) hipLaunchKernelGGL(gk_chol_update, dim3(nupd), dim3(256), 0, s, pr, upd, jb);
  return hipGetLastError();
}

// A factored problem (status 0) adopts C as its factor, rounded to FP32,
// and its merged mean as the pivot; a failed one keeps both.
__global__ __launch_bounds__(256) void gk_adopt(const BProb* __restrict__ pr, const BTile* __restrict__ dd_tl) {
  const BTile t = dd_tl[blockIdx.x];
  const BProb& b = pr[t.g];
  if (*b.info != 0) return;
  const long e = (long)t.a * 256 + threadIdx.x;
  if (e < (long)b.d * b.d) {
    b.L[e] = b.C[e];
    round_factor_elem(P32, b.L, b.Llow, b.d, e);
    b.Lp[(e % b.d) + (e / b.d) * b.ld] = b.Llow[e];
  }
  if (e < b.d) b.xr[e] = b.m[e];
}

hipError_t g_adopt(const BProb* pr, const BTile* dd_tl, int ndd, hipStream_t s) {
  hipLaunchKernelGGL(gk_adopt, dim3(ndd), dim3(256), 0, s, pr, dd_tl);
  return hipGetLastError();
}

// whitening z = L^-1 (x - x_ref) of every problem
__global__ __launch_bounds__(256) void gk_sub_ref(const BProb* __restrict__ pr, const BTile* __restrict__ dp_tl, int P) {
  const BTile t = dp_tl[blockIdx.x];
  const BProb& b = pr[t.g];
  const long e = (long)t.a * 256 + threadIdx.x;
  if (e < (long)b.d * P) sub_ref_elem(b.X, b.xr, b.Z, b.d, e);
}
__global__ __launch_bounds__(64) void gk_tri_inv(const BProb* __restrict__ pr, const BTile* __restrict__ tl) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  tri_inv_block(b.L, b.d, b.Linv, t.a);
}
__global__ __launch_bounds__(256) void gk_trsm_diag(const BProb* __restrict__ pr, const BTile* __restrict__ tl, int jb,
                                                    int P) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  const int j0 = jb * CHOL_NB, jn = min(CHOL_NB, b.d - j0);
  trsm_diag_tile(b.Linv + (long)jb * CHOL_NB * CHOL_NB, b.Z, b.d, P, j0, jn, t.a);
}
__global__ __launch_bounds__(256) void gk_trsm_update(const BProb* __restrict__ pr, const BTile* __restrict__ tl, int jb,
                                                      int P) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  const int j0 = jb * CHOL_NB, jn = min(CHOL_NB, b.d - j0);
  trsm_update_tile(b.L, b.Z, b.d, P, j0, jn, t.a, t.b);
}
__global__ __launch_bounds__(256) void gk_colnorm(const BProb* __restrict__ pr, const BTile* __restrict__ tl) {
  const BTile t = tl[blockIdx.x];
  const BProb& b = pr[t.g];
  colnorm_block(b.Z, b.d, b.zq, t.a);  // parity 0 at a window boundary
}

hipError_t g_sub_ref(const BProb* pr, const BTile* dp_tl, int ndp, int P, hipStream_t s) {
  hipLaunchKernelGGL(gk_sub_ref, dim3(ndp), dim3(256), 0, s, pr, dp_tl, P);
  return hipGetLastError();
}
hipError_t g_tri_inv(const BProb* pr, const BTile* tl, int n, hipStream_t s) {
  hipLaunchKernelGGL(gk_tri_inv, dim3(n), dim3(64), 0, s, pr, tl);
  return hipGetLastError();
}
hipError_t g_trsm_step(const BProb* pr, const BTile* diag, int ndiag, const BTile* upd, int nupd, int jb, int P,
                       hipStream_t s) {
  if (ndiag) hipLaunchKernelGGL(gk_trsm_diag, dim3(ndiag), dim3(256), 0, s, pr, diag, jb, P);
  if (nupd) hipLaunchKernelGGL(gk_trsm_update, dim3(nupd), dim3(256), 0, s, pr, upd, jb, P);
  return hipGetLastError();
}
hipError_t g_colnorm(const BProb* pr, const BTile* tl, int n, hipStream_t s) {
  hipLaunchKernelGGL(gk_colnorm, dim3(n), dim3(256), 0, s, pr, tl);
  return hipGetLastError();
}

hipError_t g_rng(uint64_t seed, const long* win, long nW, long nU, int P, float* W, double* U, hipStream_t s) {
  long nq = (nW + 3) / 4;
  int blocks = (int)((nq + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(gk_normals, dim3(blocks), dim3(256), 0, s, (uint32_t)seed, (uint32_t)(seed >> 32), win, nW, nW, W);
  hipLaunchKernelGGL(gk_uniforms, dim3((unsigned)((nU + 255) / 256)), dim3(256), 0, s, (uint32_t)seed,
                     (uint32_t)(seed >> 32), win, nU, P, U);
  return hipGetLastError();
}

hipError_t g_bump(long* win, double* N, double K, hipStream_t s) {
  hipLaunchKernelGGL(gk_bump, dim3(1), dim3(64), 0, s, win, N, K);
  return hipGetLastError();
}

}  // namespace dk
