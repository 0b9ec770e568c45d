// Concurrent-chain logistics with M > 1 intervals per batch (Section 2.4.1):
// between global merges every chain proposes with its own factor L_p and
// pivot x_ref_p, refactorised from its local update of the global moments
// (eqs. mom2pg, mom1pg, cov2pg).  FP64 throughout.
//
// Layouts: the window store and the normals are step-major (column t P + p is
// chain p at step t, d rows); L_p are P lower d x d column-major factors,
// chain p at Lp + p d^2; G_p (P x d x d) and h_p (d x P) are chain p's sums
// of y y^T and y over the batch so far, y = x - s with s the shared pivot of
// the batch (the shift the window store already carries).
#include "common.h"
#include "kernels.h"

namespace dk {

namespace {

constexpr int PC_TM = 64;   // rows per tile
constexpr int PC_TN = 32;   // steps per tile of the proposal contraction
constexpr int PC_TK = 32;   // contraction chunk

// Xi[:, tP+p] = c L_p W[:, tP+p] + (1 - rho)(xr_p - xr).  With the step's
// x' = xr + rho (x - xr) + Xi this is eq. diam about chain p's own pivot:
// x' = xr_p + rho (x - xr_p) + c L_p W.  Tile: 64 rows x 32 steps of one
// chain, 256 threads holding 4 rows x 2 steps each; only the lower triangle
// of L_p is read (the upper part of the buffer is not a factor entry).
__global__ __launch_bounds__(256) void k_pc_gemm(const double* __restrict__ Lp, const double* __restrict__ W,
                                                 const double* __restrict__ xrp, const double* __restrict__ xr,
                                                 double* __restrict__ Xi, int d, int P, int n, double c,
                                                 double omr) {
  __shared__ double As[PC_TK][PC_TM + 1];
  __shared__ double Bs[PC_TK][PC_TN + 1];
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
  const int i0 = blockIdx.x * PC_TM, t0 = blockIdx.y * PC_TN, p = blockIdx.z;
  const double* L = Lp + (long)p * d * d;
  double acc[4][2] = {};
  const int kend = min(d, i0 + PC_TM);
  for (int k0 = 0; k0 < kend; k0 += PC_TK) {
#pragma unroll
    for (int e = 0; e < PC_TM * PC_TK / 256; ++e) {
      const int idx = tid + e * 256, r = idx % PC_TM, k = idx / PC_TM;
      const int i = i0 + r, kk = k0 + k;
      As[k][r] = (i < d && kk <= i) ? L[i + (long)kk * d] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < PC_TK * PC_TN / 256; ++e) {
      const int idx = tid + e * 256, k = idx % PC_TK, tt = idx / PC_TK;
      const int kk = k0 + k, t = t0 + tt;
      Bs[k][tt] = (kk < d && t < n) ? W[kk + ((long)t * P + p) * d] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < PC_TK; ++k) {
      double a[4], b[2];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[k][tr * 4 + r];
      b[0] = Bs[k][tc * 2];
      b[1] = Bs[k][tc * 2 + 1];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc[r][0] = __fma_rn(a[r], b[0], acc[r][0]);
        acc[r][1] = __fma_rn(a[r], b[1], acc[r][1]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + tr * 4 + r;
    if (i >= d) continue;
    const double corr = omr * (xrp[i + (long)p * d] - xr[i]);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int t = t0 + tc * 2 + q;
      if (t < n) Xi[i + ((long)t * P + p) * d] = __fma_rn(c, acc[r][q], corr);
    }
  }
}

// G_p += sum_t y_t y_t^T over one window (y = the stored shifted states of
// chain p).  Tile 64 x 64 of G_p, 256 threads with 4 x 4 entries each; each
// tile is owned by one workgroup, so the update is a plain read-add-write.
__global__ __launch_bounds__(256) void k_pc_scatter(const double* __restrict__ win, double* __restrict__ Gp, int d,
                                                    int P, int n) {
  __shared__ double Yi[PC_TK][PC_TM + 1];
  __shared__ double Yj[PC_TK][PC_TM + 1];
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
  const int i0 = blockIdx.x * PC_TM, j0 = blockIdx.y * PC_TM, p = blockIdx.z;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < n; k0 += PC_TK) {
#pragma unroll
    for (int e = 0; e < PC_TM * PC_TK / 256; ++e) {
      const int idx = tid + e * 256, r = idx % PC_TM, k = idx / PC_TM;
      const int t = k0 + k;
      const long col = ((long)t * P + p) * d;
      Yi[k][r] = (t < n && i0 + r < d) ? win[i0 + r + col] : 0.0;
      Yj[k][r] = (t < n && j0 + r < d) ? win[j0 + r + col] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < PC_TK; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a[r] = Yi[k][tr * 4 + r];
        b[r] = Yj[k][tc * 4 + r];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = __fma_rn(a[r], b[q], acc[r][q]);
    }
    __syncthreads();
  }
  double* G = Gp + (long)p * d * d;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + tr * 4 + r;
    if (i >= d) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + tc * 4 + q;
      if (j < d) G[i + (long)j * d] += acc[r][q];
    }
  }
}

// h_p += sum_t y_t: one thread per (row, chain), the window's steps in order.
__global__ __launch_bounds__(256) void k_pc_rowsum(const double* __restrict__ win, double* __restrict__ hp, int d,
                                                   int P, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x, p = blockIdx.y;
  if (i >= d) return;
  double s = 0.0;
  for (int t = 0; t < n; ++t) s += win[i + ((long)t * P + p) * d];
  hp[i + (long)p * d] += s;
}

// Chain p's local update of the global moments (eqs. mom2pg, mom1pg) with
// sample-count weights: raw sums of its n batch samples x = y + s are
// G + h s^T + s h^T + n s s^T and h + n s, so
//   S_pg = (N S + G + h s^T + s h^T + n s s^T) / (N + n),
//   m_pg = (N m + h + n s) / (N + n).
__global__ __launch_bounds__(256) void k_pc_moments(const double* __restrict__ S, const double* __restrict__ m,
                                                    double N, const double* __restrict__ G,
                                                    const double* __restrict__ h, const double* __restrict__ sft,
                                                    double n, double* __restrict__ Spg, double* __restrict__ mpg,
                                                    int d) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const double inv = 1.0 / (N + n);
  if (e < (long)d * d) {
    const int i = (int)(e % d), j = (int)(e / d);
    const double raw = G[e] + h[i] * sft[j] + sft[i] * h[j] + n * sft[i] * sft[j];
    Spg[e] = (N * S[e] + raw) * inv;
  }
  if (e < d) mpg[e] = (N * m[e] + (h[e] + n * sft[e])) * inv;
}

// Sums over the chains for the global merge: G = sum_p G_p, h = sum_p h_p.
__global__ __launch_bounds__(256) void k_pc_sum(const double* __restrict__ Gp, const double* __restrict__ hp,
                                                double* __restrict__ G, double* __restrict__ h, int d, int P) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x, dd = (long)d * d;
  if (e < dd) {
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += Gp[e + p * dd];
    G[e] = s;
  }
  if (e < d) {
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += hp[e + (long)p * d];
    h[e] = s;
  }
}

// Every chain's covariance C_p = S_pg - m_pg m_pg^T (lower triangle, zeros
// above) and pivot m_pg at once, blockIdx.z = chain: the arithmetic of
// k_pc_moments followed by the covariance assembly, operation for operation,
// so a chain's C_p is bitwise what the one-chain path assembles.
__global__ __launch_bounds__(256) void k_pc_cov(const double* __restrict__ S, const double* __restrict__ m, double N,
                                                const double* __restrict__ Gp, const double* __restrict__ hp,
                                                const double* __restrict__ sft, double n, double* __restrict__ Cp,
                                                double* __restrict__ mpgp, int d) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x, dd = (long)d * d;
  const int z = blockIdx.z;
  const double* h = hp + (long)z * d;
  const double inv = 1.0 / (N + n);
  if (e < dd) {
    const int i = (int)(e % d), j = (int)(e / d);
    double v = 0.0;
    if (i >= j) {
      const double raw = Gp[e + z * dd] + h[i] * sft[j] + sft[i] * h[j] + n * sft[i] * sft[j];
      const double Spg = (N * S[e] + raw) * inv;
      const double mi = (N * m[i] + (h[i] + n * sft[i])) * inv;
      const double mj = (N * m[j] + (h[j] + n * sft[j])) * inv;
      v = Spg - mi * mj;
    }
    Cp[e + z * dd] = v;
  }
  if (e < d) mpgp[e + (long)z * d] = (N * m[e] + (h[e] + n * sft[e])) * inv;
}

// Every chain starts the batch's local updates from the shared pair.
__global__ __launch_bounds__(256) void k_pc_bcast(const double* __restrict__ L, const double* __restrict__ xr,
                                                  double* __restrict__ Lp, double* __restrict__ xrp, int d) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x, dd = (long)d * d;
  const int z = blockIdx.z;
  if (e < dd) Lp[e + z * dd] = L[e];
  if (e < d) xrp[e + (long)z * d] = xr[e];
}

// Chains whose factorisation succeeded (skip[z] == 0) adopt factor and pivot.
__global__ __launch_bounds__(256) void k_pc_adopt(const double* __restrict__ Cp, const double* __restrict__ mpgp,
                                                  const int* __restrict__ skip, double* __restrict__ Lp,
                                                  double* __restrict__ xrp, int d) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x, dd = (long)d * d;
  const int z = blockIdx.z;
  if (skip[z]) return;
  if (e < dd) Lp[e + z * dd] = Cp[e + z * dd];
  if (e < d) xrp[e + (long)z * d] = mpgp[e + (long)z * d];
}

long cdiv_l(long a, long b) { return (a + b - 1) / b; }

}  // namespace

hipError_t pc_gemm(const double* Lp, const double* W, const double* xrp, const double* xr, double* Xi, int d, int P,
                   int n, double c, double one_minus_rho, hipStream_t s) {
  if (d < 1 || P < 1 || n < 1 || P > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)cdiv_l(d, PC_TM), (unsigned)cdiv_l(n, PC_TN), (unsigned)P);
  hipLaunchKernelGGL(k_pc_gemm, grid, dim3(256), 0, s, Lp, W, xrp, xr, Xi, d, P, n, c, one_minus_rho);
  return hipGetLastError();
}

hipError_t pc_scatter(const double* win, double* Gp, double* hp, int d, int P, int n, hipStream_t s) {
  if (d < 1 || P < 1 || n < 1 || P > 65535) return hipErrorInvalidValue;
  const unsigned tiles = (unsigned)cdiv_l(d, PC_TM);
  hipLaunchKernelGGL(k_pc_scatter, dim3(tiles, tiles, (unsigned)P), dim3(256), 0, s, win, Gp, d, P, n);
  hipLaunchKernelGGL(k_pc_rowsum, dim3((unsigned)cdiv_l(d, 256), (unsigned)P), dim3(256), 0, s, win, hp, d, P, n);
  return hipGetLastError();
}

hipError_t pc_moments(const double* S, const double* m, double N, const double* G, const double* h,
                      const double* sft, double n, double* Spg, double* mpg, int d, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_moments, dim3((unsigned)cdiv_l((long)d * d, 256)), dim3(256), 0, s, S, m, N, G, h, sft,
                     n, Spg, mpg, d);
  return hipGetLastError();
}

hipError_t pc_cov(const double* S, const double* m, double N, const double* Gp, const double* hp, const double* sft,
                  double n, double* Cp, double* mpgp, int d, int P, hipStream_t s) {
  if (P < 1 || P > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pc_cov, dim3((unsigned)cdiv_l((long)d * d, 256), 1, (unsigned)P), dim3(256), 0, s, S, m, N, Gp,
                     hp, sft, n, Cp, mpgp, d);
  return hipGetLastError();
}

hipError_t pc_bcast(const double* L, const double* xr, double* Lp, double* xrp, int d, int P, hipStream_t s) {
  if (P < 1 || P > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pc_bcast, dim3((unsigned)cdiv_l((long)d * d, 256), 1, (unsigned)P), dim3(256), 0, s, L, xr, Lp,
                     xrp, d);
  return hipGetLastError();
}

hipError_t pc_adopt(const double* Cp, const double* mpgp, const int* skip, double* Lp, double* xrp, int d, int P,
                    hipStream_t s) {
  if (P < 1 || P > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pc_adopt, dim3((unsigned)cdiv_l((long)d * d, 256), 1, (unsigned)P), dim3(256), 0, s, Cp, mpgp,
                     skip, Lp, xrp, d);
  return hipGetLastError();
}

hipError_t pc_sum(const double* Gp, const double* hp, double* G, double* h, int d, int P, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_sum, dim3((unsigned)cdiv_l((long)d * d, 256)), dim3(256), 0, s, Gp, hp, G, h, d, P);
  return hipGetLastError();
}

}  // namespace dk
