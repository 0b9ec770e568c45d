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
#include "gemm.h"
#include "kernels.h"

using namespace gemm;

namespace dk {

namespace {

constexpr int PC_T = 64;    // 64 x 64 output tiles on the FP64 MFMA engine
constexpr int PC_BK = 16;   // K slice

// lower tile t of the row-by-row enumeration: (0,0), (1,0), (1,1), (2,0), ...
DEV void lower_tile(int t, int& bi, int& bj) {
  int b = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((b + 1) * (b + 2) / 2 <= t) ++b;
  while (b * (b + 1) / 2 > t) --b;
  bi = b;
  bj = t - b * (b + 1) / 2;
}

// Xi[:, tP+p] = c L_p W[:, tP+p] + (1 - rho)(xr_p - xr).  With the step's
// x' = xr + rho (x - xr) + Xi this is eq. diam about chain p's own pivot:
// x' = xr_p + rho (x - xr_p) + c L_p W.  One workgroup per (64 rows, 64
// steps, chain) on the FP64 MFMA engine; chain p's normals are the d x n
// operand at W + p d with leading dimension P d.  K stops at the tile's last
// row: the factor buffers hold zeros above the diagonal.
__global__ __launch_bounds__(256) void k_pc_gemm(const double* __restrict__ Lp, const double* __restrict__ W,
                                                 const double* __restrict__ xrp, const double* __restrict__ xr,
                                                 double* __restrict__ Xi, int d, int P, int n, double c,
                                                 double omr) {
  __shared__ double lds[e_lds_elems<double, PC_T, PC_T, PC_BK>()];
  const int i0 = blockIdx.x * PC_T, t0 = blockIdx.y * PC_T, p = blockIdx.z;
  const long ldw = (long)P * d;
  EFrag<double, PC_T, PC_T> f;
  f.zero();
  e_gemm<double, PC_T, PC_T, PC_BK, false, true>(f, Lp + (long)p * d * d, d, d, W + (long)p * d, ldw, n, i0, t0, 0,
                                                 min(d, i0 + PC_T), lds);
#pragma unroll
  for (int m = 0; m < EFrag<double, PC_T, PC_T>::FM; ++m)
#pragma unroll
    for (int q = 0; q < EFrag<double, PC_T, PC_T>::FN; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ti, tj;
        frag_coords<PC_T, PC_T, double>(m, q, r, ti, tj);
        const int i = i0 + ti, t = t0 + tj;
        if (i < d && t < n)
          Xi[i + ((long)t * P + p) * d] = __fma_rn(c, f.c[m][q][r], omr * (xrp[i + (long)p * d] - xr[i]));
      }
}

// G_p += sum_t y_t y_t^T over one window (y = the stored shifted states of
// chain p: the d x n operand at win + p d, leading dimension P d).  Lower
// 64 x 64 tiles only, on the FP64 MFMA engine; entry (i, j), i >= j, is added
// at (i, j) and (j, i) by the one workgroup that owns it, so G_p stays
// exactly symmetric and needs no atomics.
__global__ __launch_bounds__(256) void k_pc_scatter(const double* __restrict__ win, double* __restrict__ Gp, int d,
                                                    int P, int n) {
  __shared__ double lds[e_lds_elems<double, PC_T, PC_T, PC_BK>()];
  int bi, bj;
  lower_tile(blockIdx.x, bi, bj);
  const int i0 = bi * PC_T, j0 = bj * PC_T, p = blockIdx.z;
  const double* Y = win + (long)p * d;
  const long ld = (long)P * d;
  EFrag<double, PC_T, PC_T> f;
  f.zero();
  e_gemm<double, PC_T, PC_T, PC_BK, false, false>(f, Y, ld, d, Y, ld, d, i0, j0, 0, n, lds);
  double* G = Gp + (long)p * d * d;
#pragma unroll
  for (int m = 0; m < EFrag<double, PC_T, PC_T>::FM; ++m)
#pragma unroll
    for (int q = 0; q < EFrag<double, PC_T, PC_T>::FN; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ti, tj;
        frag_coords<PC_T, PC_T, double>(m, q, r, ti, tj);
        const int i = i0 + ti, j = j0 + tj;
        if (i < d && j <= i) {
          G[i + (long)j * d] += f.c[m][q][r];
          if (j < i) G[j + (long)i * d] += f.c[m][q][r];
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
  dim3 grid((unsigned)cdiv_l(d, PC_T), (unsigned)cdiv_l(n, PC_T), (unsigned)P);
  hipLaunchKernelGGL(k_pc_gemm, grid, dim3(256), 0, s, Lp, W, xrp, xr, Xi, d, P, n, c, one_minus_rho);
  return hipGetLastError();
}

hipError_t pc_scatter(const double* win, double* Gp, double* hp, int d, int P, int n, hipStream_t s) {
  if (d < 1 || P < 1 || n < 1 || P > 65535) return hipErrorInvalidValue;
  const long nb = cdiv_l(d, PC_T);
  hipLaunchKernelGGL(k_pc_scatter, dim3((unsigned)(nb * (nb + 1) / 2), 1, (unsigned)P), dim3(256), 0, s, win, Gp, d, P,
                     n);
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
