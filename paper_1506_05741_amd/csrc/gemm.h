// Workgroup tile engines for the dense contractions of the sampler.
//
// A workgroup of 256 threads (4 wavefronts in a 2 x 2 arrangement) computes
// a BM x BN tile  C(i, j) = sum_k A(i, k) B(k, j)  over a K range, staging
// BK-deep slices of both operands through LDS with double buffering.
// Operands are described by (row, k) pairs: A's rows are i, B's rows are j.
// KC ("k-contiguous") selects the global layout of an operand:
//   KC = true : element (r, k) at p[r * ld + k]
//   KC = false: element (r, k) at p[r + k * ld]
// Out-of-range elements are read as zero, so ragged edges need no padding.
// In LDS both operands are stored row-major over k with one element of
// padding per row, which keeps the MFMA fragment reads free of bank
// conflicts for the 16 rows a quarter-wavefront touches.
#pragma once
#include "common.h"

namespace gemm {

constexpr int NT = 256;  // threads per workgroup

// ---------------------------------------------------------------------------
// Element engines: f64 (mfma 16x16x4 f64) and f32 (mfma 16x16x4 f32).
// ---------------------------------------------------------------------------
template <typename T> struct EAcc;
template <> struct EAcc<double> { typedef d4_t V; };
template <> struct EAcc<float> { typedef f4_t V; };

template <typename T> DEVM typename EAcc<T>::V mfma_e(T a, T b, typename EAcc<T>::V c);
template <> DEVM d4_t mfma_e<double>(double a, double b, d4_t c) { return mfma_f64(a, b, c); }
template <> DEVM f4_t mfma_e<float>(float a, float b, f4_t c) { return mfma_f32(a, b, c); }

template <typename T, int ROWS, int BK>
struct EStage {
  // per-thread staging registers for one operand slice of ROWS x BK
  static constexpr int PER = ROWS * BK / NT;
  T v[PER];
};

// Load an operand slice [r0, r0+ROWS) x [k0, k0+BK) into registers.
template <typename T, int ROWS, int BK, bool KC>
DEV void e_load(EStage<T, ROWS, BK>& s, const T* __restrict__ p, long ld, int nrows, int r0, int k0, int kend) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < EStage<T, ROWS, BK>::PER; ++e) {
    int idx = t + e * NT;
    int r, k;
    if (KC) { r = idx / BK; k = idx % BK; } else { k = idx / ROWS; r = idx % ROWS; }
    int gr = r0 + r, gk = k0 + k;
    T val = T(0);
    if (gr < nrows && gk < kend) val = KC ? p[(long)gr * ld + gk] : p[gr + (long)gk * ld];
    s.v[e] = val;
  }
}

template <typename T, int ROWS, int BK, bool KC>
DEV void e_store(const EStage<T, ROWS, BK>& s, T* lds) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < EStage<T, ROWS, BK>::PER; ++e) {
    int idx = t + e * NT;
    int r, k;
    if (KC) { r = idx / BK; k = idx % BK; } else { k = idx / ROWS; r = idx % ROWS; }
    lds[r * (BK + 1) + k] = s.v[e];
  }
}

// Accumulators of one wave: FM x FN blocks of 16 x 16.
template <typename T, int BM, int BN>
struct EFrag {
  static constexpr int FM = BM / 32, FN = BN / 32;
  typename EAcc<T>::V c[FM][FN];
  DEVM void zero() {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) c[a][b][r] = T(0);
  }
};

// Wave (wm, wn) owns rows [wm*BM/2, +BM/2) and columns [wn*BN/2, +BN/2).
template <typename T, int BM, int BN, int BK>
DEV void e_compute(EFrag<T, BM, BN>& f, const T* As, const T* Bs) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < BK; ks += 4) {
    T a[EFrag<T, BM, BN>::FM], b[EFrag<T, BM, BN>::FN];
#pragma unroll
    for (int m = 0; m < EFrag<T, BM, BN>::FM; ++m)
      a[m] = As[(wm * (BM / 2) + m * 16 + lr) * (BK + 1) + ks + lk];
#pragma unroll
    for (int n = 0; n < EFrag<T, BM, BN>::FN; ++n)
      b[n] = Bs[(wn * (BN / 2) + n * 16 + lr) * (BK + 1) + ks + lk];
#pragma unroll
    for (int m = 0; m < EFrag<T, BM, BN>::FM; ++m)
#pragma unroll
      for (int n = 0; n < EFrag<T, BM, BN>::FN; ++n) f.c[m][n] = mfma_e<T>(a[m], b[n], f.c[m][n]);
  }
}

// LDS footprint in elements (two buffers per operand)
template <int BM, int BN, int BK>
constexpr int e_lds_elems() { return 2 * (BM + BN) * (BK + 1); }

// Full K loop over [kbeg, kend).  lds must hold e_lds_elems<BM,BN,BK>() T's.
template <typename T, int BM, int BN, int BK, bool AKC, bool BKC>
DEV void e_gemm(EFrag<T, BM, BN>& f, const T* __restrict__ A, long lda, int M, const T* __restrict__ B, long ldb,
                int N, int i0, int j0, int kbeg, int kend, T* lds) {
  T* As[2] = {lds, lds + BM * (BK + 1)};
  T* Bs[2] = {lds + 2 * BM * (BK + 1), lds + 2 * BM * (BK + 1) + BN * (BK + 1)};
  EStage<T, BM, BK> sa;
  EStage<T, BN, BK> sb;
  const int nk = (kend - kbeg + BK - 1) / BK;
  if (nk <= 0) return;
  e_load<T, BM, BK, AKC>(sa, A, lda, M, i0, kbeg, kend);
  e_load<T, BN, BK, BKC>(sb, B, ldb, N, j0, kbeg, kend);
  e_store<T, BM, BK, AKC>(sa, As[0]);
  e_store<T, BN, BK, BKC>(sb, Bs[0]);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      e_load<T, BM, BK, AKC>(sa, A, lda, M, i0, kbeg + (kt + 1) * BK, kend);
      e_load<T, BN, BK, BKC>(sb, B, ldb, N, j0, kbeg + (kt + 1) * BK, kend);
    }
    e_compute<T, BM, BN, BK>(f, As[cur], Bs[cur]);
    if (kt + 1 < nk) {
      e_store<T, BM, BK, AKC>(sa, As[cur ^ 1]);
      e_store<T, BN, BK, BKC>(sb, Bs[cur ^ 1]);
    }
    __syncthreads();
  }
}

// Coordinates of accumulator element (m, n, r) of this lane inside the tile.
// The 16 x 16 result blocks differ in how rows map to registers:
//   f32 / bf16 MFMA: c[r] = C[4*(lane/16) + r][lane%16]
//   f64 MFMA:        c[r] = C[4*r + lane/16][lane%16]
template <int BM, int BN, typename ACC = float>
DEV void frag_coords(int m, int n, int r, int& ti, int& tj) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int rr = (sizeof(ACC) == 8) ? (4 * r + (lane >> 4)) : (4 * (lane >> 4) + r);
  ti = wm * (BM / 2) + m * 16 + rr;
  tj = wn * (BN / 2) + n * 16 + (lane & 15);
}

// ---------------------------------------------------------------------------
// BF16 engine: mfma 16x16x32 bf16 with fp32 accumulation.  Both operands
// must be k-contiguous in global memory (element (r, k) at p[r*ld + k]).
// LDS rows hold BK = 32 bf16 (64 B) plus 8 bf16 of padding.
// ---------------------------------------------------------------------------
constexpr int BBK = 32;
constexpr int BPAD = 8;

template <int ROWS>
struct BStage {
  static constexpr int VEC = 8;                    // bf16 per 16-byte load
  static constexpr int PER = ROWS * BBK / VEC / NT;  // 16-byte chunks per thread
  uint4 v[PER > 0 ? PER : 1];
};

// vec_ok: ld % 8 == 0 and the base is 16-byte aligned (then every chunk is).
template <int ROWS>
DEV void b_load(BStage<ROWS>& s, const u16* __restrict__ p, long ld, int nrows, int r0, int k0, int kend, bool vec_ok) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < BStage<ROWS>::PER; ++e) {
    int idx = t + e * NT;
    int r = idx / (BBK / 8), k = (idx % (BBK / 8)) * 8;
    int gr = r0 + r, gk = k0 + k;
    uint4 val = make_uint4(0, 0, 0, 0);
    if (gr < nrows) {
      const u16* q = p + (long)gr * ld + gk;
      if (vec_ok && gk + 8 <= kend) {
        val = *(const uint4*)q;
      } else {
        u16 h[8];
#pragma unroll
        for (int x = 0; x < 8; ++x) h[x] = (gk + x < kend) ? q[x] : (u16)0;
        val.x = h[0] | ((uint32_t)h[1] << 16);
        val.y = h[2] | ((uint32_t)h[3] << 16);
        val.z = h[4] | ((uint32_t)h[5] << 16);
        val.w = h[6] | ((uint32_t)h[7] << 16);
      }
    }
    s.v[e] = val;
  }
}

template <int ROWS>
DEV void b_store(const BStage<ROWS>& s, u16* lds) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < BStage<ROWS>::PER; ++e) {
    int idx = t + e * NT;
    int r = idx / (BBK / 8), k = (idx % (BBK / 8)) * 8;
    *(uint4*)(lds + r * (BBK + BPAD) + k) = s.v[e];
  }
}

template <int BM, int BN>
struct BFrag {
  static constexpr int FM = BM / 32, FN = BN / 32;
  f4_t c[FM][FN];
  DEVM void zero() {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) c[a][b][r] = 0.f;
  }
};

template <int BM, int BN>
DEV void b_compute(BFrag<BM, BN>& f, const u16* As, const u16* Bs) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  bf8_t a[BFrag<BM, BN>::FM], b[BFrag<BM, BN>::FN];
#pragma unroll
  for (int m = 0; m < BFrag<BM, BN>::FM; ++m)
    a[m] = *(const bf8_t*)(As + (wm * (BM / 2) + m * 16 + lr) * (BBK + BPAD) + lk);
#pragma unroll
  for (int n = 0; n < BFrag<BM, BN>::FN; ++n)
    b[n] = *(const bf8_t*)(Bs + (wn * (BN / 2) + n * 16 + lr) * (BBK + BPAD) + lk);
#pragma unroll
  for (int m = 0; m < BFrag<BM, BN>::FM; ++m)
#pragma unroll
    for (int n = 0; n < BFrag<BM, BN>::FN; ++n) f.c[m][n] = mfma_bf16(a[m], b[n], f.c[m][n]);
}

template <int BM, int BN>
constexpr int b_lds_elems() { return 2 * (BM + BN) * (BBK + BPAD); }

template <int BM, int BN>
DEV void b_gemm(BFrag<BM, BN>& f, const u16* __restrict__ A, long lda, int M, bool avec, const u16* __restrict__ B,
                long ldb, int N, bool bvec, int i0, int j0, int kbeg, int kend, u16* lds) {
  u16* As[2] = {lds, lds + BM * (BBK + BPAD)};
  u16* Bs[2] = {lds + 2 * BM * (BBK + BPAD), lds + 2 * BM * (BBK + BPAD) + BN * (BBK + BPAD)};
  BStage<BM> sa;
  BStage<BN> sb;
  const int nk = (kend - kbeg + BBK - 1) / BBK;
  if (nk <= 0) return;
  b_load<BM>(sa, A, lda, M, i0, kbeg, kend, avec);
  b_load<BN>(sb, B, ldb, N, j0, kbeg, kend, bvec);
  b_store<BM>(sa, As[0]);
  b_store<BN>(sb, Bs[0]);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      b_load<BM>(sa, A, lda, M, i0, kbeg + (kt + 1) * BBK, kend, avec);
      b_load<BN>(sb, B, ldb, N, j0, kbeg + (kt + 1) * BBK, kend, bvec);
    }
    b_compute<BM, BN>(f, As[cur], Bs[cur]);
    if (kt + 1 < nk) {
      b_store<BM>(sa, As[cur ^ 1]);
      b_store<BN>(sb, Bs[cur ^ 1]);
    }
    __syncthreads();
  }
}

}  // namespace gemm
