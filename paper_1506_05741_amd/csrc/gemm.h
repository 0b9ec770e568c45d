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

// LDS layout of an operand slice: row r holds its BK values in the order
// k' = (k % 4) * (BK / 4) + k / 4, so the BK/4 values one lane feeds to the
// MFMA (k = lk, lk + 4, ...) are contiguous and load as 16-byte vectors.
// The row stride ELD() is BK plus 16 bytes of padding, which makes the 16
// rows read by a quarter-wavefront land on distinct banks.
template <typename T, int BK>
constexpr int eld() { return BK + 16 / (int)sizeof(T); }
template <int BK>
DEV int eperm(int k) { return (k & 3) * (BK / 4) + (k >> 2); }

// Element (r, k) at which staging vector c of an operand slice starts; the
// vector runs along k (KC) or along r.  Column-major FP64 slices with BK = 16
// give the 16 lanes of a quarter-wavefront four row pairs at four k = k0,
// k0 + 4, k0 + 8, k0 + 12, whose LDS slots (order eperm) are adjacent, so
// their 8-byte LDS stores cover the banks once, where sixteen row pairs at
// one k put four lanes on each bank.  Lane bits 0 and 3 pick the k, bits 1,
// 2 and 4 the row pair: each group of 8 lanes then also stores both rows of
// its pairs on distinct banks.  Column-major FP32 slices with BK = 32 (a
// vector is four rows at one k): lane bits 0 and 1 pick k among four values
// four apart, bit 2 the neighbour k + 1, bits 3 to 5 one of eight row quads.
// Where sixteen row quads at four adjacent k put eight lanes on one bank, a
// wavefront's stores then meet each bank at most twice, and its global reads
// stay eight 128-byte column segments.  Which thread moves which element
// changes nothing else.
template <typename T, int ROWS, int BK, bool KC>
DEV void e_slot(int c, int& r, int& k) {
  constexpr int VEC = 16 / (int)sizeof(T);
  if (KC) {
    r = c / (BK / VEC);
    k = (c % (BK / VEC)) * VEC;
  } else if (sizeof(T) == 8 && BK == 16 && ROWS % 16 == 0) {
    const int hi = c >> 5;
    const int q = (c & 1) | ((c >> 2) & 2);
    const int jp = ((c >> 1) & 3) | ((c >> 2) & 4);
    r = 2 * (jp + 8 * (hi >> 2));
    k = (hi & 3) + 4 * q;
  } else if (sizeof(T) == 4 && BK == 32 && ROWS % 16 == 0) {
    const int kh = (c & 3) | (((c >> 6) & 1) << 2);
    const int j = ((c >> 3) & 7) | ((c >> 8) << 3);
    r = 4 * j;
    k = 4 * kh + ((c >> 2) & 1) + 2 * ((c >> 7) & 1);
  } else {
    k = c / (ROWS / VEC);
    r = (c % (ROWS / VEC)) * VEC;
  }
}

// Staging registers of one operand slice (ROWS x BK) for one thread of a
// 256-thread k-group: NV vectors of VEC elements (16 bytes each).
template <typename T, int ROWS, int BK>
struct EStage {
  static constexpr int VEC = 16 / (int)sizeof(T);
  static constexpr int NV = ROWS * BK / VEC / NT;
  static_assert(NV >= 1 && BK % VEC == 0 && ROWS % VEC == 0, "tile too small for 16-byte staging");
  T v[NV * VEC];
};

// Load an operand slice [r0, r0+ROWS) x [k0, k0+BK) into registers.  Each
// thread moves 16-byte vectors along the operand's contiguous direction.
// FAST: the slice lies inside the operand and is aligned (no guards, so the
// compiler keeps the loads in flight across the MFMA work); otherwise every
// element is range-checked and read as zero outside.
template <typename T, int ROWS, int BK, bool KC, bool FAST>
DEV void e_load(EStage<T, ROWS, BK>& s, int t, const T* __restrict__ p, long ld, int nrows, int r0, int k0, int kend) {
  constexpr int VEC = EStage<T, ROWS, BK>::VEC;
#pragma unroll
  for (int e = 0; e < EStage<T, ROWS, BK>::NV; ++e) {
    const int c = t + e * NT;
    int r, k;
    e_slot<T, ROWS, BK, KC>(c, r, k);
    const int gr = r0 + r, gk = k0 + k;
    T* dst = &s.v[e * VEC];
    const T* q = KC ? p + (long)gr * ld + gk : p + gr + (long)gk * ld;
    if (FAST) {
      *(u32x4_t*)dst = *(const u32x4_t*)q;
    } else {
#pragma unroll
      for (int x = 0; x < VEC; ++x) {
        const bool ok = KC ? (gr < nrows && gk + x < kend) : (gr + x < nrows && gk < kend);
        dst[x] = ok ? q[x] : T(0);
      }
    }
  }
}

template <typename T, int ROWS, int BK, bool KC>
DEV void e_store(const EStage<T, ROWS, BK>& s, int t, T* lds) {
  constexpr int VEC = EStage<T, ROWS, BK>::VEC;
  constexpr int LD = eld<T, BK>();
#pragma unroll
  for (int e = 0; e < EStage<T, ROWS, BK>::NV; ++e) {
    const int c = t + e * NT;
    int r, k;
    e_slot<T, ROWS, BK, KC>(c, r, k);
#pragma unroll
    for (int x = 0; x < VEC; ++x) {
      if (KC) lds[r * LD + eperm<BK>(k + x)] = s.v[e * VEC + x];
      else lds[(r + x) * LD + eperm<BK>(k)] = s.v[e * VEC + x];
    }
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

// Wave (wm, wn) of a k-group owns rows [wm*BM/2, +BM/2) and columns
// [wn*BN/2, +BN/2) of the tile.  Each lane reads its BK/4 operand values per
// block row as 16-byte vectors, then issues BK/4 MFMAs per block pair.
template <typename T, int BM, int BN, int BK>
DEV void e_compute(EFrag<T, BM, BN>& f, const T* As, const T* Bs) {
  constexpr int FM = EFrag<T, BM, BN>::FM, FN = EFrag<T, BM, BN>::FN, Q = BK / 4;
  constexpr int LD = eld<T, BK>();
  const int lane = threadIdx.x & 63, w = (threadIdx.x & (NT - 1)) >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int lr = lane & 15, lk = lane >> 4;
  T a[FM][Q], b[FN][Q];
#pragma unroll
  for (int m = 0; m < FM; ++m) {
    const T* src = As + (wm * (BM / 2) + m * 16 + lr) * LD + lk * Q;
#pragma unroll
    for (int v = 0; v < Q; v += 16 / (int)sizeof(T)) *(u32x4_t*)&a[m][v] = *(const u32x4_t*)(src + v);
  }
#pragma unroll
  for (int n = 0; n < FN; ++n) {
    const T* src = Bs + (wn * (BN / 2) + n * 16 + lr) * LD + lk * Q;
#pragma unroll
    for (int v = 0; v < Q; v += 16 / (int)sizeof(T)) *(u32x4_t*)&b[n][v] = *(const u32x4_t*)(src + v);
  }
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int m = 0; m < FM; ++m)
#pragma unroll
      for (int n = 0; n < FN; ++n) f.c[m][n] = mfma_e<T>(a[m][q], b[n][q], f.c[m][n]);
}

// LDS footprint of one k-group in elements (two buffers per operand).
template <typename T, int BM, int BN, int BK>
constexpr int e_lds_elems() { return 2 * (BM + BN) * eld<T, BK>(); }

template <typename T, int BM, int BN, int BK, bool AKC, bool BKC, bool FAST>
DEV void e_loop(EFrag<T, BM, BN>& f, const T* __restrict__ A, long lda, int M, const T* __restrict__ B, long ldb,
                int N, int i0, int j0, int kbeg, int kend, T* base, int g, int t, int KG, int nit) {
  constexpr int LD = eld<T, BK>();
  // the two buffers are fixed offsets from the shared array (the loop is
  // unrolled by two), so every access compiles to an LDS instruction
  T* const A0 = base;
  T* const A1 = base + BM * LD;
  T* const B0 = base + 2 * BM * LD;
  T* const B1 = base + 2 * BM * LD + BN * LD;
  EStage<T, BM, BK> sa;
  EStage<T, BN, BK> sb;
  e_load<T, BM, BK, AKC, FAST>(sa, t, A, lda, M, i0, kbeg + g * BK, kend);
  e_load<T, BN, BK, BKC, FAST>(sb, t, B, ldb, N, j0, kbeg + g * BK, kend);
  e_store<T, BM, BK, AKC>(sa, t, A0);
  e_store<T, BN, BK, BKC>(sb, t, B0);
  __syncthreads();
  for (int it = 0; it < nit; it += 2) {
    {
      const int kn = kbeg + ((it + 1) * KG + g) * BK;
      const bool more = it + 1 < nit;
      if (more) {
        e_load<T, BM, BK, AKC, FAST>(sa, t, A, lda, M, i0, kn, kend);
        e_load<T, BN, BK, BKC, FAST>(sb, t, B, ldb, N, j0, kn, kend);
      }
      e_compute<T, BM, BN, BK>(f, A0, B0);
      if (more) {
        e_store<T, BM, BK, AKC>(sa, t, A1);
        e_store<T, BN, BK, BKC>(sb, t, B1);
      }
      __syncthreads();
      if (!more) break;
    }
    {
      const int kn = kbeg + ((it + 2) * KG + g) * BK;
      const bool more = it + 2 < nit;
      if (more) {
        e_load<T, BM, BK, AKC, FAST>(sa, t, A, lda, M, i0, kn, kend);
        e_load<T, BN, BK, BKC, FAST>(sb, t, B, ldb, N, j0, kn, kend);
      }
      e_compute<T, BM, BN, BK>(f, A1, B1);
      if (more) {
        e_store<T, BM, BK, AKC>(sa, t, A0);
        e_store<T, BN, BK, BKC>(sb, t, B0);
      }
      __syncthreads();
    }
  }
}

// K loop over [kbeg, kend) by a workgroup of KG k-groups of 256 threads.
// k-group g takes the BK-slices g, g + KG, g + 2 KG, ... with its own double
// buffer, so each SIMD runs KG wavefronts; at the end the groups' partial
// accumulators are added into group 0 in fixed order (deterministic).  Only
// group 0's accumulators hold the result.  lds: KG * e_lds_elems elements.
// Tiles that lie inside both operands with aligned rows take the unguarded
// fast loop over whole rounds of KG slices and a guarded loop for the rest.
template <typename T, int BM, int BN, int BK, bool AKC, bool BKC, int KG = 1>
DEV void e_gemm(EFrag<T, BM, BN>& f, const T* __restrict__ A, long lda, int M, const T* __restrict__ B, long ldb,
                int N, int i0, int j0, int kbeg, int kend, T* lds) {
  static_assert(KG == 1 || (KG - 1) * BM * BN <= KG * e_lds_elems<T, BM, BN, BK>(), "exchange does not fit");
  constexpr int VEC = 16 / (int)sizeof(T);
  const int g = threadIdx.x / NT, t = threadIdx.x % NT;
  T* base = lds + g * e_lds_elems<T, BM, BN, BK>();
  const int nk = (kend - kbeg + BK - 1) / BK;
  const int nit = (nk + KG - 1) / KG;
  const bool aligned = ((uintptr_t)A % 16 == 0) && (lda % VEC == 0) && ((uintptr_t)B % 16 == 0) &&
                       (ldb % VEC == 0) && (kbeg % VEC == 0);
  const bool fast = aligned && (i0 + BM <= M) && (j0 + BN <= N);
  if (nit > 0) {
    if (fast) {
      // whole rounds of KG slices unguarded, the remaining slices guarded;
      // slice s still goes to k-group s % KG, as in a single guarded loop
      const int nfull = (kend - kbeg) / (BK * KG);
      const int kmid = kbeg + nfull * BK * KG;
      if (nfull > 0)
        e_loop<T, BM, BN, BK, AKC, BKC, true>(f, A, lda, M, B, ldb, N, i0, j0, kbeg, kmid, base, g, t, KG, nfull);
      if (kmid < kend) {
        const int nit2 = ((kend - kmid + BK - 1) / BK + KG - 1) / KG;
        e_loop<T, BM, BN, BK, AKC, BKC, false>(f, A, lda, M, B, ldb, N, i0, j0, kmid, kend, base, g, t, KG, nit2);
      }
    } else {
      e_loop<T, BM, BN, BK, AKC, BKC, false>(f, A, lda, M, B, ldb, N, i0, j0, kbeg, kend, base, g, t, KG, nit);
    }
  }
  if (KG > 1) {
    constexpr int FM = EFrag<T, BM, BN>::FM, FN = EFrag<T, BM, BN>::FN;
    const int lane = threadIdx.x & 63, w = t >> 6;
    if (g > 0) {
#pragma unroll
      for (int m = 0; m < FM; ++m)
#pragma unroll
        for (int n = 0; n < FN; ++n)
#pragma unroll
          for (int r = 0; r < 4; ++r) lds[(((((g - 1) * 4 + w) * FM + m) * FN + n) * 4 + r) * 64 + lane] = f.c[m][n][r];
    }
    __syncthreads();
    if (g == 0) {
      for (int gg = 1; gg < KG; ++gg)
#pragma unroll
        for (int m = 0; m < FM; ++m)
#pragma unroll
          for (int n = 0; n < FN; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              f.c[m][n][r] += lds[(((((gg - 1) * 4 + w) * FM + m) * FN + n) * 4 + r) * 64 + lane];
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
  const int lane = threadIdx.x & 63, w = (threadIdx.x & (NT - 1)) >> 6;
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
  // fixed buffer offsets, loop unrolled by two: LDS instructions throughout
  u16* const A0 = lds;
  u16* const A1 = lds + BM * (BBK + BPAD);
  u16* const B0 = lds + 2 * BM * (BBK + BPAD);
  u16* const B1 = lds + 2 * BM * (BBK + BPAD) + BN * (BBK + BPAD);
  BStage<BM> sa;
  BStage<BN> sb;
  const int nk = (kend - kbeg + BBK - 1) / BBK;
  if (nk <= 0) return;
  b_load<BM>(sa, A, lda, M, i0, kbeg, kend, avec);
  b_load<BN>(sb, B, ldb, N, j0, kbeg, kend, bvec);
  b_store<BM>(sa, A0);
  b_store<BN>(sb, B0);
  __syncthreads();
  for (int kt = 0; kt < nk; kt += 2) {
    {
      const bool more = kt + 1 < nk;
      if (more) {
        b_load<BM>(sa, A, lda, M, i0, kbeg + (kt + 1) * BBK, kend, avec);
        b_load<BN>(sb, B, ldb, N, j0, kbeg + (kt + 1) * BBK, kend, bvec);
      }
      b_compute<BM, BN>(f, A0, B0);
      if (more) {
        b_store<BM>(sa, A1);
        b_store<BN>(sb, B1);
      }
      __syncthreads();
      if (!more) break;
    }
    {
      const bool more = kt + 2 < nk;
      if (more) {
        b_load<BM>(sa, A, lda, M, i0, kbeg + (kt + 2) * BBK, kend, avec);
        b_load<BN>(sb, B, ldb, N, j0, kbeg + (kt + 2) * BBK, kend, bvec);
      }
      b_compute<BM, BN>(f, A1, B1);
      if (more) {
        b_store<BM>(sa, A0);
        b_store<BN>(sb, B0);
      }
      __syncthreads();
    }
  }
}

// Segmented K loop for the bf16 engine: nseg segments each covering
// [0, kend) of K, segment s reading A + (s & 1) * dA and B + (s >> 1) * dB.
// With hi/lo operand pairs laid out at fixed element offsets this forms
// (A_hi + A_lo)(B_hi + B_lo) in one pipelined loop.
template <int BM, int BN>
DEV void b_gemm_seg(BFrag<BM, BN>& f, const u16* __restrict__ A, long dA, long lda, int M, const u16* __restrict__ B,
                    long dB, long ldb, int N, bool vec, int i0, int j0, int kend, int nseg, u16* lds) {
  u16* const A0 = lds;
  u16* const A1 = lds + BM * (BBK + BPAD);
  u16* const B0 = lds + 2 * BM * (BBK + BPAD);
  u16* const B1 = lds + 2 * BM * (BBK + BPAD) + BN * (BBK + BPAD);
  BStage<BM> sa;
  BStage<BN> sb;
  const int nks = (kend + BBK - 1) / BBK;
  const int nk = nks * nseg;
  if (nks <= 0) return;
  auto load = [&](int kt) {
    const int sgm = kt / nks, k0 = (kt - sgm * nks) * BBK;
    b_load<BM>(sa, A + (sgm & 1) * dA, lda, M, i0, k0, kend, vec);
    b_load<BN>(sb, B + (sgm >> 1) * dB, ldb, N, j0, k0, kend, vec);
  };
  load(0);
  b_store<BM>(sa, A0);
  b_store<BN>(sb, B0);
  __syncthreads();
  for (int kt = 0; kt < nk; kt += 2) {
    {
      const bool more = kt + 1 < nk;
      if (more) load(kt + 1);
      b_compute<BM, BN>(f, A0, B0);
      if (more) {
        b_store<BM>(sa, A1);
        b_store<BN>(sb, B1);
      }
      __syncthreads();
      if (!more) break;
    }
    {
      const bool more = kt + 2 < nk;
      if (more) load(kt + 2);
      b_compute<BM, BN>(f, A1, B1);
      if (more) {
        b_store<BM>(sa, A0);
        b_store<BN>(sb, B0);
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Wide BF16 engine: WGM x WGN wavefronts (64 * WGM * WGN threads) over a
// BM x BN tile, each wave holding a BM/WGM x BN/WGN block of 16 x 16
// accumulators; K is staged through LDS in 64-deep slices (two 16x16x32
// MFMA k-steps per slice) with double buffering, the next slice's global
// loads in flight while the current one is multiplied.  Large wave blocks
// cut LDS reads per MFMA (a fragment read feeds FN or FM MFMAs).
// Segmented K as b_gemm_seg (hi/lo operand pairs).
// ---------------------------------------------------------------------------
constexpr int WBK = 64;
constexpr int WLD = WBK + 8;  // LDS row stride (bf16): 144 bytes

template <int BM, int BN, int WGM, int WGN>
struct WFrag {
  static constexpr int NTH = 64 * WGM * WGN;
  static constexpr int FM = BM / (16 * WGM), FN = BN / (16 * WGN);
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

template <int ROWS, int NTH>
struct WStage {
  static constexpr int PER = ROWS * WBK / 8 / NTH;  // 16-byte chunks per thread
  static_assert(PER >= 1, "tile too small for the wide engine");
  uint4 v[PER];
};

template <int ROWS, int NTH>
DEV void w_load(WStage<ROWS, NTH>& s, const u16* __restrict__ p, long ld, int nrows, int r0, int k0, int kend,
                bool vec_ok) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < WStage<ROWS, NTH>::PER; ++e) {
    const int idx = t + e * NTH;
    const int r = idx >> 3, k = (idx & 7) * 8;
    const int gr = r0 + r, gk = k0 + k;
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

template <int ROWS, int NTH>
DEV void w_store(const WStage<ROWS, NTH>& s, u16* lds) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < WStage<ROWS, NTH>::PER; ++e) {
    const int idx = t + e * NTH;
    const int r = idx >> 3, k = (idx & 7) * 8;
    *(uint4*)(lds + r * WLD + k) = s.v[e];
  }
}

template <int BM, int BN, int WGM, int WGN>
DEV void w_compute(WFrag<BM, BN, WGM, WGN>& f, const u16* As, const u16* Bs) {
  typedef WFrag<BM, BN, WGM, WGN> F;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w % WGM, wn = w / WGM;
  const int lr = lane & 15, lk = (lane >> 4) * 8;
#pragma unroll
  for (int ks = 0; ks < WBK; ks += 32) {
    bf8_t a[F::FM], b[F::FN];
#pragma unroll
    for (int m = 0; m < F::FM; ++m) a[m] = *(const bf8_t*)(As + (wm * (BM / WGM) + m * 16 + lr) * WLD + ks + lk);
#pragma unroll
    for (int n = 0; n < F::FN; ++n) b[n] = *(const bf8_t*)(Bs + (wn * (BN / WGN) + n * 16 + lr) * WLD + ks + lk);
#pragma unroll
    for (int m = 0; m < F::FM; ++m)
#pragma unroll
      for (int n = 0; n < F::FN; ++n) f.c[m][n] = mfma_bf16(a[m], b[n], f.c[m][n]);
  }
}

template <int BM, int BN>
constexpr int w_lds_elems() { return 2 * (BM + BN) * WLD; }

// Coordinates of accumulator (m, n, r) of this lane inside the tile.
template <int BM, int BN, int WGM, int WGN>
DEV void w_coords(int m, int n, int r, int& ti, int& tj) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w % WGM, wn = w / WGM;
  ti = wm * (BM / WGM) + m * 16 + 4 * (lane >> 4) + r;
  tj = wn * (BN / WGN) + n * 16 + (lane & 15);
}

// K range [kbeg, kend) per segment (kbeg a multiple of 8 for vector loads).
template <int BM, int BN, int WGM, int WGN>
DEV void w_gemm_seg(WFrag<BM, BN, WGM, WGN>& f, const u16* __restrict__ A, long dA, long lda, int M,
                    const u16* __restrict__ B, long dB, long ldb, int N, bool vec, int i0, int j0, int kbeg, int kend,
                    int nseg, u16* lds) {
  constexpr int NTH = 64 * WGM * WGN;
  u16* const A0 = lds;
  u16* const A1 = lds + BM * WLD;
  u16* const B0 = lds + 2 * BM * WLD;
  u16* const B1 = lds + 2 * BM * WLD + BN * WLD;
  WStage<BM, NTH> sa;
  WStage<BN, NTH> sb;
  const int nks = (kend - kbeg + WBK - 1) / WBK;
  const int nk = nks * nseg;
  if (nks <= 0) return;
  auto load = [&](int kt) {
    const int sgm = kt / nks, k0 = kbeg + (kt - sgm * nks) * WBK;
    w_load<BM, NTH>(sa, A + (sgm & 1) * dA, lda, M, i0, k0, kend, vec);
    w_load<BN, NTH>(sb, B + (sgm >> 1) * dB, ldb, N, j0, k0, kend, vec);
  };
  load(0);
  w_store<BM, NTH>(sa, A0);
  w_store<BN, NTH>(sb, B0);
  __syncthreads();
  for (int kt = 0; kt < nk; kt += 2) {
    {
      const bool more = kt + 1 < nk;
      if (more) load(kt + 1);
      w_compute<BM, BN, WGM, WGN>(f, A0, B0);
      if (more) {
        w_store<BM, NTH>(sa, A1);
        w_store<BN, NTH>(sb, B1);
      }
      __syncthreads();
      if (!more) break;
    }
    {
      const bool more = kt + 2 < nk;
      if (more) load(kt + 2);
      w_compute<BM, BN, WGM, WGN>(f, A1, B1);
      if (more) {
        w_store<BM, NTH>(sa, A0);
        w_store<BN, NTH>(sb, B0);
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Hi/lo BF16 engine with direct-to-LDS loads.  C = (A_hi + A_lo)(B_hi + B_lo)
// over K: each 32-deep K slice of all four operand parts is copied from
// global memory straight into an LDS ring of ST stages by
// global_load_lds_dwordx4 (no staging registers; ST - 1 slices in flight),
// and every fragment read from LDS feeds two of the four products.  Each
// wave-wide copy fills 1 KB of LDS = 16 rows x 4 chunks of 16 bytes; chunk c
// of row r sits at position c ^ hswz(r).  The swizzle puts the rows that one
// LDS cycle serves on distinct banks whether a 16-byte read is served 8 or 16
// lanes at a time (rows r and r + 2 share the 128-byte bank row of 64-byte
// rows, rows r and r + 4 the 256-byte one); it depends on r mod 16 only, so
// global and tile-local row numbers give the same placement.  Unguarded: the caller
// guarantees that all rows and the whole K range lie inside the operands
// (K a multiple of 32) and that rows start on 16-byte boundaries.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void* lds_ptr_t;
constexpr int HBK = 32;

DEV int hswz(int r) { return ((r >> 2) ^ (r >> 1)) & 3; }

DEV void h_copy_block(const u16* __restrict__ p, long ld, int r0, int k0, u16* lds_block) {
  const int lane = threadIdx.x & 63;
  const int r = r0 + (lane >> 2);
  const int c = (lane & 3) ^ hswz(r);
  __builtin_amdgcn_global_load_lds((const void*)(p + (long)r * ld + k0 + c * 8), (lds_ptr_t)lds_block, 16, 0, 0);
}

template <int BM, int BN, int ST>
constexpr int h_lds_elems() { return ST * 2 * (BM + BN) * HBK; }

template <int BM, int BN, int WGM, int WGN, int ST>
DEV void h_gemm(WFrag<BM, BN, WGM, WGN>& f, const u16* __restrict__ A, long dA, long lda, const u16* __restrict__ B,
                long dB, long ldb, int i0, int j0, int kend, u16* lds) {
  typedef WFrag<BM, BN, WGM, WGN> F;
  constexpr int NW = WGM * WGN;
  constexpr int SA = BM * HBK, SB = BN * HBK, SS = 2 * (SA + SB);
  constexpr int BLK_A = BM / 16, BLK_B = BN / 16, NBLK = 2 * (BLK_A + BLK_B);
  static_assert(NBLK % NW == 0, "copy blocks must divide among the waves");
  constexpr int LPW = NBLK / NW;
  const int nk = kend / HBK;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  auto issue = [&](int kt) {
    const int k0 = kt * HBK;
    u16* st = lds + (kt % ST) * SS;
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
      const int blk = w * LPW + q;
      if (blk < 2 * BLK_A) {
        const int h = blk / BLK_A, b = blk % BLK_A;
        h_copy_block(A + h * dA, lda, i0 + b * 16, k0, st + h * SA + b * 512);
      } else {
        const int bb = blk - 2 * BLK_A, h = bb / BLK_B, b = bb % BLK_B;
        h_copy_block(B + h * dB, ldb, j0 + b * 16, k0, st + 2 * SA + h * SB + b * 512);
      }
    }
  };
  const int wm = w % WGM, wn = w / WGM;
  const int lr = lane & 15, lk = lane >> 4;
  // the ring may still be read by other waves from a previous call
  asm volatile("s_barrier" ::: "memory");
  for (int p = 0; p < ST - 1 && p < nk; ++p) issue(p);
  for (int kt = 0; kt < nk; ++kt) {
    // this wave's copies of slice kt are done when at most the later
    // slices' copies are outstanding; the barrier then covers all waves
    // stage kt has landed once at most the later stages' copies are pending
    if (kt + ST - 2 < nk) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LPW * (ST - 2)) : "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    asm volatile("s_barrier" ::: "memory");
    // the ring slot refilled here was last read before this barrier
    if (kt + ST - 1 < nk) issue(kt + ST - 1);
    const u16* st = lds + (kt % ST) * SS;
    bf8_t ah[F::FM], al[F::FM], bh[F::FN], bl[F::FN];
#pragma unroll
    for (int m = 0; m < F::FM; ++m) {
      const int r = wm * (BM / WGM) + m * 16 + lr;
      const int o = r * HBK + ((lk ^ hswz(r)) * 8);
      ah[m] = *(const bf8_t*)(st + o);
      al[m] = *(const bf8_t*)(st + SA + o);
    }
#pragma unroll
    for (int n = 0; n < F::FN; ++n) {
      const int r = wn * (BN / WGN) + n * 16 + lr;
      const int o = r * HBK + ((lk ^ hswz(r)) * 8);
      bh[n] = *(const bf8_t*)(st + 2 * SA + o);
      bl[n] = *(const bf8_t*)(st + 2 * SA + SB + o);
    }
#pragma unroll
    for (int m = 0; m < F::FM; ++m)
#pragma unroll
      for (int n = 0; n < F::FN; ++n) {
        f.c[m][n] = mfma_bf16(ah[m], bh[n], f.c[m][n]);
        f.c[m][n] = mfma_bf16(al[m], bh[n], f.c[m][n]);
        f.c[m][n] = mfma_bf16(ah[m], bl[n], f.c[m][n]);
        f.c[m][n] = mfma_bf16(al[m], bl[n], f.c[m][n]);
      }
  }
}

// Plain BF16 engine with direct-to-LDS loads (one part per operand): 64-deep
// K slices, chunk c of row r at position c ^ pswz(r) (8 chunks per 128-byte
// row, conflict-free for 8 or 16 lanes per LDS cycle like hswz), ST-stage ring.  K range [kbeg, kend), both multiples of 64;
// unguarded like h_gemm.
constexpr int PBK = 64;

DEV int pswz(int r) { return (r & 7) ^ ((r >> 3) & 1); }

DEV void p_copy_block(const u16* __restrict__ p, long ld, int r0, int k0, u16* lds_block) {
  const int lane = threadIdx.x & 63;
  const int r = r0 + (lane >> 3);
  const int c = (lane & 7) ^ pswz(r);
  __builtin_amdgcn_global_load_lds((const void*)(p + (long)r * ld + k0 + c * 8), (lds_ptr_t)lds_block, 16, 0, 0);
}

template <int BM, int BN, int ST>
constexpr int p_lds_elems() { return ST * (BM + BN) * PBK; }

template <int BM, int BN, int WGM, int WGN, int ST>
DEV void p_gemm(WFrag<BM, BN, WGM, WGN>& f, const u16* __restrict__ A, long lda, const u16* __restrict__ B, long ldb,
                int i0, int j0, int kbeg, int kend, u16* lds) {
  typedef WFrag<BM, BN, WGM, WGN> F;
  constexpr int NW = WGM * WGN;
  constexpr int SA = BM * PBK, SS = (BM + BN) * PBK;
  constexpr int BLK_A = BM / 8, BLK_B = BN / 8, NBLK = BLK_A + BLK_B;
  static_assert(NBLK % NW == 0, "copy blocks must divide among the waves");
  constexpr int LPW = NBLK / NW;
  const int nk = (kend - kbeg) / PBK;
  // wave index in a scalar register: the copy assignment below branches per wave, not per lane
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  auto issue = [&](int kt) {
    const int k0 = kbeg + kt * PBK;
    u16* st = lds + (kt % ST) * SS;
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
      const int blk = w * LPW + q;
      if (blk < BLK_A) p_copy_block(A, lda, i0 + blk * 8, k0, st + blk * 512);
      else p_copy_block(B, ldb, j0 + (blk - BLK_A) * 8, k0, st + SA + (blk - BLK_A) * 512);
    }
  };
  const int wm = w % WGM, wn = w / WGM;
  const int lr = lane & 15, lk = lane >> 4;
  // the ring may still be read by other waves from a previous call
  asm volatile("s_barrier" ::: "memory");
  for (int p = 0; p < ST - 1 && p < nk; ++p) issue(p);
  for (int kt = 0; kt < nk; ++kt) {
    // stage kt has landed once at most the later stages' copies are pending
    if (kt + ST - 2 < nk) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LPW * (ST - 2)) : "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    asm volatile("s_barrier" ::: "memory");
    if (kt + ST - 1 < nk) issue(kt + ST - 1);
    const u16* As = lds + (kt % ST) * SS;
    const u16* Bs = As + SA;
#pragma unroll
    for (int ks = 0; ks < PBK / 32; ++ks) {
      bf8_t a[F::FM], b[F::FN];
#pragma unroll
      for (int m = 0; m < F::FM; ++m) {
        const int r = wm * (BM / WGM) + m * 16 + lr, c = ks * 4 + lk;
        a[m] = *(const bf8_t*)(As + r * PBK + ((c ^ pswz(r)) * 8));
      }
#pragma unroll
      for (int n = 0; n < F::FN; ++n) {
        const int r = wn * (BN / WGN) + n * 16 + lr, c = ks * 4 + lk;
        b[n] = *(const bf8_t*)(Bs + r * PBK + ((c ^ pswz(r)) * 8));
      }
#pragma unroll
      for (int m = 0; m < F::FM; ++m)
#pragma unroll
        for (int n = 0; n < F::FN; ++n) f.c[m][n] = mfma_bf16(a[m], b[n], f.c[m][n]);
    }
  }
}

// Two-part IEEE half engine (the mixed form's target contraction).  Both
// operands are given as x = x0 + x1 with f16 parts (11 significant bits
// each, scaled by powers of two into the f16 range by the caller); per 32-deep
// K slice the three products x1 y0, x0 y1, x0 y0 (everything down to relative
// weight 2^-22) accumulate in FP32, the accuracy of an FP32 product.
// A (rows x K) comes pre-tiled: each part (at element stride dA) is a
// sequence of 1 KB blocks of 16 rows x 32 columns, block (row block rb,
// column block kb) at ((kb * arb) + rb) * 512 with arb = rows / 16, and inside
// a block element (r, k) at r * 32 + ((k / 8) ^ hswz(r)) * 8 + k % 8: the
// order in which h_copy_block leaves a block in LDS, so one tile slice is a
// run of contiguous 1 KB blocks copied without address arithmetic.  B is
// row-major (rows = chains, K contiguous) at leading dimension ldb as in
// h_gemm.  Direct-to-LDS ring of ST stages; K range [kbeg, kend), both
// multiples of 32; unguarded.
template <int BM, int BN, int ST>
constexpr int h2_lds_elems() { return ST * 2 * (BM + BN) * HBK; }

DEV long h2_tile_index(int r, int k, int arb) {
  return ((long)(k >> 5) * arb + (r >> 4)) * 512 + (r & 15) * 32 + ((((k & 31) >> 3) ^ hswz(r)) << 3) + (k & 7);
}

DEV void h_copy_flat(const u16* __restrict__ src, u16* lds_block) {
  const int lane = threadIdx.x & 63;
  __builtin_amdgcn_global_load_lds((const void*)(src + lane * 8), (lds_ptr_t)lds_block, 16, 0, 0);
}

// Accumulators of a 32 x 32-fragment wave tile: the workgroup tile BM x BN
// is split over WGM x WGN waves, each holding FM x FN fragments of 32 x 32.
template <int BM, int BN, int WGM, int WGN>
struct W32Frag {
  static constexpr int FM = BM / (32 * WGM), FN = BN / (32 * WGN);
  static_assert(FM >= 1 && FN >= 1, "wave tile smaller than one 32 x 32 fragment");
  f16v_t c[FM][FN];
  DEVM void zero() {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) c[a][b] = (f16v_t)0.0f;
  }
};

// Tile coordinates of register group g (entries 4g .. 4g + 3, four
// consecutive rows) of fragment (m, n).
template <int BM, int BN, int WGM, int WGN>
DEV void w32_coords(int m, int n, int g, int& ti, int& tj) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w % WGM, wn = w / WGM;
  ti = wm * (BM / WGM) + m * 32 + 8 * g + 4 * (lane >> 5);
  tj = wn * (BN / WGN) + n * 32 + (lane & 31);
}

template <int BM, int BN, int WGM, int WGN, int ST>
DEV void h2_gemm(W32Frag<BM, BN, WGM, WGN>& f, const u16* __restrict__ A, long dA, int arb, const u16* __restrict__ B,
                 long dB, long ldb, int i0, int j0, int kbeg, int kend, u16* lds) {
  // Software-pipelined: the fragments of slice kt + 1 are read from LDS while
  // the products of slice kt run, and copies run ST - 2 slices ahead of the
  // reads.  At the barrier of step kt every wave has completed its reads of
  // slice kt - 1 and stage kt + 1 has landed; the copy of slice kt + ST - 1
  // then refills the stage of slice kt - 1.  Products on the 32 x 32 x 16
  // instruction, two per 32-deep slice and part pair.
  static_assert(ST >= 3, "the pipelined ring needs three stages or more");
  typedef W32Frag<BM, BN, WGM, WGN> F;
  constexpr int NW = WGM * WGN;
  constexpr int SA = BM * HBK, SB = BN * HBK, SS = 2 * (SA + SB);
  constexpr int BLK_A = BM / 16, BLK_B = BN / 16, NBLK = 2 * (BLK_A + BLK_B);
  static_assert(NBLK % NW == 0, "copy blocks must divide among the waves");
  constexpr int LPW = NBLK / NW;
  const int nk = (kend - kbeg) / HBK;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  auto issue = [&](int kt) {
    const int k0 = kbeg + kt * HBK;
    u16* st = lds + (kt % ST) * SS;
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
      const int blk = w * LPW + q;
      if (blk < 2 * BLK_A) {
        const int h = blk / BLK_A, b = blk % BLK_A;
        h_copy_flat(A + h * dA + ((long)(k0 >> 5) * arb + (i0 >> 4) + b) * 512, st + h * SA + b * 512);
      } else {
        const int bb = blk - 2 * BLK_A, h = bb / BLK_B, b = bb % BLK_B;
        h_copy_block(B + h * dB, ldb, j0 + b * 16, k0, st + 2 * SA + h * SB + b * 512);
      }
    }
  };
  const int wm = w % WGM, wn = w / WGM;
  const int lr = lane & 31, lh = lane >> 5;
  // [k half][part][fragment]
  struct Frags {
    h8_t a[2][2][F::FM], b[2][2][F::FN];
  };
  auto read = [&](int kt, Frags& g) {
    const u16* st = lds + (kt % ST) * SS;
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      const int ch = 2 * kh + lh;  // 8-column chunk of the 32-deep slice
#pragma unroll
      for (int m = 0; m < F::FM; ++m) {
        const int r = wm * (BM / WGM) + m * 32 + lr;
        const int o = r * HBK + ((ch ^ hswz(r)) * 8);
        g.a[kh][0][m] = *(const h8_t*)(st + o);
        g.a[kh][1][m] = *(const h8_t*)(st + SA + o);
      }
#pragma unroll
      for (int n = 0; n < F::FN; ++n) {
        const int r = wn * (BN / WGN) + n * 32 + lr;
        const int o = r * HBK + ((ch ^ hswz(r)) * 8);
        g.b[kh][0][n] = *(const h8_t*)(st + 2 * SA + o);
        g.b[kh][1][n] = *(const h8_t*)(st + 2 * SA + SB + o);
      }
    }
  };
  auto mma = [&](const Frags& g) {
#pragma unroll
    for (int kh = 0; kh < 2; ++kh)
#pragma unroll
      for (int m = 0; m < F::FM; ++m)
#pragma unroll
        for (int n = 0; n < F::FN; ++n) {
          // smallest terms first
          f.c[m][n] = mfma32_f16(g.a[kh][1][m], g.b[kh][0][n], f.c[m][n]);
          f.c[m][n] = mfma32_f16(g.a[kh][0][m], g.b[kh][1][n], f.c[m][n]);
          f.c[m][n] = mfma32_f16(g.a[kh][0][m], g.b[kh][0][n], f.c[m][n]);
        }
  };
  auto step = [&](int kt, const Frags& cur, Frags& nxt) {
    if (kt + 1 < nk) {
      // slices issued after kt + 1: min(ST - 3, nk - 2 - kt)
      if (kt + ST - 2 < nk) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LPW * (ST - 3)) : "memory");
      else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    asm volatile("s_barrier" ::: "memory");
    if (kt + ST - 1 < nk) issue(kt + ST - 1);
    // unconditional, so that the products below wait only for the reads of
    // the step before (the last step re-reads a landed stage, unused)
    read(kt + 1 < nk ? kt + 1 : kt, nxt);
    // keep the reads ahead of the products (neither sunk below them nor
    // interleaved by the scheduler); the products use registers whose reads
    // completed at the end of the step before, so they start at once
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    mma(cur);
    // every LDS read of this step done (s_waitcnt lgkmcnt(0), visible to the
    // compiler's wait tracking unlike an asm wait), after the products
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_sched_barrier(0);
  };
  for (int p = 0; p < ST - 1 && p < nk; ++p) issue(p);
  if (nk >= ST - 1) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LPW * (ST - 2)) : "memory");
  else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  asm volatile("s_barrier" ::: "memory");
  Frags fa, fb;
  read(0, fa);
  asm volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_sched_barrier(0);
  for (int kt = 0; kt < nk; kt += 2) {
    step(kt, fa, fb);
    if (kt + 1 < nk) step(kt + 1, fb, fa);
  }
}

}  // namespace gemm
