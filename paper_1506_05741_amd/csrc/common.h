// Device-side building blocks shared by every DIAM kernel (gfx950 / CDNA4).
//
// * MFMA wrappers with their lane layouts (64-wide wavefront):
//     f64 16x16x4 and f32 16x16x4:  a = A[l%16][l/16], b = B[l/16][l%16]
//     bf16 and f16 16x16x32:        a[e] = A[l%16][8*(l/16)+e], b[e] = B[8*(l/16)+e][l%16]
//     result f32 and bf16:          c[r] = C[4*(l/16)+r][l%16]
//     bf16 and f16 32x32x16:        a[e] = A[l%32][8*(l/32)+e], b[e] = B[8*(l/32)+e][l%32]
//     result (16 floats):           c[r] = C[8*(r/4)+4*(l/32)+r%4][l%32]
//     result f64:                   c[r] = C[4*r+l/16][l%16]
// * bf16 conversion (round to nearest even) and the hi/lo split; the two-part
//   IEEE half split.
// * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals.
// * cross-lane moves and deterministic wavefront reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef float f16v_t __attribute__((ext_vector_type(16)));
typedef uint16_t u16;
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

#define DEV static __device__ __forceinline__
#define DEVM __device__ __forceinline__

DEV d4_t mfma_f64(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
DEV f4_t mfma_f32(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
DEV f4_t mfma_bf16(bf8_t a, bf8_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
DEV f4_t mfma_f16(h8_t a, h8_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
// 32 x 32 x 16: measured on MI355X at about 1.6x the throughput of the
// 16 x 16 x 32 form for the same flops (the larger tile per instruction).
DEV f16v_t mfma32_f16(h8_t a, h8_t b, f16v_t c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}
DEV f16v_t mfma32_bf16(bf8_t a, bf8_t b, f16v_t c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// ---- IEEE half precision ------------------------------------------------------
// hi = f16(v), lo = f16(v - hi) (round to nearest even): hi + lo carries 22
// significant bits of v when |v| lies in the normal range of both parts.
DEV void split_f16(double v, u16& hi, u16& lo) {
  const _Float16 h = (_Float16)(float)v;
  const _Float16 l = (_Float16)(float)(v - (double)h);
  hi = __builtin_bit_cast(u16, h);
  lo = __builtin_bit_cast(u16, l);
}

// ---- bfloat16 -------------------------------------------------------------
// Round-to-nearest-even from fp32; inputs are finite in every use here.
DEV u16 f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (u16)(u >> 16);
}
DEV float bf16_bits_to_f32(u16 h) { return __uint_as_float(((uint32_t)h) << 16); }

// hi = bf16(w), lo = bf16(w - hi): hi + lo carries 16 significant bits of w.
DEV void split_bf16(float w, u16& hi, u16& lo) {
  hi = f32_to_bf16_bits(w);
  lo = f32_to_bf16_bits(w - bf16_bits_to_f32(hi));
}

// ---- Philox4x32-10 --------------------------------------------------------
struct u4_t { uint32_t x, y, z, w; };

DEV u4_t philox4x32_10(u4_t c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    u4_t n;
    n.x = hi1 ^ c.y ^ k0;
    n.y = lo1;
    n.z = hi0 ^ c.w ^ k1;
    n.w = lo0;
    c = n;
  }
  return c;
}

// uniform in (0,1) from 52 random bits: (k + 0.5) 2^-52, exact in fp64
DEV double u01_f64(uint32_t a, uint32_t b) {
  uint64_t k = (((uint64_t)a << 32) | b) >> 12;
  return ((double)k + 0.5) * 0x1.0p-52;
}
// uniform in (0,1) from 24 random bits, exact in fp32; a Box-Muller radius
// sqrt(-2 ln u) built from it is at most sqrt(50 ln 2) ~ 5.89
DEV float u01_f32(uint32_t a) { return ((float)(a >> 8) + 0.5f) * 0x1.0p-24f; }

// ---- cross-lane moves without the LDS unit ---------------------------------
// The value of lane l ^ OFF, for OFF = 32 and 16 by the gfx950 lane-swap
// instructions (v_permlane32_swap: lanes 32..63 of the first operand trade
// with lanes 0..31 of the second; v_permlane16_swap: odd 16-lane rows of the
// first trade with even rows of the second; with both operands the same
// value, one of the two results holds the partner), OFF = 8 by a rotation of
// each 16-lane row by 8 and OFF = 2, 1 by quad permutations (all exact
// partners for any values).  Every lane of the wavefront must be active.
template <int CTRL> DEV uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
enum { DPP_QUAD_XOR1 = 0xB1, DPP_QUAD_XOR2 = 0x4E, DPP_ROW_ROR4 = 0x124, DPP_ROW_ROR8 = 0x128 };

template <int OFF> DEV uint32_t lane_xor_u32(uint32_t v) {
  static_assert(OFF == 32 || OFF == 16 || OFF == 8 || OFF == 2 || OFF == 1, "no exact move for this offset");
  if (OFF == 32 || OFF == 16) {
    const auto r = OFF == 32 ? __builtin_amdgcn_permlane32_swap(v, v, false, false)
                             : __builtin_amdgcn_permlane16_swap(v, v, false, false);
    const bool low = (__lane_id() & OFF) == 0;
    return low ? r[1] : r[0];
  }
  return dpp_u32<OFF == 8 ? DPP_ROW_ROR8 : OFF == 2 ? DPP_QUAD_XOR2 : DPP_QUAD_XOR1>(v);
}
template <int OFF> DEV float lane_xor_f32(float v) { return __uint_as_float(lane_xor_u32<OFF>(__float_as_uint(v))); }
template <int OFF> DEV double lane_xor_f64(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = lane_xor_u32<OFF>((uint32_t)b), hi = lane_xor_u32<OFF>((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// ---- wavefront reductions (fixed butterfly order: deterministic) ----------
// v + v(l ^ 32), v + v(l ^ 16), ..., v + v(l ^ 1): every lane gets the same
// sum.  The xor-4 partner is taken by rotating each 16-lane row by 4, which
// reaches a lane congruent to l ^ 4 mod 8; after the 32, 16 and 8 steps the
// values depend on the lane only mod 8, so that lane holds the partner's
// value and the sum is the butterfly's bit for bit.
template <typename T> DEV T wave_sum_t(T v) {
  v += sizeof(T) == 8 ? (T)lane_xor_f64<32>((double)v) : (T)lane_xor_f32<32>((float)v);
  v += sizeof(T) == 8 ? (T)lane_xor_f64<16>((double)v) : (T)lane_xor_f32<16>((float)v);
  v += sizeof(T) == 8 ? (T)lane_xor_f64<8>((double)v) : (T)lane_xor_f32<8>((float)v);
  if (sizeof(T) == 8) {
    const uint64_t b = (uint64_t)__double_as_longlong((double)v);
    const uint32_t lo = dpp_u32<DPP_ROW_ROR4>((uint32_t)b), hi = dpp_u32<DPP_ROW_ROR4>((uint32_t)(b >> 32));
    v += (T)__longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
  } else {
    v += (T)__uint_as_float(dpp_u32<DPP_ROW_ROR4>(__float_as_uint((float)v)));
  }
  v += sizeof(T) == 8 ? (T)lane_xor_f64<2>((double)v) : (T)lane_xor_f32<2>((float)v);
  v += sizeof(T) == 8 ? (T)lane_xor_f64<1>((double)v) : (T)lane_xor_f32<1>((float)v);
  return v;
}
DEV double wave_sum_f64(double v) { return wave_sum_t<double>(v); }
DEV float wave_sum_f32(float v) { return wave_sum_t<float>(v); }
// Sum over each 16-lane row in the butterfly order 8, 4, 2, 1 (every lane of
// the row gets it; the xor-4 step as in wave_sum_t).
DEV double row16_sum_f64(double v) {
  v += lane_xor_f64<8>(v);
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = dpp_u32<DPP_ROW_ROR4>((uint32_t)b), hi = dpp_u32<DPP_ROW_ROR4>((uint32_t)(b >> 32));
  v += __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
  v += lane_xor_f64<2>(v);
  v += lane_xor_f64<1>(v);
  return v;
}
// Largest value of the wavefront (every lane gets it; the maximum does not
// depend on the order of the comparisons).
DEV float wave_max_f32(float v) {
  v = fmaxf(v, lane_xor_f32<32>(v));
  v = fmaxf(v, lane_xor_f32<16>(v));
  v = fmaxf(v, lane_xor_f32<8>(v));
  v = fmaxf(v, __uint_as_float(dpp_u32<DPP_ROW_ROR4>(__float_as_uint(v))));
  v = fmaxf(v, lane_xor_f32<2>(v));
  v = fmaxf(v, lane_xor_f32<1>(v));
  return v;
}

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }
