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
// * deterministic wavefront reductions.
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
// uniform in (0,1) from 24 random bits, exact in fp32
DEV float u01_f32(uint32_t a) { return ((float)(a >> 8) + 0.5f) * 0x1.0p-24f; }

// ---- wavefront reductions (fixed butterfly order: deterministic) ----------
DEV double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
DEV float wave_sum_f32(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }
