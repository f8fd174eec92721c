// Internal device helpers shared by the gfx950 kernels of the k-point AFQMC library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/afqmc_kpt.h"

namespace afqmc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// The FP32 and BF16X3 contractions keep complex64 copies of L and Lh.
__host__ __device__ __forceinline__ bool low_prec(int prec) {
  return prec == AFQMC_PREC_FP32 || prec == AFQMC_PREC_BF16X3;
}

// Digits per operand of an int8-split energy precision (0 for the others).
__host__ __device__ __forceinline__ int int8_digits(int prec) {
  return prec == AFQMC_PREC_INT8X5 ? 5 : (prec == AFQMC_PREC_INT8X4 ? 4 : 0);
}

// A placed precision (AFQMC_PREC_PLACE) resolves to the precision of the step contractions
// (force bias, HS potential, Taylor products) and to that of the local energy and its
// adjoint; a plain afqmc_prec value is both.
__host__ __device__ __forceinline__ int step_prec(int prec) { return prec & 15; }
__host__ __device__ __forceinline__ int energy_prec(int prec) {
  return (prec >> 4) ? (prec >> 4) - 1 : (prec & 15);
}

// Complex values as plain (re, im) pairs of the storage type.
template <typename T>
struct cpx {
  T re, im;
};

// MFMA 16x16x4 wrappers.  Lane l of a wave supplies A[l%16][l/16] and B[l/16][l%16]
// and receives four entries of column l%16 of D; their rows depend on the instruction
// (measured on gfx950): FP32 rows 4*(l/16) + v, FP64 rows l/16 + 4*v, v = 0..3.
// drow(lane, v) gives that row.
template <typename T>
struct mfma16;

template <>
struct mfma16<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <>
struct mfma16<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Complex multiply-accumulate of one 16x16x4 block on real MFMA:
//   Dre += Are Bre - Aim Bim,  Dim += Are Bim + Aim Bre.
template <typename T>
__device__ __forceinline__ void cmfma(T ar, T ai, T br, T bi, typename mfma16<T>::acc_t& dr,
                                      typename mfma16<T>::acc_t& di) {
  dr = mfma16<T>::mac(ar, br, dr);
  di = mfma16<T>::mac(ar, bi, di);
  dr = mfma16<T>::mac(-ai, bi, dr);
  di = mfma16<T>::mac(ai, br, di);
}

// Workgroups are dealt round-robin over the 8 XCDs (workgroup i runs on XCD i % 8).  This
// bijection of [0, total) gives XCD x the contiguous range of work items
// [x q + min(x, r), ...) with q = total / 8, r = total % 8, so that items sharing an
// operand stay in one L2.
__device__ __forceinline__ long long xcd_remap(long long bid, long long total) {
  const long long q = total >> 3, r = total & 7;
  const long long x = bid & 7, i = bid >> 3;
  return x * q + (x < r ? x : r) + i;
}

// bfloat16 bits of x, round to nearest even; and the split x = hi + lo (+ O(2^-16 |x|)).
__device__ __forceinline__ unsigned short bf16_bits_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ void bf16_split(float x, unsigned short& hi, unsigned short& lo) {
  hi = bf16_bits_rne(x);
  lo = bf16_bits_rne(x - __uint_as_float((unsigned int)hi << 16));
}

// Split of two floats into packed (hi, lo) BF16 pairs, element 0 in the low half:
// hi = bf16_rne(x), lo = bf16_rne(x - hi) (the difference is exact in FP32).  The
// conversions compile to the packed round-to-nearest-even conversion of gfx950.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void bf16_split2(float x0, float x1, unsigned int& hi,
                                            unsigned int& lo) {
  const bf16x2_t h = {(__bf16)x0, (__bf16)x1};
  hi = __builtin_bit_cast(unsigned int, h);
  const float r0 = x0 - __uint_as_float(hi << 16);
  const float r1 = x1 - __uint_as_float(hi & 0xffff0000u);
  const bf16x2_t l = {(__bf16)r0, (__bf16)r1};
  lo = __builtin_bit_cast(unsigned int, l);
}

// 16x16x32 BF16 MFMA on raw bf16 bits.  Lane l supplies A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16], i < 8; D as for the FP32 16x16x4 instruction.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v4f mfma_bf16(const u16x8& a, const u16x8& b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Negation of eight packed BF16 values: one 32-bit XOR of the two sign bits per register.
// (Written as a vector XOR, the combiner narrows it to 16-bit lanes, which cost three
// instructions per register.)
__device__ __forceinline__ u16x8 bf16_neg(const u16x8& x) {
  typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
  u32x4_t v = __builtin_bit_cast(u32x4_t, x);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    unsigned int r;
    asm("v_xor_b32 %0, 0x80008000, %1" : "=v"(r) : "v"(v[i]));
    v[i] = r;
  }
  return __builtin_bit_cast(u16x8, v);
}

// d += (ah + al)(bh + bl) without the al bl term (three BF16 passes)
__device__ __forceinline__ v4f mul3(const u16x8& ah, const u16x8& al, const u16x8& bh,
                                    const u16x8& bl, v4f d) {
  d = mfma_bf16(al, bh, d);
  d = mfma_bf16(ah, bl, d);
  return mfma_bf16(ah, bh, d);
}

// k-point index algebra on the device (mesh row-major linearisation).
struct KMesh {
  int m0, m1, m2;
  __host__ __device__ __forceinline__ int kmq(int k, int q) const {  // index of k - q
    int k0 = k / (m1 * m2), k1 = (k / m2) % m1, k2 = k % m2;
    int q0 = q / (m1 * m2), q1 = (q / m2) % m1, q2 = q % m2;
    int a = k0 - q0; a += (a < 0) ? m0 : 0;
    int b = k1 - q1; b += (b < 0) ? m1 : 0;
    int c = k2 - q2; c += (c < 0) ? m2 : 0;
    return (a * m1 + b) * m2 + c;
  }
  __host__ __device__ __forceinline__ int neg(int q) const {  // index of -q
    int q0 = q / (m1 * m2), q1 = (q / m2) % m1, q2 = q % m2;
    int a = q0 ? m0 - q0 : 0, b = q1 ? m1 - q1 : 0, c = q2 ? m2 - q2 : 0;
    return (a * m1 + b) * m2 + c;
  }
};

__host__ __device__ __forceinline__ KMesh make_mesh(const afqmc_kpt_problem& p) {
  return KMesh{p.mesh[0], p.mesh[1], p.mesh[2]};
}

template <typename T>
__device__ __forceinline__ cpx<T> ld(const void* base, int64_t idx) {
  const cpx<T>* b = reinterpret_cast<const cpx<T>*>(base);
  return b[idx];
}

// Load a complex128 and return it in the storage precision T.
template <typename T>
__device__ __forceinline__ cpx<T> ld_d(const void* base, int64_t idx) {
  const cpx<double>* b = reinterpret_cast<const cpx<double>*>(base);
  cpx<double> v = b[idx];
  return cpx<T>{(T)v.re, (T)v.im};
}

}  // namespace afqmc
