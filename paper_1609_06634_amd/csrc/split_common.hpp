// Device helpers of the split-precision (matrix-core) posterior kernels.
#pragma once

#include "common.hpp"

namespace bioem {
namespace split {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// hi/lo split of two FP32 values into packed 16-bit pairs.
template <bool BF> struct Prec;
template <> struct Prec<false> {
  using V = h8;
  static __device__ __forceinline__ f4 mma(V a, V b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  // hi = RNE fp16 pair; lo = fp16(x - hi) with the difference taken exactly
  // by a mixed-precision FMA on the fp16 half.
  static __device__ __forceinline__ void split2(float x0, float x1, uint32_t& hi, uint32_t& lo) {
    uint32_t hp, lp;
    float l0, l1;
    asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(hp) : "v"(x0), "v"(x1));
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(l0) : "v"(hp), "v"(x0));
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(l1) : "v"(hp), "v"(x1));
    asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(lp) : "v"(l0), "v"(l1));
    hi = hp;
    lo = lp;
  }
};
template <> struct Prec<true> {
  using V = b8;
  static __device__ __forceinline__ f4 mma(V a, V b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  // hi = upper 16 bits (bf16 truncation, exact as FP32), lo = RNE bf16 of the
  // exact remainder.
  static __device__ __forceinline__ void split2(float x0, float x1, uint32_t& hi, uint32_t& lo) {
    const uint32_t b0 = __float_as_uint(x0) & 0xffff0000u, b1 = __float_as_uint(x1) & 0xffff0000u;
    hi = (b0 >> 16) | b1;
    const float l0 = x0 - __uint_as_float(b0), l1 = x1 - __uint_as_float(b1);
    // both remainders rounded (RNE) and packed by one instruction
    asm("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(lo) : "v"(l0), "v"(l1));
  }
};

template <bool BF>
__device__ __forceinline__ void split8(const float (&x)[8], typename Prec<BF>::V& hi,
                                       typename Prec<BF>::V& lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) Prec<BF>::split2(x[2 * r], x[2 * r + 1], h[r], l[r]);
  hi = __builtin_bit_cast(typename Prec<BF>::V, make_uint4(h[0], h[1], h[2], h[3]));
  lo = __builtin_bit_cast(typename Prec<BF>::V, make_uint4(l[0], l[1], l[2], l[3]));
}


// Eight consecutive values of one stored column; columns are zero-padded to a
// multiple of 32 rows, so a K-step never reads past its column.
__device__ __forceinline__ void load8c(const float2* __restrict__ col, int l0, float2 (&o)[8]) {
  const float4* p = reinterpret_cast<const float4*>(col + l0);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float4 t = p[r];
    o[2 * r] = make_float2(t.x, t.y);
    o[2 * r + 1] = make_float2(t.z, t.w);
  }
}

__device__ __forceinline__ void load8r(const float* __restrict__ col, int l0, float (&o)[8]) {
  const float4* p = reinterpret_cast<const float4*>(col + l0);
  const float4 t0 = p[0], t1 = p[1];
  o[0] = t0.x; o[1] = t0.y; o[2] = t0.z; o[3] = t0.w;
  o[4] = t1.x; o[5] = t1.y; o[6] = t1.z; o[7] = t1.w;
}

// Value of the lane 8 positions away within each row of 16 lanes.
__device__ __forceinline__ float lane_xor8(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xf, 0xf, false));
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

// log(1 + u) for u >= 0 with relative accuracy near FP32 epsilon (the
// rounding of 1 + u is compensated by u / ((1 + u) - 1)).
__device__ __forceinline__ float log1p_acc(float u) {
  const float w = 1.0f + u;
  const float d = w - 1.0f;
  return d == 0.0f ? u : __logf(w) * (u / d);
}


}  // namespace split
}  // namespace bioem
