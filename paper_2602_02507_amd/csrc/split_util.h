// Narrow-float splitting of FP64 operands (device helpers).
//
// A FP64 value x is written as a sum of narrow floats:
//   BF16 x3:  x ~ hi + mid + lo, each a bfloat16 (8 significant bits), the
//             remainders taken exactly in FP64, so |x - (hi+mid+lo)| <~ 2^-25 |x|;
//   FP16 x2:  x ~ hi + lo, each a binary16 (11 significant bits),
//             |x - (hi+lo)| <~ 2^-23 |x| while lo stays in the binary16 range
//             (rows are scaled by a power of two into [-1, 1) first).
//
// Layout of every split operand: k-slab major, planes interleaved,
//   [k / 16][row][plane][k % 16],
// so that the 16-wide K step of 128 consecutive rows is one contiguous run of
// 128 x planes x 32 bytes -- each contraction stage is a fully coalesced copy
// from global memory to LDS.
#pragma once
#include <cmath>

#include "mpole_internal.h"

namespace mpole {

__device__ inline uint16_t to_bf16(float f) {
  // round to nearest even on the upper 16 bits (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline double from_bf16(uint16_t h) { return (double)__uint_as_float((uint32_t)h << 16); }

__device__ inline uint16_t to_fp16(float f) {
  const _Float16 h = (_Float16)f;
  return *reinterpret_cast<const uint16_t *>(&h);
}
__device__ inline double from_fp16(uint16_t u) { return (double)*reinterpret_cast<const _Float16 *>(&u); }

template <int KIND>
constexpr int split_planes() {
  return KIND == kSplitBf16x3 ? 3 : 2;
}

// element (row, k) of a split operand with `rows` rows; plane p adds 16 p
template <int KIND>
__device__ inline size_t slab_index(int row, int k, int rows) {
  return ((size_t)(k >> 4) * rows + row) * (split_planes<KIND>() * 16) + (k & 15);
}

// element (row, k) of a row-major split operand (the packed source of the
// moment contraction): [row][k/16][plane][k%16], npad = padded row length;
// one shell's row is a contiguous run, and so is each 16-wide K step of it
template <int KIND>
__device__ inline size_t row_index(int row, int k, int npad) {
  return (size_t)row * npad * split_planes<KIND>() + (size_t)(k >> 4) * (split_planes<KIND>() * 16) + (k & 15);
}

// planes of x; stride = distance between planes in elements
template <int KIND>
__device__ inline void split_store(double x, uint16_t *dst, size_t stride) {
  if (KIND == kSplitBf16x3) {
    const uint16_t h = to_bf16((float)x);
    const double r1 = x - from_bf16(h);
    const uint16_t m = to_bf16((float)r1);
    const double r2 = r1 - from_bf16(m);
    dst[0] = h;
    dst[stride] = m;
    dst[2 * stride] = to_bf16((float)r2);
  } else {
    const uint16_t h = to_fp16((float)x);
    dst[0] = h;
    dst[stride] = to_fp16((float)(x - from_fp16(h)));
  }
}

// power of two 2^e with max_abs 2^-e in [0.5, 1); 1 for an all-zero row
__device__ inline double row_scale(double max_abs) {
  if (!(max_abs > 0.0)) return 1.0;
  int e;
  frexp(max_abs, &e);
  return ldexp(1.0, e);
}

}  // namespace mpole
