// FP64 MFMA tile pieces shared by the dense and the separable contractions:
// 64 x 64 output tiles of four waves (2 x 2, each 32 x 32 as 2 x 2
// v_mfma_f64_16x16x4 tiles), K staged 16 at a time through LDS in one of two
// layouts.  f64 MFMA 16x16x4 lane layout on gfx950 (checked on the device):
// lane l supplies A[l%16][l/16] and B[l/16][l%16]; result element (i, j) sits
// in lane 16*(i%4) + j, accumulator register i/4.
#pragma once
#include "device_util.h"

namespace mpole {
namespace f64mma {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, NTHREADS = 256;
constexpr int RK = BK + 1;      // pitch of a row-major [row][k] stage, in doubles
constexpr int KR = BM + 4;      // pitch of a k-major [k][row] stage, in doubles
constexpr int STAGE = BM * RK;  // doubles per stage (both layouts)
static_assert(BK * KR == STAGE, "stage sizes");

// Element (row, k) of a stage in either layout.
template <bool ROWMAJOR>
__device__ inline double lds_at(const double *S, int row, int k) {
  return ROWMAJOR ? S[row * RK + k] : S[k * KR + row];
}

template <bool A_ROWMAJOR, bool B_ROWMAJOR>
__device__ inline void mfma_stage(const double *As, const double *Bs, int wm, int wn, int lane, d4 acc[2][2]) {
#pragma unroll
  for (int kk = 0; kk < BK / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
    const int c = lane & 15;
    const double a0 = lds_at<A_ROWMAJOR>(As, wm * 32 + c, kr);
    const double a1 = lds_at<A_ROWMAJOR>(As, wm * 32 + 16 + c, kr);
    const double b0 = lds_at<B_ROWMAJOR>(Bs, wn * 32 + c, kr);
    const double b1 = lds_at<B_ROWMAJOR>(Bs, wn * 32 + 16 + c, kr);
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

}  // namespace f64mma
}  // namespace mpole
