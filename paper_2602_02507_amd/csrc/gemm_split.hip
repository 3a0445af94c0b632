// The two angular contractions with split narrow-float operands on MFMA:
// the per-phase kernels over all fields of a batch (the device code is in
// gemm_split_impl.h, shared with the persistent batched launch).
#include "gemm_split_impl.h"

namespace mpole {
namespace {

template <int KIND, bool EXPAND>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(EXPAND ? 2 : 3))) void k_gemm_split(BatchDev B) {
  __shared__ u4 lds[split_lds_slots<KIND>()];
  const Job J = job_of(B, EXPAND ? PH_EXPAND : PH_MOMENT, xcd_remap(blockIdx.x, gridDim.x));
  split_item<KIND, EXPAND>(B, J, lds);
}

}  // namespace

hipError_t launch_moment_split(const BatchDev &B, int wgs, int kind, hipStream_t s) {
  if (wgs <= 0) return hipSuccess;
  if (kind == kSplitBf16x3)
    hipLaunchKernelGGL((k_gemm_split<kSplitBf16x3, false>), dim3(wgs), dim3(NTH), 0, s, B);
  else
    hipLaunchKernelGGL((k_gemm_split<kSplitFp16x2, false>), dim3(wgs), dim3(NTH), 0, s, B);
  return hipGetLastError();
}

hipError_t launch_expand_split(const BatchDev &B, int wgs, int kind, hipStream_t s) {
  if (wgs <= 0) return hipSuccess;
  if (kind == kSplitBf16x3)
    hipLaunchKernelGGL((k_gemm_split<kSplitBf16x3, true>), dim3(wgs), dim3(NTH), 0, s, B);
  else
    hipLaunchKernelGGL((k_gemm_split<kSplitFp16x2, true>), dim3(wgs), dim3(NTH), 0, s, B);
  return hipGetLastError();
}

hipError_t launch_moment(const BatchDev &B, int precision, int wgs, hipStream_t s) {
  return precision == 0 ? launch_moment_f64(B, wgs, s) : launch_moment_split(B, wgs, precision, s);
}

hipError_t launch_expand(const BatchDev &B, int precision, int wgs, hipStream_t s) {
  return precision == 0 ? launch_expand_f64(B, wgs, s) : launch_expand_split(B, wgs, precision, s);
}

}  // namespace mpole
