// The two angular contractions in FP64 on MFMA: the per-phase kernels over
// all fields of a batch (device code in gemm_f64_impl.h, shared with the
// persistent batched launch).
#include "gemm_f64_impl.h"

namespace mpole {
namespace {

__global__ __launch_bounds__(NTHREADS) void k_moment_f64(BatchDev B) {
  __shared__ double lds[F64_LDS];
  moment_f64_item(B, job_of(B, PH_MOMENT, xcd_remap(blockIdx.x, gridDim.x)), lds);
}

__global__ __launch_bounds__(NTHREADS) void k_expand_f64(BatchDev B) {
  __shared__ double lds[F64_LDS];
  expand_f64_item(B, job_of(B, PH_EXPAND, xcd_remap(blockIdx.x, gridDim.x)), lds);
}

}  // namespace

hipError_t launch_moment_f64(const BatchDev &B, int wgs, hipStream_t s) {
  if (wgs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_moment_f64, dim3(wgs), dim3(NTHREADS), 0, s, B);
  return hipGetLastError();
}

hipError_t launch_expand_f64(const BatchDev &B, int wgs, hipStream_t s) {
  if (wgs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand_f64, dim3(wgs), dim3(NTHREADS), 0, s, B);
  return hipGetLastError();
}

}  // namespace mpole
