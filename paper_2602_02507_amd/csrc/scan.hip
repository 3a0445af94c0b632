// Radial part of the solve: the per-phase kernels over all fields of a batch
// (device code in scan_impl.h, shared with the persistent batched launch).
#include "scan_impl.h"

namespace mpole {
namespace {

__global__ __launch_bounds__(256) void k_reduce(BatchDev B) { reduce_item(job_of(B, PH_REDUCE, blockIdx.x)); }

template <int SCAN_MODES>
__global__ __launch_bounds__(SCAN_MODES * SCAN_CHUNKS) void k_scan(BatchDev B) {
  __shared__ double lds[scan_lds<SCAN_MODES>()];
  scan_item<SCAN_MODES>(job_of(B, PH_SCAN, blockIdx.x), lds);
}

}  // namespace

hipError_t launch_reduce(const BatchDev &B, int wgs, hipStream_t s) {
  if (wgs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(wgs), dim3(256), 0, s, B);
  return hipGetLastError();
}

hipError_t launch_scan(const BatchDev &B, int wgs, int modes, hipStream_t s) {
  if (wgs <= 0) return hipSuccess;
  if (modes == kScanModesWide)
    hipLaunchKernelGGL(k_scan<kScanModesWide>, dim3(wgs), dim3(kScanModesWide * SCAN_CHUNKS), 0, s, B);
  else
    hipLaunchKernelGGL(k_scan<kScanModesNarrow>, dim3(wgs), dim3(kScanModesNarrow * SCAN_CHUNKS), 0, s, B);
  return hipGetLastError();
}

}  // namespace mpole
