// Density streaming kernels of a batch (device code in pack_impl.h, shared
// with the persistent batched launch) and the completion stamps.
#include "pack_impl.h"

namespace mpole {
namespace {

// 8 waves per SIMD: a packing workgroup is short and mostly waits for its
// loads, so more of them in flight move more bytes (BF16 x3: 59.8 -> 58.6 us,
// FP16 x2 106 -> 100 us on the production mesh, though BF16 x3 spills 12
// bytes per lane at this size)
template <int MODE>
__global__ __launch_bounds__(PACK_THREADS) __attribute__((amdgpu_waves_per_eu(8))) void k_pack(BatchDev B) {
  __shared__ __align__(16) char lds[MODE == kSplitBf16x3 ? PACK_LDS : 256];
  // batch start: the first workgroup of the first launch of the solve
  pack_item<MODE>(B, job_of(B, PH_PACK, blockIdx.x), lds, blockIdx.x == 0);
}

__global__ __launch_bounds__(256) void k_split_rows_fp16(BatchDev B) {
  __shared__ double red[4];
  split_rows_item(B, job_of(B, PH_SPLITROWS, blockIdx.x), red);
}

}  // namespace

__global__ __launch_bounds__(256) void k_stamp_reset(unsigned long long *stamps, int nf) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < nf) stamps[t] = 0ull;
  if (t == nf) stamps[nf] = ~0ull;
}

__global__ void k_stamp(unsigned long long *stamps, int idx) {
  if (threadIdx.x == 0) stamps[idx] = wall_clock64();
}

hipError_t launch_stamp(unsigned long long *stamps, int idx, hipStream_t s) {
  if (stamps == nullptr) return hipSuccess;
  hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, stamps, idx);
  return hipGetLastError();
}

hipError_t launch_stamp_reset(const BatchDev &B, hipStream_t s) {
  if (B.stamps == nullptr) return hipSuccess;
  hipLaunchKernelGGL(k_stamp_reset, dim3((B.nf + 1 + 255) / 256), dim3(256), 0, s, B.stamps, B.nf);
  return hipGetLastError();
}

hipError_t launch_pack(const BatchDev &B, int precision, int wgs, hipStream_t s) {
  if (wgs <= 0) return hipSuccess;
  if (precision == 0)
    hipLaunchKernelGGL(k_pack<0>, dim3(wgs), dim3(PACK_THREADS), 0, s, B);
  else if (precision == kSplitBf16x3)
    hipLaunchKernelGGL(k_pack<kSplitBf16x3>, dim3(wgs), dim3(PACK_THREADS), 0, s, B);
  else
    hipLaunchKernelGGL(k_pack<kSplitFp16x2>, dim3(wgs), dim3(PACK_THREADS), 0, s, B);
  return hipGetLastError();
}

hipError_t launch_split_rows(const BatchDev &B, int wgs, hipStream_t s) {
  if (wgs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_rows_fp16, dim3(wgs), dim3(256), 0, s, B);
  return hipGetLastError();
}

}  // namespace mpole
