// Operand preparation for the split-precision contractions: the kernel
// table is split once at bind time (bounded by sqrt((2l+1)/4pi), so it needs
// no scaling), into the expansion operand [n/16][b][plane][n%16] and the
// transposed moment operand [b/16][n][plane][b%16]; the expansion
// coefficients are split per solve with one power-of-two scale per shell
// (the packed source is split by the packing kernel).
#include <algorithm>

#include "device_util.h"
#include "split_util.h"
#include "coef_impl.h"

namespace mpole {
namespace {

// The split operands over pairs: expansion rows = pairs, k = expansion mode
// column; moment rows = moment mode column, k = pairs (pair_kernel gives the
// pair's kernel of a natural mode, 0 for padding).
template <int KIND>
__global__ __launch_bounds__(256) void k_split_tables(PlanDev P, ClassDev C) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long ne = (long)C.npair_pad * P.namp_e, nm = (long)C.npair_pad * P.namp_m;
  if (t < ne) {
    const int q = (int)(t / P.namp_e), col = (int)(t % P.namp_e);
    const int n = P.perm_e ? P.perm_e[col] : col;
    split_store<KIND>(pair_kernel(P, C, q, n), C.tplanes + slab_index<KIND>(q, col, C.npair_pad), 16);
  }
  if (t < nm) {
    const int q = (int)(t / P.namp_m), col = (int)(t % P.namp_m);
    const int n = P.perm_m ? P.perm_m[col] : col;
    split_store<KIND>(pair_kernel(P, C, q, n), C.ttplanes + slab_index<KIND>(col, q, P.namp_m), 16);
  }
}

template <int KIND>
__global__ __launch_bounds__(256) void k_split_coef(BatchDev B) {
  __shared__ double red[256 / 64];
  split_coef_item<KIND>(job_of(B, PH_COEF, blockIdx.x), red);
}

__global__ __launch_bounds__(256) void k_perm_coef(BatchDev B) { perm_coef_item(job_of(B, PH_COEF, blockIdx.x)); }

}  // namespace

hipError_t launch_split_tables(const PlanDev &P, const ClassDev *host_classes, int kind, hipStream_t s) {
  for (int c = 0; c < P.nclasses; ++c) {
    const ClassDev &C = host_classes[c];
    const long n = (long)C.npair_pad * std::max(P.namp_m, P.namp_e);
    const dim3 g((unsigned)((n + 255) / 256));
    if (kind == kSplitBf16x3)
      hipLaunchKernelGGL(k_split_tables<kSplitBf16x3>, g, dim3(256), 0, s, P, C);
    else
      hipLaunchKernelGGL(k_split_tables<kSplitFp16x2>, g, dim3(256), 0, s, P, C);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_split_coef(const BatchDev &B, int precision, int wgs, hipStream_t s) {
  if (wgs <= 0) return hipSuccess;
  if (precision == 0)
    hipLaunchKernelGGL(k_perm_coef, dim3(wgs), dim3(256), 0, s, B);
  else if (precision == kSplitBf16x3)
    hipLaunchKernelGGL(k_split_coef<kSplitBf16x3>, dim3(wgs), dim3(256), 0, s, B);
  else
    hipLaunchKernelGGL(k_split_coef<kSplitFp16x2>, dim3(wgs), dim3(256), 0, s, B);
  return hipGetLastError();
}

}  // namespace mpole
