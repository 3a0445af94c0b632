// Operand preparation for the split-precision contractions: the kernel
// table is split once at bind time (bounded by sqrt((2l+1)/4pi), so it needs
// no scaling), into the expansion operand [n/16][b][plane][n%16] and the
// transposed moment operand [b/16][n][plane][b%16]; the expansion
// coefficients are split per solve with one power-of-two scale per shell
// (the packed source is split by the packing kernel).
#include "device_util.h"
#include "split_util.h"

namespace mpole {
namespace {

template <int KIND>
__global__ __launch_bounds__(256) void k_split_tables(ClassDev C, int namp) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n_el = (long)C.nblocks_pad * namp;
  if (t >= n_el) return;
  const int b = (int)(t / namp), n = (int)(t % namp);
  const double x = C.table[t];
  split_store<KIND>(x, C.tplanes + slab_index<KIND>(b, n, C.nblocks_pad), 16);   // expansion: rows b, k = n
  split_store<KIND>(x, C.ttplanes + slab_index<KIND>(n, b, namp), 16);           // moment: rows n, k = b
}

// One workgroup per shell: scale and split the expansion coefficients.
template <int KIND>
__global__ __launch_bounds__(256) void k_split_coef(BatchDev B) {
  __shared__ double red[256 / 64];
  const Job J = job_of(B, PH_COEF, blockIdx.x);
  const PlanDev &P = J.P;
  const int i = J.local;
  const double *__restrict__ c = P.coef + (size_t)i * P.namp;
  double mx = 0.0;
  for (int n = threadIdx.x + 1; n < P.nam; n += 256) mx = fmax(mx, fabs(c[n]));
  const double scale = row_scale(block_max(mx, red));
  const double inv = 1.0 / scale;
  // the l = 0 term is added in FP64 by the expansion epilogue
  for (int n = threadIdx.x; n < P.namp; n += 256)
    split_store<KIND>((n > 0 && n < P.nam) ? c[n] * inv : 0.0, P.cplanes + slab_index<KIND>(i, n, P.nr), 16);
  if (threadIdx.x == 0) P.cscale[i] = scale;
}

}  // namespace

hipError_t launch_split_tables(const PlanDev &P, const ClassDev *host_classes, int kind, hipStream_t s) {
  for (int c = 0; c < P.nclasses; ++c) {
    const ClassDev &C = host_classes[c];
    const long n = (long)C.nblocks_pad * P.namp;
    const dim3 g((unsigned)((n + 255) / 256));
    if (kind == kSplitBf16x3)
      hipLaunchKernelGGL(k_split_tables<kSplitBf16x3>, g, dim3(256), 0, s, C, P.namp);
    else
      hipLaunchKernelGGL(k_split_tables<kSplitFp16x2>, g, dim3(256), 0, s, C, P.namp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_split_coef(const BatchDev &B, int precision, int wgs, hipStream_t s) {
  if (wgs <= 0 || precision == 0) return hipSuccess;
  if (precision == kSplitBf16x3)
    hipLaunchKernelGGL(k_split_coef<kSplitBf16x3>, dim3(wgs), dim3(256), 0, s, B);
  else
    hipLaunchKernelGGL(k_split_coef<kSplitFp16x2>, dim3(wgs), dim3(256), 0, s, B);
  return hipGetLastError();
}

}  // namespace mpole
