// Coarsening operation of Sec. 2.3: every cell of a coarsening block takes
// the volume-weighted block mean sum_j V_j K_j / sum_j V_j over the block's
// member cells j.  Within one shell V_j is the shell's (r^3 difference)/3
// times the solid angle of the angular cell, so the weights reduce to the
// solid angles dOmega_j = (cos th_j - cos th_j+1) dphi_k.
//
// Grid: x = spans of kPackSpan blocks (up to the largest class), y = shells.
// A span of single-cell blocks at consecutive cells (the plan's span0 >= 0;
// most of a shell away from the origin and the axis) is a coalesced copy;
// otherwise each thread gathers, averages and scatters whole blocks, so a
// thread reads all members of its block before writing any and in-place
// calls (in == out) are safe; blocks of more than kLargeBlock cells get a
// workgroup each (launch_large).  HBM-bound: 8 B read and 8 B written per cell.
#include <algorithm>

#include "device_util.h"

namespace mpole {
namespace {

constexpr int CO_THREADS = 256, CO_UNROLL = kPackSpan / CO_THREADS;

__global__ __launch_bounds__(CO_THREADS) void k_coarsen(PlanDev P, const double *in_, double *out_) {
  const int i = blockIdx.y, sp = blockIdx.x;
  const ClassDev C = ld_const(P.classes + ld_const(P.shell_class + i));
  if (C.bands != nullptr) return;            // banded classes: launch_bands
  if (sp * kPackSpan >= C.nblocks) return;   // span past this class's blocks
  const auto in = gmem(in_ + (size_t)i * P.ncell);
  const auto out = gmem(out_ + (size_t)i * P.ncell);
  const int run0 = ld_const(C.span0 + sp);
  const int b0 = sp * kPackSpan + threadIdx.x;
  if (run0 >= 0) {
    double v[CO_UNROLL];
#pragma unroll
    for (int u = 0; u < CO_UNROLL; ++u) {
      const int b = b0 + u * CO_THREADS;
      v[u] = b < C.nblocks ? in[run0 + b - sp * kPackSpan] : 0.0;
    }
    if (in_ == out_) return;
#pragma unroll
    for (int u = 0; u < CO_UNROLL; ++u) {
      const int b = b0 + u * CO_THREADS;
      if (b < C.nblocks) out[run0 + b - sp * kPackSpan] = v[u];
    }
    return;
  }
  const auto moff = gmem(C.moff), mem = gmem(C.mem);
  for (int u = 0; u < CO_UNROLL; ++u) {
    const int b = b0 + u * CO_THREADS;
    if (b >= C.nblocks) break;
    const int e0 = moff[b], e1 = moff[b + 1];
    if (e1 - e0 == 1) {   // a block of one cell keeps its value
      const int q = mem[e0];
      out[q] = in[q];
      continue;
    }
    if (e1 - e0 > kLargeBlock) continue;   // one workgroup each, in launch_large
    double num = 0.0, den = 0.0;
    block_wsum(C, P.dom, in_ + (size_t)i * P.ncell, P.nphi, b, num, den);
    block_fill(C, out_ + (size_t)i * P.ncell, P.nphi, b, num / den);
  }
}

}  // namespace

hipError_t launch_coarsen(const PlanDev &P, const ClassDev *host_classes, const double *in, double *out,
                          hipStream_t s) {
  int nb = 0;
  for (int c = 0; c < P.nclasses; ++c) nb = std::max(nb, host_classes[c].nblocks);
  const unsigned spans = (unsigned)((nb + kPackSpan - 1) / kPackSpan);
  if (spans == 0 || P.nr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarsen, dim3(spans, (unsigned)P.nr), dim3(CO_THREADS), 0, s, P, in, out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_bands(P, kBandCoarsen, in, out, s);
  if (e == hipSuccess) e = launch_large(P, kLargeMean, in, out, s);
  return e;
}

}  // namespace mpole
