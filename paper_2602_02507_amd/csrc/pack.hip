// Density streaming (the front of the solve): each coarsening block of each
// shell gets its share of the source, sum over members of 4 pi G dOmega rho,
// i.e. dOmega_b S_b with S_b the solid-angle weighted block mean (GenASiS II
// Sec. 2.1 coarsening blocks; Eq. AngularMomentsDiscrete weights dOmega S).
// One thread per (shell, block); consecutive threads take consecutive blocks
// whose members are consecutive cells, so reads of rho stay coalesced.
#include <algorithm>

#include "mpole_internal.h"

namespace mpole {
namespace {

__global__ __launch_bounds__(256) void k_pack_f64(PlanDev P, const double *__restrict__ rho) {
  const int i = blockIdx.y;
  const int c = P.shell_class[i];
  const ClassDev C = P.classes[c];
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= C.nblocks) return;
  const int row = P.shell_row[i];
  const double *__restrict__ src = rho + (size_t)i * P.ncell;
  double s = 0.0;
  for (int e = C.moff[b]; e < C.moff[b + 1]; ++e) {
    const int q = C.mem[e];
    s += P.weight[q] * src[q];
  }
  C.pack[(size_t)row * C.nblocks_pad + b] = s;
}

}  // namespace

hipError_t launch_pack_f64(const PlanDev &P, const ClassDev *host_classes, const double *rho, hipStream_t s) {
  int maxb = 0;
  for (int c = 0; c < P.nclasses; ++c) maxb = std::max(maxb, host_classes[c].nblocks);
  hipLaunchKernelGGL(k_pack_f64, dim3((maxb + 255) / 256, P.nr), dim3(256), 0, s, P, rho);
  return hipGetLastError();
}

}  // namespace mpole
