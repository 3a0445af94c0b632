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

constexpr int PACK_THREADS = 256, PACK_UNROLL = 4;

// dOmega S of block b of shell i: members in ascending cell order
__device__ inline double block_source(const ClassDev &C, const double *__restrict__ w,
                                      const double *__restrict__ src, int nphi, int b) {
  double s = 0.0;
  if (C.rect != nullptr) {
    const int4 r = C.rect[b];
    for (int j = r.x; j < r.x + r.z; ++j) {
      const int q0 = j * nphi;
      for (int k = r.y; k < r.y + r.w; ++k) s += w[q0 + k] * src[q0 + k];
    }
  } else {
    for (int e = C.moff[b]; e < C.moff[b + 1]; ++e) {
      const int q = C.mem[e];
      s += w[q] * src[q];
    }
  }
  return s;
}

// Each thread packs PACK_UNROLL blocks PACK_THREADS apart.  Single-cell
// blocks (the common case) take a branch-free path whose loads are all
// issued before any is consumed, so enough bytes are in flight to stream rho.
__global__ __launch_bounds__(PACK_THREADS) void k_pack_f64(PlanDev P, const double *__restrict__ rho) {
  const int i = blockIdx.y;
  const ClassDev C = P.classes[P.shell_class[i]];
  const int b0 = blockIdx.x * (PACK_THREADS * PACK_UNROLL) + threadIdx.x;
  if (b0 >= C.nblocks) return;
  const int row = P.shell_row[i];
  const double *__restrict__ src = rho + (size_t)i * P.ncell;
  const double *__restrict__ w = P.weight;
  double *__restrict__ dst = C.pack + (size_t)row * C.nblocks_pad;
  if (C.rect != nullptr) {
    int4 r[PACK_UNROLL];
    double s[PACK_UNROLL];
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int b = b0 + u * PACK_THREADS;
      r[u] = (b < C.nblocks) ? C.rect[b] : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int q = r[u].x * P.nphi + r[u].y;
      s[u] = (r[u].z == 1 && r[u].w == 1) ? w[q] * src[q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int b = b0 + u * PACK_THREADS;
      if (b >= C.nblocks) continue;
      if (r[u].z != 1 || r[u].w != 1) s[u] = block_source(C, w, src, P.nphi, b);
      dst[b] = s[u];
    }
  } else {
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int b = b0 + u * PACK_THREADS;
      if (b < C.nblocks) dst[b] = block_source(C, w, src, P.nphi, b);
    }
  }
}

}  // namespace

hipError_t launch_pack_f64(const PlanDev &P, const ClassDev *host_classes, const double *rho, hipStream_t s) {
  int maxb = 0;
  for (int c = 0; c < P.nclasses; ++c) maxb = std::max(maxb, host_classes[c].nblocks);
  const int per = PACK_THREADS * PACK_UNROLL;
  hipLaunchKernelGGL(k_pack_f64, dim3((maxb + per - 1) / per, P.nr), dim3(PACK_THREADS), 0, s, P, rho);
  return hipGetLastError();
}

}  // namespace mpole
