// Device helpers shared by the kernels of the library.
#pragma once
#include "mpole_internal.h"

namespace mpole {

// Linear workgroup id -> logical tile id such that XCD x (which receives the
// hardware ids w = x mod 8 of a launch) owns the contiguous logical ids
// [x*q + min(x, r), ...): tiles that share operand panels then share an L2.
__device__ inline int xcd_remap(int w, int g) {
  const int q = g >> 3, r = g & 7, x = w & 7;
  return x * q + min(x, r) + (w >> 3);
}

// Field of workgroup wg in a launch of phase h (binary search of the prefix
// sums; the searched values are uniform across the workgroup).
__device__ inline int field_of(const BatchDev &B, int h, int wg) {
  const int32_t *pre = B.prefix + h * (B.nf + 1);
  int lo = 0, hi = B.nf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= wg) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline SolveIO io_of(const BatchDev &B, int f) { return B.io ? B.io[f] : B.io1; }

// A solve-time workgroup's field, its plan and its workgroup id within the field.
struct Job {
  PlanDev P;
  SolveIO io;
  int f, local;
};
__device__ inline Job job_of(const BatchDev &B, int h, int wg) {
  Job j;
  j.f = field_of(B, h, wg);
  j.P = B.plans[j.f];
  j.io = io_of(B, j.f);
  j.local = wg - B.prefix[h * (B.nf + 1) + j.f];
  return j;
}

// Completion stamp of a field (wall clock, constant rate), after the whole
// workgroup has issued its stores.
__device__ inline void stamp_done(const BatchDev &B, int f) {
  if (B.stamps == nullptr) return;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(&B.stamps[f], (unsigned long long)wall_clock64());
}

// dOmega_b S_b of block b of one shell: the sum over the block's member
// cells, in ascending cell order, of 4 pi G dOmega_q rho_q.
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

// Workgroup sum in a fixed order (butterfly within each wavefront, then the
// wavefront totals in order); red holds blockDim.x/64 doubles.
__device__ inline double block_sum(double v, double *red) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < nw; ++q) s += red[q];
  __syncthreads();
  return s;
}

__device__ inline double block_max(double v, double *red) {
  v = fabs(v);
  for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double m = 0.0;
  for (int q = 0; q < nw; ++q) m = fmax(m, red[q]);
  __syncthreads();
  return m;
}

}  // namespace mpole
