// Device helpers shared by the kernels of the library.
#pragma once
#include "mpole_internal.h"

namespace mpole {

// int pair as a plain vector type (loads through global address-space pointers)
typedef int i2v __attribute__((ext_vector_type(2)));

// Thread index within the workgroup, as the per-phase device code (the work
// items) reads it.  A translation unit that runs items in a loop (the
// persistent batched kernel) defines MPOLE_ITEM_LOOP: the index then passes
// through an empty asm statement on every read, so that the index arithmetic
// of an item cannot be hoisted out of the loop, where it would stay live in
// vector registers across every item.
#ifdef MPOLE_ITEM_LOOP
static __device__ __forceinline__ int item_tid() {
  int t = (int)threadIdx.x;
  __asm__ volatile("" : "+v"(t));
  __builtin_assume(t >= 0 && t < 1024);
  return t;
}
#else
static __device__ __forceinline__ int item_tid() { return (int)threadIdx.x; }
#endif

// Linear workgroup id -> logical tile id such that XCD x (which receives the
// hardware ids w = x mod 8 of a launch) owns the contiguous logical ids
// [x*q + min(x, r), ...): tiles that share operand panels then share an L2.
__device__ inline int xcd_remap(int w, int g) {
  const int q = g >> 3, r = g & 7, x = w & 7;
  return x * q + min(x, r) + (w >> 3);
}

// Plan descriptors (plans, classes, prefix sums, shell maps) are written
// before a solve and only read by its kernels.  Reading them through the
// constant address space lets workgroup-uniform loads go to scalar
// registers instead of occupying vector registers for the whole kernel.
template <class T>
__device__ inline T ld_const(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "descriptor size");
  typedef const __attribute__((address_space(4))) uint32_t cword;
  const cword *q = (const cword *)p;
  T v;
  uint32_t *d = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = q[i];
  return v;
}

// Device buffers reached through a descriptor are plain global memory; saying
// so lets the compiler use global (not flat) loads and stores for them.
template <class T>
__device__ inline __attribute__((address_space(1))) T *gmem(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

// (l, m, a) of natural mode n = l^2 (m = 0), l^2 + 2m - 1 (cos), l^2 + 2m (sin).
__device__ inline void mode_lma(int n, int &l, int &m, int &a) {
  l = (int)sqrt((double)n);
  while ((l + 1) * (l + 1) <= n) ++l;
  while (l * l > n) --l;
  const int d = n - l * l;
  m = (d + 1) >> 1;
  a = (d > 0 && (d & 1) == 0) ? 1 : 0;
}

// Kernel of natural mode n for pair q of a class: the rep block's table
// entry; zero for padding, and for the odd modes of a block that is its own
// mirror image when the plan is folded (their cell averages vanish).
__device__ inline double pair_kernel(const PlanDev &P, const ClassDev &C, int q, int n) {
  if (q >= C.npair || n < 0 || n >= P.nam) return 0.0;
  const int2 pr = C.pairs[q];
  if (P.fold && pr.x == pr.y) {
    int l, m, a;
    mode_lma(n, l, m, a);
    if ((l + m) & 1) return 0.0;
  }
  return C.table[(size_t)pr.x * P.namp + n];
}

// cos t0 - cos t1 as a product, exact for thin theta cells.
__device__ inline double cos_diff(double t0, double t1) {
  return 2.0 * sin(0.5 * (t0 + t1)) * sin(0.5 * (t1 - t0));
}

// Field of workgroup wg in a launch of phase h (binary search of the prefix
// sums; the searched values are uniform across the workgroup).
__device__ inline int field_of(const BatchDev &B, int h, int wg) {
  const int32_t *pre = B.prefix + h * (B.nf + 1);
  int lo = 0, hi = B.nf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ld_const(pre + mid) <= wg) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline SolveIO io_of(const BatchDev &B, int f) { return B.io ? ld_const(B.io + f) : B.io1; }

// A solve-time workgroup's field, its plan and its workgroup id within the field.
struct Job {
  PlanDev P;
  SolveIO io;
  int f, local;
};
__device__ inline Job job_of(const BatchDev &B, int h, int wg) {
  Job j;
  j.f = field_of(B, h, wg);
  j.P = ld_const(B.plans + j.f);
  j.io = io_of(B, j.f);
  j.local = wg - ld_const(B.prefix + h * (B.nf + 1) + j.f);
  return j;
}

// Completion stamp of a field (wall clock, constant rate), after the whole
// workgroup has issued its stores.
__device__ inline void stamp_done(const BatchDev &B, int f) {
  if (B.stamps == nullptr) return;
  __syncthreads();
  if (item_tid() == 0) atomicMax(&B.stamps[f], (unsigned long long)wall_clock64());
}

// dOmega_b S_b of block b of one shell: the sum over the block's member
// cells, in ascending cell order, of 4 pi G dOmega_q rho_q.
__device__ inline double block_source(const ClassDev &C, const double *w_, const double *src_, int nphi, int b) {
  const auto w = gmem(w_), src = gmem(src_);
  double s = 0.0;
  if (C.rect != nullptr) {
    const auto rect = gmem(reinterpret_cast<const int *>(C.rect));
    const int j0 = rect[4 * b], k0 = rect[4 * b + 1], nj = rect[4 * b + 2], nk = rect[4 * b + 3];
    for (int j = j0; j < j0 + nj; ++j) {
      const int q0 = j * nphi;
      for (int k = k0; k < k0 + nk; ++k) s += w[q0 + k] * src[q0 + k];
    }
  } else {
    const auto moff = gmem(C.moff), mem = gmem(C.mem);
    for (int e = moff[b]; e < moff[b + 1]; ++e) {
      const int q = mem[e];
      s += w[q] * src[q];
    }
  }
  return s;
}

// Solid-angle weighted sums over the members of block b of a shell row x:
// num += sum dOmega x, den += sum dOmega.  Rectangular blocks are walked row
// by row with direct indexing, others through the member list.
__device__ inline void block_wsum(const ClassDev &C, const double *dom_, const double *x_, int nphi, int b,
                                  double &num, double &den) {
  const auto dom = gmem(dom_), x = gmem(x_);
  if (C.rect != nullptr) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    const i4 r = gmem(reinterpret_cast<const i4 *>(C.rect))[b];   // (j0, k0, nj, nk)
    for (int j = 0; j < r.z; ++j) {
      const int q0 = (r.x + j) * nphi + r.y;
      for (int k = 0; k < r.w; ++k) {
        const double w = dom[q0 + k];
        num += w * x[q0 + k];
        den += w;
      }
    }
  } else {
    const auto moff = gmem(C.moff), mem = gmem(C.mem);
    for (int e = moff[b]; e < moff[b + 1]; ++e) {
      const int q = mem[e];
      const double w = dom[q];
      num += w * x[q];
      den += w;
    }
  }
}

// Writes v to every member cell of block b of a shell row out.
__device__ inline void block_fill(const ClassDev &C, double *out_, int nphi, int b, double v) {
  const auto out = gmem(out_);
  if (C.rect != nullptr) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    const i4 r = gmem(reinterpret_cast<const i4 *>(C.rect))[b];
    for (int j = 0; j < r.z; ++j)
      for (int k = 0; k < r.w; ++k) out[(r.x + j) * nphi + r.y + k] = v;
  } else {
    const auto moff = gmem(C.moff), mem = gmem(C.mem);
    for (int e = moff[b]; e < moff[b + 1]; ++e) out[mem[e]] = v;
  }
}

// Source sum of a block of more than kLargeBlock cells of shell i, computed
// by launch_large(kLargeSum) before the packing kernel.
__device__ inline double large_source(const PlanDev &P, const ClassDev &C, int i, int b) {
  return gmem(P.lsum)[ld_const(P.lbase + i) + gmem(C.lidx)[b]];
}

// Workgroup sum in a fixed order (butterfly within each wavefront, then the
// wavefront totals in order); red holds blockDim.x/64 doubles.
__device__ inline double block_sum(double v, double *red) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  const int w = item_tid() >> 6, nw = blockDim.x >> 6;
  if ((item_tid() & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < nw; ++q) s += red[q];
  __syncthreads();
  return s;
}

__device__ inline double block_max(double v, double *red) {
  v = fabs(v);
  for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
  const int w = item_tid() >> 6, nw = blockDim.x >> 6;
  if ((item_tid() & 63) == 0) red[w] = v;
  __syncthreads();
  double m = 0.0;
  for (int q = 0; q < nw; ++q) m = fmax(m, red[q]);
  __syncthreads();
  return m;
}

}  // namespace mpole
