// Operand preparation for the split-precision contractions.
//
// A FP64 value x (after an exact power-of-two row scaling into [-1, 1)) is
// written as a sum of narrow floats:
//   BF16 x3:  x ~ hi + mid + lo, each a bfloat16 (8 significant bits), the
//             remainders taken exactly in FP64, so |x - (hi+mid+lo)| <~ 2^-25 |x|;
//   FP16 x2:  x ~ hi + lo, each a binary16 (11 significant bits),
//             |x - (hi+lo)| <~ 2^-23 |x| while lo stays in the binary16 range.
// The kernel table is split once at bind time (bounded by sqrt((2l+1)/4pi),
// so it needs no scaling); the packed source and the expansion coefficients
// are split per solve with one power-of-two scale per radial shell.
//
// Layout of every split operand: k-slab major, planes interleaved,
//   [k / 16][row][plane][k % 16],
// so that the 16-wide K step of 128 consecutive rows is one contiguous run
// of 128 x planes x 32 bytes -- each contraction stage is a fully coalesced
// copy from global memory to LDS.
#include <cmath>

#include "mpole_internal.h"

namespace mpole {
namespace {

__device__ inline uint16_t to_bf16(float f) {
  // round to nearest even on the upper 16 bits (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline double from_bf16(uint16_t h) { return (double)__uint_as_float((uint32_t)h << 16); }

__device__ inline uint16_t to_fp16(float f) {
  const _Float16 h = (_Float16)f;
  return *reinterpret_cast<const uint16_t *>(&h);
}
__device__ inline double from_fp16(uint16_t u) { return (double)*reinterpret_cast<const _Float16 *>(&u); }

// element (row, k) of a split operand with `rows` rows; plane p adds 16 * p
template <int KIND>
__device__ inline size_t slab_index(int row, int k, int rows) {
  constexpr int NP = KIND == kSplitBf16x3 ? 3 : 2;
  return ((size_t)(k >> 4) * rows + row) * (NP * 16) + (k & 15);
}

// planes of x; stride = distance between planes in elements
template <int KIND>
__device__ inline void split_store(double x, uint16_t *dst, size_t stride) {
  if (KIND == kSplitBf16x3) {
    const uint16_t h = to_bf16((float)x);
    const double r1 = x - from_bf16(h);
    const uint16_t m = to_bf16((float)r1);
    const double r2 = r1 - from_bf16(m);
    dst[0] = h;
    dst[stride] = m;
    dst[2 * stride] = to_bf16((float)r2);
  } else {
    const uint16_t h = to_fp16((float)x);
    dst[0] = h;
    dst[stride] = to_fp16((float)(x - from_fp16(h)));
  }
}

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

// power of two 2^e with max_abs * 2^-e in [0.5, 1); 1 for an all-zero row
__device__ inline double row_scale(double max_abs) {
  if (!(max_abs > 0.0)) return 1.0;
  int e;
  frexp(max_abs, &e);
  return ldexp(1.0, e);
}

constexpr int ROW_THREADS = 1024;   // one workgroup per shell row

__device__ inline double block_sum(double v, double *red) {
  // workgroup sum, fixed order (butterfly in each wavefront, then wavefronts in order)
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

// dOmega S of block b: members in ascending cell order (same sums as the FP64 pack)
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

// One workgroup per shell: packed source in FP64 (kept in C.pack), its
// max-abs power-of-two scale, the split planes of the scaled row, and the
// monopole moment sum_b P_b T_b0 in FP64 (fixed tree order).
template <int KIND>
__global__ __launch_bounds__(ROW_THREADS) void k_pack_split(PlanDev P, const double *__restrict__ rho) {
  __shared__ double red[ROW_THREADS / 64];
  const int i = blockIdx.x;
  const ClassDev C = P.classes[P.shell_class[i]];
  const int row = P.shell_row[i];
  const double *__restrict__ src = rho + (size_t)i * P.ncell;
  double *__restrict__ prow = C.pack + (size_t)row * C.nblocks_pad;
  double mx = 0.0, mono = 0.0;
  for (int b = threadIdx.x; b < C.nblocks; b += ROW_THREADS) {
    const double s = block_source(C, P.weight, src, P.nphi, b);
    prow[b] = s;
    mx = fmax(mx, fabs(s));
    mono += s * C.table[(size_t)b * P.namp];
  }
  mono = block_sum(mono, red);
  const double scale = row_scale(block_max(mx, red));
  const double inv = 1.0 / scale;   // exact: a power of two
  for (int b = threadIdx.x; b < C.nblocks; b += ROW_THREADS)
    split_store<KIND>(prow[b] * inv, C.ppacks + slab_index<KIND>(row, b, C.nrows), 16);
  if (threadIdx.x == 0) {
    C.pscale[row] = scale;
    P.mono[i] = mono;
  }
}

// One workgroup per shell: scale and split the expansion coefficients.
template <int KIND>
__global__ __launch_bounds__(256) void k_split_coef(PlanDev P) {
  __shared__ double red[256 / 64];
  const int i = blockIdx.x;
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

hipError_t launch_pack_split(const PlanDev &P, const double *rho, int kind, hipStream_t s) {
  if (kind == kSplitBf16x3)
    hipLaunchKernelGGL(k_pack_split<kSplitBf16x3>, dim3(P.nr), dim3(ROW_THREADS), 0, s, P, rho);
  else
    hipLaunchKernelGGL(k_pack_split<kSplitFp16x2>, dim3(P.nr), dim3(ROW_THREADS), 0, s, P, rho);
  return hipGetLastError();
}

hipError_t launch_split_coef(const PlanDev &P, int kind, hipStream_t s) {
  if (kind == kSplitBf16x3)
    hipLaunchKernelGGL(k_split_coef<kSplitBf16x3>, dim3(P.nr), dim3(256), 0, s, P);
  else
    hipLaunchKernelGGL(k_split_coef<kSplitFp16x2>, dim3(P.nr), dim3(256), 0, s, P);
  return hipGetLastError();
}

}  // namespace mpole
