// Coarsening blocks with many member cells (more than kLargeBlock): near the
// origin a block can hold a large part of a shell (Sec. 2.1 groups cells
// until the block is as wide as the core's radial cell), too much work for
// the one thread per block that the packing, averaging and potential
// streaming kernels give to ordinary blocks.  Each large block of each shell
// is cut into chunks of at most kLargeChunk members, one workgroup each:
// members are read with a block-wide stride and combined by a fixed-order
// workgroup sum into a per-chunk partial; a second launch adds a block's
// partials in chunk order (the same result on every chunk) and writes the
// mean with the same stride.  The two launches order every read of a mean
// before its writes, so in-place means are safe.
//
// Block maps made of theta bands (every block of rows [j0, j0 + nj) an
// nj x nk rectangle at a phi column divisible by nk, the layout of
// power-of-two coarsening) take the band kernel for block means instead of
// one thread per block: coalesced column sums and lane butterflies.
#include "bcast_impl.h"
#include "device_util.h"

namespace mpole {
namespace {

constexpr int LB_THREADS = 256;

struct Chunk {
  int i, b, e0, e1;   // shell, block, member range
};

__device__ inline Chunk chunk_of(const PlanDev &P, const ClassDev &C, int4 ch) {
  const int2 it = ld_const(P.litems + ch.x);
  const int m0 = gmem(C.moff)[it.y], m1 = gmem(C.moff)[it.y + 1];
  const int e0 = m0 + ch.y * kLargeChunk;
  return Chunk{it.x, it.y, e0, min(m1, e0 + kLargeChunk)};
}

// partial (sum w x, sum w) of each chunk; w = dOmega (means) or 4 pi G dOmega (sums)
template <bool SUM>
__global__ __launch_bounds__(LB_THREADS) void k_large_part(PlanDev P, const double *in_) {
  __shared__ double red[LB_THREADS / 64];
  const int4 ch = ld_const(P.lchunks + blockIdx.x);
  const int i = ld_const(P.litems + ch.x).x;
  const ClassDev C = ld_const(P.classes + ld_const(P.shell_class + i));
  const Chunk k = chunk_of(P, C, ch);
  const auto mem = gmem(C.mem);
  const auto in = gmem(in_ + (size_t)k.i * P.ncell);
  const auto wt = gmem(SUM ? P.weight : P.dom);
  double num = 0.0, den = 0.0;
  for (int e = k.e0 + threadIdx.x; e < k.e1; e += LB_THREADS) {
    const int q = mem[e];
    const double w = wt[q];
    num += w * in[q];
    den += w;
  }
  num = block_sum(num, red);
  den = block_sum(den, red);
  if (threadIdx.x == 0) {
    gmem(P.lpart)[2 * blockIdx.x] = num;
    gmem(P.lpart)[2 * blockIdx.x + 1] = den;
  }
}

// MODE kLargeMean: the block mean on this chunk's members; kLargeSum: the
// block's weighted sum into lsum (first chunk only); kLargeBcast: the value
// at the block's first member on this chunk's other members.
template <int MODE>
__global__ __launch_bounds__(LB_THREADS) void k_large_fill(PlanDev P, double *out_) {
  const int4 ch = ld_const(P.lchunks + blockIdx.x);
  if (MODE == kLargeSum) {
    if (ch.y != 0 || threadIdx.x != 0) return;
    const auto part = gmem(P.lpart);
    double num = 0.0;
    for (int c = ch.w; c < ch.w + ch.z; ++c) num += part[2 * c];
    gmem(P.lsum)[ch.x] = num;
    return;
  }
  const int i = ld_const(P.litems + ch.x).x;
  const ClassDev C = ld_const(P.classes + ld_const(P.shell_class + i));
  const Chunk k = chunk_of(P, C, ch);
  const auto mem = gmem(C.mem);
  const auto out = gmem(out_ + (size_t)k.i * P.ncell);
  double v;
  int e0 = k.e0;
  if (MODE == kLargeBcast) {
    const int first = gmem(C.moff)[k.b];
    v = out[mem[first]];
    if (e0 == first) ++e0;
  } else {
    const auto part = gmem(P.lpart);
    double num = 0.0, den = 0.0;
    for (int c = ch.w; c < ch.w + ch.z; ++c) {
      num += part[2 * c];
      den += part[2 * c + 1];
    }
    v = num / den;
  }
  for (int e = e0 + threadIdx.x; e < k.e1; e += LB_THREADS) out[mem[e]] = v;
}

// One workgroup per theta band of shell blockIdx.y: each thread takes phi
// columns k = threadIdx.x + 256 u, sums dOmega x and dOmega down the band's
// rows, and the nk lanes of a block (aligned, nk a power of two <= 64, so
// inside one wavefront) add their column sums by xor butterflies: every lane
// of a block ends with the same sums (each step adds the same two partials),
// and writes the mean down its column.  Coalesced, no member lists; a thread
// reads its columns before writing them, so in == out is safe.
template <bool COPY>
__global__ __launch_bounds__(LB_THREADS) void k_band(PlanDev P, const double *in_, double *out_, int skip_nk) {
  const int i = blockIdx.y;
  const ClassDev C = ld_const(P.classes + ld_const(P.shell_class + i));
  if (C.bands == nullptr || (int)blockIdx.x >= C.nbands) return;
  const int4 bd = ld_const(C.bands + blockIdx.x);   // (j0, nj, nk, kind)
  const auto in = gmem(in_ + (size_t)i * P.ncell);
  const auto out = gmem(out_ + (size_t)i * P.ncell);
  if (bd.w == 0) {   // single cells
    if (COPY && in_ != out_) {
      const int q0 = bd.x * P.nphi, q1 = (bd.x + bd.y) * P.nphi;
      for (int q = q0 + threadIdx.x; q < q1; q += LB_THREADS) __builtin_nontemporal_store((double)in[q], &out[q]);
    }
    return;
  }
  if (bd.w != 1) return;   // large blocks: launch_large
  if (bd.y == 1 && bd.z <= skip_nk) return;   // averaged by the caller's own kernels
  const auto dom = gmem(P.dom);
  for (int k0 = 0; k0 < P.nphi; k0 += LB_THREADS) {
    const int k = k0 + threadIdx.x;
    double a = 0.0, w = 0.0;
    if (k < P.nphi)
      for (int j = bd.x; j < bd.x + bd.y; ++j) {
        const int q = j * P.nphi + k;
        const double d = dom[q];
        a += d * in[q];
        w += d;
      }
    for (int d = 1; d < bd.z; d <<= 1) {
      a += __shfl_xor(a, d, 64);
      w += __shfl_xor(w, d, 64);
    }
    if (k < P.nphi) {
      const double v = a / w;
      for (int j = bd.x; j < bd.x + bd.y; ++j) {
        // the coarsened field streams out; block means of the solve stay
        // cached for the kernel that reads them next
        if constexpr (COPY) __builtin_nontemporal_store(v, &out[j * P.nphi + k]);
        else out[j * P.nphi + k] = v;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_bcast(BatchDev B) { bcast_item(B, job_of(B, PH_BCAST, blockIdx.x)); }

}  // namespace

hipError_t launch_bcast(const BatchDev &B, int wgs, hipStream_t s) {
  if (wgs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bcast, dim3(wgs), dim3(256), 0, s, B);
  return hipGetLastError();
}

hipError_t launch_bands(const PlanDev &P, int mode, const double *in, double *out, hipStream_t s, int skip_nk) {
  if (P.max_bands == 0 || P.nr == 0) return hipSuccess;
  const dim3 grid((unsigned)P.max_bands, (unsigned)P.nr), block(LB_THREADS);
  if (mode == kBandCoarsen)
    hipLaunchKernelGGL(k_band<true>, grid, block, 0, s, P, in, out, 0);
  else
    hipLaunchKernelGGL(k_band<false>, grid, block, 0, s, P, in, out, skip_nk);
  return hipGetLastError();
}

hipError_t launch_large(const PlanDev &P, int mode, const double *in, double *out, hipStream_t s) {
  if (P.n_lchunks == 0) return hipSuccess;
  const dim3 grid((unsigned)P.n_lchunks), block(LB_THREADS);
  switch (mode) {
    case kLargeMean:
      hipLaunchKernelGGL(k_large_part<false>, grid, block, 0, s, P, in);
      if (hipPeekAtLastError() != hipSuccess) break;
      hipLaunchKernelGGL(k_large_fill<kLargeMean>, grid, block, 0, s, P, out);
      break;
    case kLargeSum:
      hipLaunchKernelGGL(k_large_part<true>, grid, block, 0, s, P, in);
      if (hipPeekAtLastError() != hipSuccess) break;
      hipLaunchKernelGGL(k_large_fill<kLargeSum>, grid, block, 0, s, P, nullptr);
      break;
    case kLargeBcast: hipLaunchKernelGGL(k_large_fill<kLargeBcast>, grid, block, 0, s, P, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mpole
