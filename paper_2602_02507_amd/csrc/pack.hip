// Density streaming (the front of the solve): each coarsening block of each
// shell gets its share of the source, the sum over members of
// 4 pi G dOmega rho, i.e. dOmega_b S_b with S_b the solid-angle weighted block
// mean (GenASiS II Sec. 2.1 coarsening blocks; Eq. AngularMomentsDiscrete
// weights dOmega S).
//
// One thread per block of a shell, PACK_UNROLL blocks per thread spaced
// PACK_THREADS apart; single-cell blocks (the common case) take a branch-free
// path whose loads are all issued before any is consumed, so enough bytes are
// in flight to stream rho at HBM rate.  Output by precision:
//   FP64      the packed row in FP64 (operand of the f64 moment contraction);
//   BF16 x3   the split planes of the deviation from the shell's mean
//             (below; bfloat16 has the exponent range of FP32, so the row
//             needs no scaling), plus per-workgroup partial sums of the FP64
//             monopole moment sum_b P_b T_b0;
//   FP16 x2   the FP64 deviation row, per-workgroup partial maxima and
//             monopole sums; a second kernel scales and splits once the row
//             maximum is known.
#include <algorithm>

#include "device_util.h"
#include "split_util.h"

namespace mpole {
namespace {

constexpr int PACK_THREADS = 256, PACK_UNROLL = 4, PACK_SPAN = PACK_THREADS * PACK_UNROLL;
static_assert(PACK_SPAN == kPackSpan, "packing span");

template <int MODE>   // 0 = FP64, kSplitBf16x3, kSplitFp16x2
__global__ __launch_bounds__(PACK_THREADS) void k_pack(BatchDev B) {
  __shared__ double red[PACK_THREADS / 64];
  const Job J = job_of(B, PH_PACK, blockIdx.x);
  const PlanDev &P = J.P;
  // batch start: the first workgroup of the first launch of the solve
  if (B.stamps != nullptr && blockIdx.x == 0 && threadIdx.x == 0) B.stamps[B.nf] = wall_clock64();
  const int bx = J.local % P.pack_parts, i = J.local / P.pack_parts;   // (part, shell)
  const double *__restrict__ rho = J.io.rho;
  const ClassDev C = ld_const(P.classes + ld_const(P.shell_class + i));
  const int b0 = bx * PACK_SPAN + threadIdx.x;
  if (bx * PACK_SPAN >= C.nblocks) return;   // whole workgroup idle for this class
  const int row = ld_const(P.shell_row + i);
  const double *__restrict__ src = rho + (size_t)i * P.ncell;
  const double *__restrict__ w = P.weight;
  const auto srcg = gmem(src), wg = gmem(w);
  // Split precisions carry only the deviation of the source from c times the
  // block weight, c a per-shell reference density (exact identity, l >= 1):
  //   sum_b P_b T_bn = sum_b (P_b - c W_b) T_bn + c sum_b W_b T_bn,
  // with W_b the block's 4 pi G dOmega; the last sum is a bind-time FP64
  // constant (zero for l >= 1 up to quadrature error) added back by the
  // reduction.  For a near-spherical source the deviation is a small
  // fraction of P, and so are the rounding errors of the narrow operands and
  // of the FP32 accumulation; any c keeps the sums exact.  c is the
  // weight-averaged density of kShiftSamples cells at spread-out theta (phi
  // index 0), read with uniform loads by every thread of every workgroup of
  // the shell and combined in the same order, so all agree bitwise; the
  // monopole sums below use P itself.
  double shift = 0.0;
  if (MODE != 0) {
    double a = 0.0, wsm = 0.0;
#pragma unroll
    for (int k = 0; k < kShiftSamples; ++k) {
      const int q = (int)(((2L * k + 1) * P.ntheta) / (2 * kShiftSamples)) * P.nphi;
      a += wg[q] * srcg[q];
      wsm += wg[q];
    }
    shift = wsm > 0.0 ? a / wsm : 0.0;   // stored at the end: no store ahead of the loads
  }
  double s[PACK_UNROLL], wb[PACK_UNROLL];   // block source and block weight
  const int run0 = ld_const(C.span0 + bx);
  if (run0 >= 0) {
    // the span is a run of single-cell blocks at consecutive cells: coalesced
    // loads, no block descriptors
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int b = b0 + u * PACK_THREADS;
      const int q = run0 + threadIdx.x + u * PACK_THREADS;
      wb[u] = (b < C.nblocks) ? wg[q] : 0.0;
      s[u] = (b < C.nblocks) ? wb[u] * srcg[q] : 0.0;
    }
  } else if (C.rect != nullptr) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    const auto rect = gmem(reinterpret_cast<const i4 *>(C.rect));   // (j0, k0, nj, nk) per block
    i4 r[PACK_UNROLL];
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int b = b0 + u * PACK_THREADS;
      r[u] = (b < C.nblocks) ? rect[b] : i4{0, 0, 0, 0};
    }
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int q = r[u].x * P.nphi + r[u].y;
      const bool one = r[u].z == 1 && r[u].w == 1;
      wb[u] = one ? wg[q] : 0.0;
      s[u] = one ? wb[u] * srcg[q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int b = b0 + u * PACK_THREADS;
      if (b < C.nblocks && (r[u].z != 1 || r[u].w != 1)) {
        s[u] = r[u].z * r[u].w > kLargeBlock ? large_source(P, C, i, b) : block_source(C, w, src, P.nphi, b);
        wb[u] = gmem(C.wsum)[b];
      }
    }
  } else {
    const auto moff = gmem(C.moff);
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int b = b0 + u * PACK_THREADS;
      s[u] = 0.0;
      if (b < C.nblocks)
        s[u] = moff[b + 1] - moff[b] > kLargeBlock ? large_source(P, C, i, b) : block_source(C, w, src, P.nphi, b);
      wb[u] = (b < C.nblocks && MODE != 0) ? gmem(C.wsum)[b] : 0.0;
    }
  }
  double dev[PACK_UNROLL];
#pragma unroll
  for (int u = 0; u < PACK_UNROLL; ++u) dev[u] = MODE != 0 ? s[u] - shift * wb[u] : s[u];
  double mono = 0.0, mx = 0.0;
  if (MODE == kSplitBf16x3) {
    // split into an LDS copy of this workgroup's 64 k-slab groups of 16
    // blocks, [group][plane][16], then write each group's 96 contiguous bytes
    __shared__ uint16_t stage[PACK_SPAN / 16][3][16];
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int bl = threadIdx.x + u * PACK_THREADS;   // block within this workgroup
      const int b = b0 + u * PACK_THREADS;
      split_store<kSplitBf16x3>(b < C.nblocks ? dev[u] : 0.0, &stage[bl >> 4][0][bl & 15], 16);
    }
    __syncthreads();
    const int g0 = bx * (PACK_SPAN / 16);                        // first k slab of the workgroup
    const int ngroups = min(PACK_SPAN / 16, C.nblocks_pad / 16 - g0);
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4 *st = reinterpret_cast<const u4 *>(&stage[0][0][0]);
    for (int v = threadIdx.x; v < ngroups * 6; v += PACK_THREADS) {   // 6 x 16 B per group
      const int g = v / 6, part = v % 6;
      const auto dst = gmem(reinterpret_cast<u4 *>(C.ppacks + ((size_t)(g0 + g) * C.nrows + row) * 48));
      dst[part] = st[g * 6 + part];
    }
  }
#pragma unroll
  for (int u = 0; u < PACK_UNROLL; ++u) {
    const int b = b0 + u * PACK_THREADS;
    // the FP64 row including its zero padding up to nblocks_pad (the padding
    // lies in the span of the last block: spans are multiples of 16 long)
    if (MODE != kSplitBf16x3 && b < C.nblocks_pad)
      gmem(C.pack)[(size_t)row * C.nblocks_pad + b] = b < C.nblocks ? dev[u] : 0.0;
    if (b >= C.nblocks) continue;
    if (MODE != 0) {
      mono += s[u] * gmem(C.tcol0)[b];
      mx = fmax(mx, fabs(dev[u]));
    }
  }
  if (MODE != 0) {
    if (bx == 0 && threadIdx.x == 0) {
      gmem(P.shift)[i] = shift;
      if (MODE == kSplitBf16x3) gmem(C.pscale)[row] = 1.0;   // BF16 x3 rows are not scaled
    }
    mono = block_sum(mono, red);
    if (MODE == kSplitFp16x2) mx = block_max(mx, red);
    if (threadIdx.x == 0) {
      P.mono_part[(size_t)i * P.mono_stride + bx] = mono;
      if (MODE == kSplitFp16x2) P.max_part[(size_t)i * P.mono_stride + bx] = mx;
    }
  }
}

// FP16 x2: per shell, the row's power-of-two scale from the partial maxima,
// then the scaled split planes of the FP64 row.
__global__ __launch_bounds__(256) void k_split_rows_fp16(BatchDev B) {
  const Job J = job_of(B, PH_SPLITROWS, blockIdx.x);
  const PlanDev &P = J.P;
  const int i = J.local;
  const ClassDev C = ld_const(P.classes + ld_const(P.shell_class + i));
  const int row = ld_const(P.shell_row + i);
  const int nparts = (C.nblocks + PACK_SPAN - 1) / PACK_SPAN;
  double mx = 0.0;
  for (int q = 0; q < nparts; ++q) mx = fmax(mx, P.max_part[(size_t)i * P.mono_stride + q]);
  const double scale = row_scale(mx);
  const double inv = 1.0 / scale;   // exact: a power of two
  const double *__restrict__ prow = C.pack + (size_t)row * C.nblocks_pad;
  for (int b = threadIdx.x; b < C.nblocks_pad; b += 256)   // zero planes past the last block
    split_store<kSplitFp16x2>(b < C.nblocks ? prow[b] * inv : 0.0,
                              C.ppacks + slab_index<kSplitFp16x2>(row, b, C.nrows), 16);
  if (threadIdx.x == 0) C.pscale[row] = scale;
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
