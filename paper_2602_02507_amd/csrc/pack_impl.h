// Density streaming (the front of the solve): each coarsening block of each
// shell gets its share of the source, the sum over members of
// 4 pi G dOmega rho, i.e. dOmega_b S_b with S_b the solid-angle weighted block
// mean (GenASiS II Sec. 2.1 coarsening blocks; Eq. AngularMomentsDiscrete
// weights dOmega S).  The contractions run over block pairs (a block and its
// mirror image about the equator on a folded plan, else the block alone), so
// each pair gets the sum (even modes) and the difference (odd modes) of its
// two blocks' sources.
//
// One thread per pair of a shell, PACK_UNROLL pairs per thread spaced
// PACK_THREADS apart; runs of single-cell pairs (the common case) take a
// branch-free path whose loads are all issued before any is consumed, so
// enough bytes are in flight to stream rho at HBM rate.  Output by precision:
//   FP64      the packed row in FP64 (operand of the f64 moment contraction);
//   BF16 x3   the split planes of the deviation from the shell's mean
//             (below; bfloat16 has the exponent range of FP32, so the row
//             needs no scaling), plus per-workgroup partial sums of the FP64
//             monopole moment sum_b P_b T_b0;
//   FP16 x2   the FP64 deviation row, per-workgroup partial maxima and
//             monopole sums; a second kernel scales and splits once the row
//             maximum is known.
#pragma once
#include <algorithm>

#include "device_util.h"
#include "split_util.h"

namespace mpole {
namespace {


constexpr int PACK_THREADS = 256, PACK_UNROLL = 4, PACK_SPAN = PACK_THREADS * PACK_UNROLL;
static_assert(PACK_SPAN == kPackSpan, "packing span");

// Source sum 4 pi G dOmega rho and weight 4 pi G dOmega of block b (< 0:
// none) of shell i: a single cell directly, larger blocks from their member
// list or, past kLargeBlock cells, from the sum launch_large wrote.
__device__ __forceinline__ void block_sw(const PlanDev &P, const ClassDev &C, int i, int b, const double *w,
                                         const double *src, double &s, double &wt) {
  s = 0.0;
  wt = 0.0;
  if (b < 0) return;
  int n;
  if (C.rect != nullptr) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    const i4 r = gmem(reinterpret_cast<const i4 *>(C.rect))[b];   // (j0, k0, nj, nk)
    if (r.z * r.w == 1) {
      const int q = r.x * P.nphi + r.y;
      wt = gmem(w)[q];
      s = wt * gmem(src)[q];
      return;
    }
    n = r.z * r.w;
  } else {
    n = gmem(C.moff)[b + 1] - gmem(C.moff)[b];
  }
  s = n > kLargeBlock ? large_source(P, C, i, b) : block_source(C, w, src, P.nphi, b);
  wt = gmem(C.wsum)[b];
}

// One pair's packed values: the even and odd sources less the shift times
// the even and odd weights; the sum of the even sources (the monopole
// moment over sqrt(4 pi): the l = 0 kernel is the constant P~_0^0 =
// 1/sqrt(4 pi) on every block) and the row maximum (FP16 x2) accumulate.
template <int MODE>
__device__ __forceinline__ void pack_vals(bool fold, double se, double so, double we, double wo, double shift,
                                          double &de, double &dod, double &mono, double &mx) {
  de = MODE != 0 ? se - shift * we : se;
  dod = MODE != 0 ? so - shift * wo : so;
  if (MODE != 0) {
    mono += se;
    mx = fmax(mx, fmax(fabs(de), fold ? fabs(dod) : 0.0));
  }
}

// Stores of one pair's packed values: the FP64 rows (FP64, FP16 x2) or the
// split planes (BF16 x3, 2-byte stores).
template <int MODE>
__device__ __forceinline__ void pack_store(const ClassDev &C, bool fold, int row, int q, double de, double dod) {
  if (MODE == kSplitBf16x3) {
    split_store<kSplitBf16x3>(de, C.ppacks + row_index<kSplitBf16x3>(row, q, C.npair_pad), 16);
    if (fold) split_store<kSplitBf16x3>(dod, C.ppacks_o + row_index<kSplitBf16x3>(row, q, C.npair_pad), 16);
  } else {
    gmem(C.pack)[(size_t)row * C.npair_pad + q] = de;
    if (fold) gmem(C.pack_o)[(size_t)row * C.npair_pad + q] = dod;
  }
}

template <int MODE>
__device__ __forceinline__ void pack_emit(const ClassDev &C, bool fold, int row, int q, double se, double so,
                                          double we, double wo, double shift, double &mono, double &mx) {
  double de, dod;
  pack_vals<MODE>(fold, se, so, we, wo, shift, de, dod, mono, mx);
  pack_store<MODE>(C, fold, row, q, de, dod);
}

// Band task tx of a class (the block map is theta bands): lanes take phi
// columns k; a task of single-cell rows (nk = 1) packs pair q0 + r nphi + k
// from cell (j0 + r, k) and its mirror cell (ntheta-1-j0-r, k); a task of
// nj x nk merged blocks sums each column down the band's rows (and the
// mirror band's), combines the nk lanes of a block by xor butterflies
// (blocks are aligned and nk <= 64 divides the wavefront), and packs pair
// q0 + k / nk.  Coalesced loads, all issued before they are used; a cell's
// weight is its row factor times its column width (bitwise the weight
// table).  BF16 x3 rows of single cells whose pairs start at multiples of 8
// go through LDS and leave as 16-byte stores of 8 pairs of one plane.
constexpr int STAGE_PAIRS = kBandCopyRows * PACK_THREADS;

// Writes the split planes staged in LDS as 16-byte pieces (8 pairs of one
// plane): runs r < nrun_rows of len pairs (a multiple of 8) starting at pair
// q_first + r * q_step (a multiple of 8), parity par at st + ((r * 2 + par)
// * 3 + plane) * PACK_THREADS.  Called by the whole workgroup.
__device__ __forceinline__ void stage_out(const ClassDev &C, bool fold, int row, const uint16_t *st, int nrun_rows,
                                          int len, int q_first, int q_step) {
  const int nh = len / 8, npar = fold ? 2 : 1;
  const int items = nrun_rows * npar * 3 * nh;
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  for (int it = item_tid(); it < items; it += PACK_THREADS) {
    const int h = it % nh, rest = it / nh;
    const int plane = rest % 3, rp = rest / 3;
    const int par = rp % npar, r = rp / npar;
    const u4 v = *reinterpret_cast<const u4 *>(st + ((r * 2 + par) * 3 + plane) * PACK_THREADS + 8 * h);
    const int q = q_first + r * q_step + 8 * h;
    uint16_t *dst = (par ? C.ppacks_o : C.ppacks) + row_index<kSplitBf16x3>(row, q, C.npair_pad) + 16 * plane;
    *gmem(reinterpret_cast<u4 *>(dst)) = v;
  }
}
template <int MODE>
__device__ __forceinline__ void pack_band(const PlanDev &P, const ClassDev &C, int row, int tx, const double *src,
                                          double shift, double &mono, double &mx, uint16_t *st) {
  const int4 tk = ld_const(C.ptasks + tx);
  const int j0 = tk.x, nj = tk.y, nk = tk.z, q0 = tk.w;
  const bool fold = P.fold != 0;
  const bool self = !fold || j0 + nj - 1 == P.ntheta - 1 - j0;   // the band is its own mirror
  const auto srcg = gmem(src);
  const auto dphi = gmem(static_cast<const double *>(P.dphi));
  const int mrow0 = P.ntheta - 1 - j0;   // mirror of row j0 (mirror of j0 + r is mrow0 - r)
  const bool staged = MODE == kSplitBf16x3 && nk == 1 && ((q0 | P.nphi) & 7) == 0;
  for (int k0 = 0; k0 < P.nphi; k0 += PACK_THREADS) {
    const int k = k0 + item_tid();
    const bool kin = k < P.nphi;
    const int kc = kin ? k : 0;
    const double dp = kin ? dphi[kc] : 0.0;
    if (nk == 1) {
      double xr[kBandCopyRows], xm[kBandCopyRows];
#pragma unroll
      for (int r = 0; r < kBandCopyRows; ++r) {
        const int rr = min(r, nj - 1);
        xr[r] = srcg[(j0 + rr) * P.nphi + kc];
        xm[r] = self ? 0.0 : srcg[(mrow0 - rr) * P.nphi + kc];
      }
#pragma unroll
      for (int r = 0; r < kBandCopyRows; ++r) {
        if (r >= nj) break;
        const double wr = ld_const(P.wrow + j0 + r) * dp;
        const double wm = self ? 0.0 : ld_const(P.wrow + mrow0 - r) * dp;
        const double sr = wr * xr[r], sm = wm * xm[r];
        const int q = q0 + r * P.nphi + k;
        if (!staged) {
          if (kin) pack_emit<MODE>(C, fold, row, q, sr + sm, sr - sm, wr + wm, wr - wm, shift, mono, mx);
        } else if (kin) {
          double de, dod;
          pack_vals<MODE>(fold, sr + sm, sr - sm, wr + wm, wr - wm, shift, de, dod, mono, mx);
          // planes of row r, parity 0/1: st[((r * 2 + par) * 3 + plane) * 256 + lane]
          split_store<kSplitBf16x3>(de, st + (r * 2 + 0) * 3 * PACK_THREADS + item_tid(), PACK_THREADS);
          if (fold) split_store<kSplitBf16x3>(dod, st + (r * 2 + 1) * 3 * PACK_THREADS + item_tid(), PACK_THREADS);
        }
      }
      if (staged) {
        __syncthreads();
        // the chunk's runs of each row: pairs q0 + r nphi + k0 ..
        stage_out(C, fold, row, st, nj, min(PACK_THREADS, P.nphi - k0), q0 + k0, P.nphi);
        __syncthreads();
      }
    } else {
      double a = 0.0, w = 0.0, am = 0.0, wn = 0.0;
#pragma unroll 4
      for (int r = 0; r < nj; ++r) {
        const double wc = ld_const(P.wrow + j0 + r) * dp, xc = srcg[(j0 + r) * P.nphi + kc];
        const double wcm = self ? 0.0 : ld_const(P.wrow + mrow0 - r) * dp;
        const double xcm = self ? 0.0 : srcg[(mrow0 - r) * P.nphi + kc];
        a += wc * xc;
        w += wc;
        am += wcm * xcm;
        wn += wcm;
      }
      if (!kin) a = w = am = wn = 0.0;
      for (int d = 1; d < nk; d <<= 1) {
        a += __shfl_xor(a, d, 64);
        w += __shfl_xor(w, d, 64);
        am += __shfl_xor(am, d, 64);
        wn += __shfl_xor(wn, d, 64);
      }
      // BF16 x3: the chunk's pairs q0 + k0/nk .. staged when they start at a
      // multiple of 8 and come in multiples of 8
      const int npc = min(PACK_THREADS, P.nphi - k0) / nk;
      const bool mstaged = MODE == kSplitBf16x3 && (((q0 + k0 / nk) | npc) & 7) == 0;
      if (kin && (k & (nk - 1)) == 0) {
        if (!mstaged) {
          pack_emit<MODE>(C, fold, row, q0 + k / nk, a + am, a - am, w + wn, w - wn, shift, mono, mx);
        } else {
          double de, dod;
          pack_vals<MODE>(fold, a + am, a - am, w + wn, w - wn, shift, de, dod, mono, mx);
          const int t = item_tid() / nk;
          split_store<kSplitBf16x3>(de, st + 0 * 3 * PACK_THREADS + t, PACK_THREADS);
          if (fold) split_store<kSplitBf16x3>(dod, st + 1 * 3 * PACK_THREADS + t, PACK_THREADS);
        }
      }
      if (mstaged) {
        __syncthreads();
        stage_out(C, fold, row, st, 1, npc, q0 + k0 / nk, 0);
        __syncthreads();
      }
    }
  }
}

// LDS of a packing item in bytes: the reduction slots, then the plane stage
// (the band path's or the span path's, never both)
constexpr int PACK_LDS = 256 + 2 * 3 * STAGE_PAIRS * 2;

// Packing workgroup J.local of field J.f (start_stamp: record the batch
// start time).
template <int MODE>   // 0 = FP64, kSplitBf16x3, kSplitFp16x2
__device__ __forceinline__ void pack_item(const BatchDev &B, const Job &J, char *lds, bool start_stamp) {
  double *red = reinterpret_cast<double *>(lds);
  const PlanDev &P = J.P;
  if (B.stamps != nullptr && start_stamp && item_tid() == 0) B.stamps[B.nf] = wall_clock64();
  const int bx = J.local % P.pack_parts, i = J.local / P.pack_parts;   // (part, shell)
  const double *__restrict__ rho = J.io.rho;
  const ClassDev C = ld_const(P.classes + ld_const(P.shell_class + i));
  const int q0 = bx * PACK_SPAN + item_tid();   // this thread's first pair
  if (bx >= C.npack) return;   // whole workgroup idle for this class
  const int row = ld_const(P.shell_row + i);
  const double *__restrict__ src = rho + (size_t)i * P.ncell;
  const double *__restrict__ w = P.weight;
  const auto srcg = gmem(src), wg = gmem(w);
  const bool fold = P.fold != 0;
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
  double mono = 0.0, mx = 0.0;
  if (C.ptasks != nullptr) {
    pack_band<MODE>(P, C, row, bx, src, shift, mono, mx, reinterpret_cast<uint16_t *>(lds + 256));
    // the padding pairs past the last one are zero
    const int q = C.npair + item_tid();
    if (bx == 0 && q < C.npair_pad) pack_emit<MODE>(C, fold, row, q, 0.0, 0.0, 0.0, 0.0, 0.0, mono, mx);
  } else {
  // per pair (rep, mir): the even and odd combinations of the two blocks'
  // sources and weights (the mirror's part left out when mir == rep)
  double se[PACK_UNROLL], so[PACK_UNROLL], we[PACK_UNROLL], wo[PACK_UNROLL];
  const int run0 = ld_const(C.pspan0 + bx);
  if (run0 >= 0) {
    // the span's rep blocks are single cells at consecutive cells and their
    // mirrors the mirror cells: coalesced loads, no block descriptors
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const bool ok = q0 + u * PACK_THREADS < C.npair;
      const int c = run0 + item_tid() + u * PACK_THREADS;
      const int cm = fold ? (P.ntheta - 1 - c / P.nphi) * P.nphi + c % P.nphi : c;
      const double wr = ok ? wg[c] : 0.0;
      const double wm = (ok && cm != c) ? wg[cm] : 0.0;
      const double sr = wr * srcg[ok ? c : run0], sm = wm * srcg[ok ? cm : run0];
      se[u] = sr + sm;
      so[u] = sr - sm;
      we[u] = wr + wm;
      wo[u] = wr - wm;
    }
  } else {
    const auto prs = gmem(reinterpret_cast<const i2v *>(C.pairs));
    i2v pr[PACK_UNROLL];
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int q = q0 + u * PACK_THREADS;
      pr[u] = q < C.npair ? prs[q] : i2v{-1, -1};
    }
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      double sr, wr, sm, wm;
      block_sw(P, C, i, pr[u].x, w, src, sr, wr);
      block_sw(P, C, i, pr[u].y != pr[u].x ? pr[u].y : -1, w, src, sm, wm);
      se[u] = sr + sm;
      so[u] = sr - sm;
      we[u] = wr + wm;
      wo[u] = wr - wm;
    }
  }
  double de[PACK_UNROLL], dod[PACK_UNROLL];
#pragma unroll
  for (int u = 0; u < PACK_UNROLL; ++u) {
    de[u] = MODE != 0 ? se[u] - shift * we[u] : se[u];
    dod[u] = MODE != 0 ? so[u] - shift * wo[u] : so[u];
  }
  if (MODE == kSplitBf16x3) {
    // split into LDS copies of this workgroup's 64 k-slab groups of 16 pairs,
    // [group][plane][16], then write each group's 96 contiguous bytes
    uint16_t(*stage)[PACK_SPAN / 16][3][16] = reinterpret_cast<uint16_t(*)[PACK_SPAN / 16][3][16]>(lds + 256);
#pragma unroll
    for (int u = 0; u < PACK_UNROLL; ++u) {
      const int ql = item_tid() + u * PACK_THREADS;   // pair within this workgroup
      const bool ok = q0 + u * PACK_THREADS < C.npair;
      split_store<kSplitBf16x3>(ok ? de[u] : 0.0, &stage[0][ql >> 4][0][ql & 15], 16);
      if (fold) split_store<kSplitBf16x3>(ok ? dod[u] : 0.0, &stage[1][ql >> 4][0][ql & 15], 16);
    }
    __syncthreads();
    const int g0 = bx * (PACK_SPAN / 16);                        // first k slab of the workgroup
    const int ngroups = min(PACK_SPAN / 16, C.npair_pad / 16 - g0);
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    for (int par = 0; par < (fold ? 2 : 1); ++par) {
      const u4 *st = reinterpret_cast<const u4 *>(&stage[par][0][0][0]);
      uint16_t *dst0 = par ? C.ppacks_o : C.ppacks;
      for (int v = item_tid(); v < ngroups * 6; v += PACK_THREADS) {   // 6 x 16 B per group
        const int g = v / 6, part = v % 6;
        const auto dst = gmem(reinterpret_cast<u4 *>(dst0 + row_index<kSplitBf16x3>(row, 16 * (g0 + g), C.npair_pad)));
        dst[part] = st[g * 6 + part];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PACK_UNROLL; ++u) {
    const int q = q0 + u * PACK_THREADS;
    // the FP64 rows including their zero padding up to npair_pad (the padding
    // lies in the span of the last pair: spans are multiples of 16 long)
    if (MODE != kSplitBf16x3 && q < C.npair_pad) {
      gmem(C.pack)[(size_t)row * C.npair_pad + q] = q < C.npair ? de[u] : 0.0;
      if (fold) gmem(C.pack_o)[(size_t)row * C.npair_pad + q] = q < C.npair ? dod[u] : 0.0;
    }
    if (q >= C.npair) continue;
    if (MODE != 0) {
      mono += se[u];
      mx = fmax(mx, fmax(fabs(de[u]), fold ? fabs(dod[u]) : 0.0));
    }
  }
  }   // span path
  if (MODE != 0) {
    if (bx == 0 && item_tid() == 0) {
      gmem(P.shift)[i] = shift;
      if (MODE == kSplitBf16x3) gmem(C.pscale)[row] = 1.0;   // BF16 x3 rows are not scaled
    }
    mono = block_sum(mono, red) * (1.0 / sqrt(4.0 * kPi));
    if (MODE == kSplitFp16x2) mx = block_max(mx, red);
    if (item_tid() == 0) {
      P.mono_part[(size_t)i * P.mono_stride + bx] = mono;
      if (MODE == kSplitFp16x2) P.max_part[(size_t)i * P.mono_stride + bx] = mx;
    }
  }
}

// FP16 x2: chunk c of shell i's row (kSplitRowChunk pairs of both parities):
// the row's power-of-two scale from the maximum of the shell's partial
// maxima (reduced across the workgroup: a maximum is exact in any order, so
// every workgroup of the shell gets the same scale), then the scaled split
// planes of the chunk's pairs.  The row loads are issued before the scale
// is known; red holds 4 doubles of LDS.
__device__ __forceinline__ void split_rows_item(const BatchDev &B, const Job &J, double *red) {
  constexpr int U = kSplitRowChunk / 256;
  const PlanDev &P = J.P;
  const int i = J.local / P.split_chunks, q0 = (J.local % P.split_chunks) * kSplitRowChunk;
  const ClassDev C = ld_const(P.classes + ld_const(P.shell_class + i));
  if (q0 >= C.npair_pad) return;   // past this class's row (workgroup-uniform)
  const int row = ld_const(P.shell_row + i);
  const int npar = P.fold ? 2 : 1;
  double v[2][U];
#pragma unroll
  for (int par = 0; par < 2; ++par)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u * 256 + item_tid();
      const double *__restrict__ prow = (par ? C.pack_o : C.pack) + (size_t)row * C.npair_pad;
      v[par][u] = par < npar && q < C.npair_pad ? prow[q] : 0.0;   // the row's zero padding included
    }
  double mx = 0.0;
  for (int q = item_tid(); q < C.npack; q += 256) mx = fmax(mx, P.max_part[(size_t)i * P.mono_stride + q]);
  mx = block_max(mx, red);
  const double scale = row_scale(mx);
  const double inv = 1.0 / scale;   // exact: a power of two
#pragma unroll
  for (int par = 0; par < 2; ++par)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u * 256 + item_tid();
      if (par < npar && q < C.npair_pad)
        split_store<kSplitFp16x2>(v[par][u] * inv,
                                  (par ? C.ppacks_o : C.ppacks) + row_index<kSplitFp16x2>(row, q, C.npair_pad), 16);
    }
  if (q0 == 0 && item_tid() == 0) C.pscale[row] = scale;
}

}  // namespace
}  // namespace mpole
