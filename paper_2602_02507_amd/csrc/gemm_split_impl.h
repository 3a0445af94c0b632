// Device code of the two angular contractions with split narrow-float operands on MFMA
// (v_mfma_f32_32x32x16_bf16 / _f16) with FP32 accumulation.
//
//   moment:  A[i][n]   = s_i sum_b  Ps[i][b] TT[n][b]      (Ps = P / s_i, split)
//   expand:  Phi[i][b] = c_i sum_n  Cs[i][n] T[b][n]       (Cs = C / c_i, split)
//
// Both are "NT" products, out[m][n] = sum_k X[m][k] Y[n][k].  Every split
// operand is stored k-slab major with its planes interleaved,
// [k/16][row][plane][k%16] (the moment contraction reads a transposed copy of
// the kernel table), so one 16-wide K stage of 128 consecutive rows is a
// contiguous run that moves to LDS as fully coalesced 16-byte copies, and each
// lane's MFMA fragment is one 16-byte LDS read.  With x = x_hi + x_mid + x_lo (BF16 x3) the product keeps the six
// terms hi.hi, hi.mid, mid.hi, hi.lo, lo.hi, mid.mid (the dropped ones are
// below 2^-24 relative); with FP16 x2 the three terms hi.hi, hi.lo, lo.hi.
//
// Workgroup: 4 wavefronts in 2 x 2, tile TM x 128 (TM = 128 or 64), each
// wavefront (TM/2) x 64 as (TM/64) x 2 MFMA 32x32 tiles; K advances 16 per LDS
// stage (one MFMA step),
// double-buffered in LDS with loads issued two stages ahead.  Accumulation is FP32.  The monopole (l = 0) carries most
// of both sums for the near-spherical sources of interest, so it is taken out
// of the FP32 sums and done in FP64 elsewhere: the monopole moment is summed in
// FP64 by the packing kernel, and the expansion coefficient of l = 0 is zeroed
// in the split planes and its term C_i0 T_b0 added in FP64 here, in the
// epilogue.  The FP32 sums then only carry the (small) l >= 1 remainder.
//
// 32x32x16 lane layout on gfx950 (checked on the device): lane l supplies
// X[l%32][8(l/32) .. 8(l/32)+7] and Y[l%32][same k]; result register r of lane
// l holds out[(r%4) + 8(r/4) + 4(l/32)][l%32].
#pragma once
#include "device_util.h"

namespace mpole {
namespace {


typedef float f16v __attribute__((ext_vector_type(16)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));   // 16 raw bytes
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

// Tile width TN and the K stage are fixed; the tile height TM is 128 or 64,
// chosen per plan and contraction (a tuning knob: 64 wastes less on short
// row counts and doubles the workgroups, 128 reuses each fragment twice).
constexpr int TMMAX = 128, TN = 128, TK = 16, NTH = 256;

template <int KIND>
struct Split;
template <>
struct Split<kSplitBf16x3> {
  static constexpr int planes = 3, products = 6;
  // (x plane, y plane) of each kept product
  static constexpr int px[6] = {0, 0, 1, 0, 2, 1};
  static constexpr int py[6] = {0, 1, 0, 2, 0, 1};
  static constexpr int sig[6] = {0, 4, 3, 7, 2, 6};   // LDS row rotation per chunk
  __device__ static inline f16v mfma(u4 a, u4 b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
  }
};
template <>
struct Split<kSplitFp16x2> {
  static constexpr int planes = 2, products = 3;
  static constexpr int px[3] = {0, 0, 1};
  static constexpr int py[3] = {0, 1, 0};
  static constexpr int sig[4] = {0, 2, 4, 6};
  __device__ static inline f16v mfma(u4 a, u4 b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
  }
};

// Operand source: element (row, k, plane) at base + ((k/16) rows + row) 16 NP + 16 plane + k%16
// (k-slab major), except the moment contraction's packed source, which is
// row-major: base + (row npair_pad/16 + k/16) 16 NP + 16 plane + k%16.
struct Operand {
  const uint16_t *base;
  int rows;
};

// One output tile of a contraction; LDS holds two stages of X (TMV rows)
// and Y (TN rows) in the slot layout described in the kernel.
template <int KIND, bool EXPAND, int TMV>
__device__ __forceinline__ void gemm_tile(const BatchDev &B, const PlanDev &P, const ClassDev &C,
                                          double *__restrict__ phi, int local, u4 *lds) {
  using S = Split<KIND>;
  constexpr int NP = S::planes, CH = 2 * NP, AT = TMV / 64;
  u4 *Xs = lds;                       // [2][CH][TMV]
  u4 *Ys = lds + 2 * CH * TMMAX;      // [2][CH][TN]
  const int m_tiles = EXPAND ? C.m_tiles_exp : C.m_tiles_mom;
  const int mt = local % m_tiles;
  const int rest = local / m_tiles;
  int nt, split = 0;
  if (EXPAND) {
    nt = rest;
  } else {
    nt = rest % C.n_tiles_mom;
    split = rest / C.n_tiles_mom;
  }
  const int m0 = mt * TMV, n0 = nt * TN;
  const int M = C.nrows;
  const int N = EXPAND ? C.npair : P.namp_m;
  int kbeg, kend;
  if (EXPAND) {
    kbeg = 0;
    kend = P.namp_e;
  } else {
    kbeg = split * C.kchunk;
    kend = min(kbeg + C.kchunk, C.npair_pad);
  }
  // operands, k-slab major with interleaved planes; a moment tile of odd mode
  // columns contracts the odd (difference) packed source
  Operand X, Y;
  if (EXPAND) {
    X = {P.cplanes, P.nr};
    Y = {C.tplanes, C.npair_pad};
  } else {
    X = {n0 >= P.odd_m0 ? C.ppacks_o : C.ppacks, C.nrows};
    Y = {C.ttplanes, P.namp_m};
  }
  const int tid = item_tid(), lane = tid & 63, w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;
  // this lane's fragment slots within a stage, per plane (rows 32 apart add 32)
  int rx_slot[NP], ry_slot[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int ch = 2 * p + (lane >> 5);
    const int low = (lane & 24) + ((lane + S::sig[ch]) & 7);
    rx_slot[p] = ch * TMV + low;
    ry_slot[p] = ch * TN + low;
  }
  // loader roles: a stage row is CH chunks of 16 bytes (plane, k half).  The
  // Y tile (128 rows) is moved by all threads, chunks t + 256 u; the X tile by
  // the first 2 TMV threads, chunks t + 2 TMV u (u < NP).
  const bool x_loader = tid < 2 * TMV;
  const int yrow_max = EXPAND ? C.npair_pad : P.namp_m;
  int lx_slot[NP], ly_slot[NP];
  bool x_ok[NP], y_ok[NP];
  size_t x_off[NP], y_off[NP];   // element offsets within a k slab
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    const int jy = tid + NTH * u, ry = jy / CH, cy = jy % CH;
    ly_slot[u] = cy * TN + (ry & ~7) + ((ry + S::sig[cy]) & 7);
    y_ok[u] = (n0 + ry) < yrow_max;
    y_off[u] = (size_t)(y_ok[u] ? n0 + ry : 0) * (16 * NP) + 8 * cy;
    const int jx = tid + 2 * TMV * u, rx = jx / CH, cx = jx % CH;
    lx_slot[u] = cx * TMV + (rx & ~7) + ((rx + S::sig[cx]) & 7);
    x_ok[u] = x_loader && (m0 + rx) < M;
    const int xr = EXPAND ? (x_ok[u] ? gmem(C.rows)[m0 + rx] : 0) : (x_ok[u] ? m0 + rx : 0);
    // expansion: k-slab major coefficients; moment: the row-major packed
    // source [row][k/16][plane][k%16], rows npair_pad long
    x_off[u] = (size_t)xr * (EXPAND ? 16 * NP : (size_t)C.npair_pad * NP) + 8 * cx;
  }
  const size_t x_slab = EXPAND ? (size_t)X.rows * 16 * NP : (size_t)16 * NP, y_slab = (size_t)Y.rows * 16 * NP;

  // accumulators: every stage goes to acc; a folded expansion parks its even
  // mode sums in acco at the parity boundary and sums the odd ones in acc
  f16v acc[AT][2], acco[EXPAND ? AT : 1][2];
#pragma unroll
  for (int a = 0; a < AT; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f16v{};
#pragma unroll
  for (int a = 0; a < (EXPAND ? AT : 1); ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acco[a][b] = f16v{};
  const int kodd = EXPAND ? P.odd_e0 : kend;   // first K of the odd mode columns
  const bool parked = EXPAND && kodd < kend;   // the K range holds odd columns

  // two register sets of staged operands: the loads of stage k+2 are issued
  // before stage k is computed and land in LDS only after stage k+1 is, so
  // each load has two stages of MFMA work to hide behind.  Loads are
  // unconditional (rows outside the operand read row 0) and go through global
  // address-space pointers, so nothing waits on them before the store.  In
  // the moment contraction a thread whose row is outside the operand stores
  // nothing: its LDS slots (it alone writes them) are zeroed once per tile
  // below, so no select on the loaded values (which the scheduler hoists into
  // the next stage's MFMAs, waiting on the loads there) is needed.  The
  // expansion, short of registers, zeroes them at the store.  With TMV = 64
  // the second half of the threads loads no X chunks (a wave-uniform
  // condition).
  typedef const __attribute__((address_space(1))) u4 *gptr;
  u4 xa[NP], ya[NP], xb[NP], yb[NP];
  const u4 zero = {0u, 0u, 0u, 0u};
#define GLOAD(XV, YV, K)                                                             \
  {                                                                                  \
    const size_t kx_ = (size_t)((K) >> 4) * x_slab, ky_ = (size_t)((K) >> 4) * y_slab; \
    _Pragma("unroll") for (int u = 0; u < NP; ++u) {                                 \
      if (TMV == TMMAX || x_loader) XV[u] = *(gptr)(X.base + kx_ + x_off[u]);        \
      YV[u] = *(gptr)(Y.base + ky_ + y_off[u]);                                      \
    }                                                                                \
  }
#define LSTORE(XV, YV, BUF)                                                          \
  {                                                                                  \
    _Pragma("unroll") for (int u = 0; u < NP; ++u) {                                 \
      if (EXPAND) {                                                                  \
        if (TMV == TMMAX || x_loader) Xs[(BUF) * CH * TMV + lx_slot[u]] = x_ok[u] ? XV[u] : zero; \
        Ys[(BUF) * CH * TN + ly_slot[u]] = y_ok[u] ? YV[u] : zero;                    \
      } else {                                                                       \
        if ((TMV == TMMAX || x_loader) && x_ok[u]) Xs[(BUF) * CH * TMV + lx_slot[u]] = XV[u]; \
        if (y_ok[u]) Ys[(BUF) * CH * TN + ly_slot[u]] = YV[u];                        \
      }                                                                              \
    }                                                                                \
  }
  auto stage = [&](int buf, f16v (&ac)[AT][2]) __attribute__((always_inline)) {
    u4 fa[AT][NP], fb[2][NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int t = 0; t < AT; ++t) fa[t][p] = Xs[buf * CH * TMV + rx_slot[p] + wm * (TMV / 2) + t * 32];
#pragma unroll
      for (int t = 0; t < 2; ++t) fb[t][p] = Ys[buf * CH * TN + ry_slot[p] + wn * 64 + t * 32];
    }
#pragma unroll
    for (int q = 0; q < S::products; ++q)
#pragma unroll
      for (int a = 0; a < AT; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) ac[a][b] = S::mfma(fa[a][S::px[q]], fb[b][S::py[q]], ac[a][b]);
  };
  // stage kt of this tile (k = kbeg + kt TK); after the last even stage of a
  // folded expansion the even sums are parked in acco and acc restarts at 0
  // for the odd stages (a workgroup-uniform branch)
  auto compute = [&](int buf, int kt) __attribute__((always_inline)) {
    stage(buf, acc);
    if constexpr (EXPAND) {
      if (parked && kbeg + (kt + 1) * TK == kodd) {
#pragma unroll
        for (int a = 0; a < AT; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            acco[a][b] = acc[a][b];
            acc[a][b] = f16v{};
          }
      }
    }
  };

  const int nk = (kend - kbeg) / TK;
  // moment: zero slots of the rows outside the operands, both stage buffers
  // (made visible by the first barrier; the LDS held other data before this
  // tile)
  if constexpr (!EXPAND) {
#pragma unroll
    for (int u = 0; u < NP; ++u)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if ((TMV == TMMAX || x_loader) && !x_ok[u]) Xs[b * CH * TMV + lx_slot[u]] = zero;
        if (!y_ok[u]) Ys[b * CH * TN + ly_slot[u]] = zero;
      }
  }
  if (nk > 0) GLOAD(xa, ya, kbeg);
  if (nk > 1) GLOAD(xb, yb, kbeg + TK);
  if (nk > 0) LSTORE(xa, ya, 0);
  __syncthreads();
  int kt = 0;
  // prefetches past the last stage re-read the last stage (branch-free, so
  // the wait before each LDS store covers only the older register set)
  const int klast = kend - TK;
  for (; kt + 1 < nk; kt += 2) {
    // even stage kt from LDS 0; register set b holds stage kt+1
    GLOAD(xa, ya, min(kbeg + (kt + 2) * TK, klast));
    compute(0, kt);
    LSTORE(xb, yb, 1);
    __syncthreads();
    // odd stage kt+1 from LDS 1; register set a holds stage kt+2
    GLOAD(xb, yb, min(kbeg + (kt + 3) * TK, klast));
    compute(1, kt + 1);
    if (kt + 2 < nk) LSTORE(xa, ya, 0);
    __syncthreads();
  }
#undef GLOAD
#undef LSTORE
  if (kt < nk) compute(0, kt);   // odd stage count: the last stage sits in LDS 0

  // epilogue: undo the row scale in FP64.  The tile's per-row values (the
  // shell, its coefficient scale and l = 0 coefficient; the moment rows'
  // source scales) are first staged in LDS, one row per thread: read per row
  // inside the store loop, each row's dependent loads would wait behind the
  // previous row's stores, a memory round trip per row.
  const auto rows = gmem(C.rows);
  const auto moff = gmem(C.moff), mem = gmem(C.mem);
  const auto tcol0 = gmem(C.tcol0);
  const auto cscale = gmem(P.cscale), coef = gmem(P.coef);
  const auto pscale = gmem(C.pscale);
  const auto part = gmem(reinterpret_cast<float *>(C.partial));
  double *e_sc = reinterpret_cast<double *>(lds);   // [TMV] row scale
  double *e_c0 = e_sc + TMV;                        // [TMV] l = 0 coefficient (expansion)
  int *e_shell = reinterpret_cast<int *>(e_c0 + TMV);   // [TMV] shell (expansion)
  __syncthreads();   // the last stage's LDS reads are done
  // This lane's two expansion pairs, read once for all its rows: l = 0
  // kernel and the member cells of both blocks, [0] the rep and [1] the
  // mirror (rect: first cell and extent; CSR: member range in bcell .. bnj).
  // The loads go in two rounds: the pairs, their l = 0 kernels and the tile
  // rows' shells; then the blocks' rectangles or member ranges and the
  // shells' scales and l = 0 coefficients (staged in LDS).
  typedef int i4v __attribute__((ext_vector_type(4)));
  bool bok[2] = {false, false}, bmir[2] = {false, false};
  double bt0[2] = {0.0, 0.0};
  int bcell[2][2] = {}, bnj[2][2] = {}, bnk[2][2] = {};
  i2v pr[2] = {};
  int shell_t = 0;
  const bool stager = tid < TMV && m0 + tid < M;
  if (EXPAND) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int q = n0 + wn * 64 + b * 32 + (lane & 31);
      bok[b] = q < N;
      if (!bok[b]) continue;
      bt0[b] = tcol0[q];
      pr[b] = gmem(reinterpret_cast<const i2v *>(C.pairs))[q];
    }
    if (stager) shell_t = rows[m0 + tid];
  } else if (stager) {
    e_sc[tid] = pscale[m0 + tid];
  }
  if (EXPAND) {
    const auto rect4 = gmem(reinterpret_cast<const i4v *>(C.rect));
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (!bok[b]) continue;
      bmir[b] = pr[b].y != pr[b].x;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int blk = h ? pr[b].y : pr[b].x;
        if (C.rect != nullptr) {
          const i4v rc = rect4[blk];   // (j0, k0, nj, nk)
          bcell[b][h] = rc.x * P.nphi + rc.y;
          bnj[b][h] = rc.z;
          bnk[b][h] = rc.w;
          // first cell only: launch_large (past kLargeBlock cells) or the
          // broadcast phase (merged blocks of a banded class) writes the rest
          if (bnj[b][h] * bnk[b][h] > kLargeBlock || C.bands != nullptr) bnj[b][h] = bnk[b][h] = 1;
        } else {
          bcell[b][h] = moff[blk];
          bnj[b][h] = moff[blk + 1];
          if (bnj[b][h] - bcell[b][h] > kLargeBlock) bnj[b][h] = bcell[b][h] + 1;
        }
      }
    }
    if (stager) {
      e_shell[tid] = shell_t;
      e_sc[tid] = cscale[shell_t];
      e_c0[tid] = coef[(size_t)shell_t * P.namp];
    }
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < AT; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int lr = wm * (TMV / 2) + a * 32 + (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5), row = m0 + lr;
      if (row >= M) continue;
      if (EXPAND) {
        const int shell = e_shell[lr];
        const double sc = e_sc[lr];
        const double c0 = e_c0[lr];   // l = 0 coefficient, FP64
        const auto dst = gmem(phi + (size_t)shell * P.ncell);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if (!bok[b]) continue;
          // rep block: even + odd parts; its mirror: even - odd (once parked,
          // acco holds the even sums and acc the odd ones)
          const double x0 = (double)acc[a][b][r], x1 = EXPAND ? (double)acco[a][b][r] : 0.0;
          const double ev = parked ? x1 : x0, od = parked ? x0 : 0.0;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            if (h == 1 && !bmir[b]) break;
            const double v = c0 * bt0[b] + sc * (h ? ev - od : ev + od);
            if (C.rect != nullptr) {
              if (bnj[b][h] == 1 && bnk[b][h] == 1) {
                __builtin_nontemporal_store(v, &dst[bcell[b][h]]);   // the potential streams out
              } else {
                for (int j = 0; j < bnj[b][h]; ++j)
                  for (int k = 0; k < bnk[b][h]; ++k) dst[bcell[b][h] + j * P.nphi + k] = v;
              }
            } else {
              for (int e = bcell[b][h]; e < bnj[b][h]; ++e) dst[mem[e]] = v;
            }
          }
        }
      } else {
        // FP32 partial sums (the accumulator type; the row scale is a power of two)
        const float sc = (float)e_sc[lr];
        const auto out = part + ((size_t)split * M + row) * P.namp_m;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int col = n0 + wn * 64 + b * 32 + (lane & 31);
          if (col < N) out[col] = sc * acc[a][b][r];
        }
      }
    }
}

// LDS of one contraction tile (u4 slots): two stages of X and Y chunks.
template <int KIND>
constexpr int split_lds_slots() {
  return 2 * (2 * Split<KIND>::planes) * (TMMAX + TN);
}

// One workgroup item of a moment (EXPAND = false) or expansion contraction
// launch: workgroup J.local of field J.f, LDS of split_lds_slots<KIND>() slots.
// LDS stage layout: [chunk][row], chunk = 2 plane + k half, with the rows of
// each chunk rotated within aligned groups of 8 by sig[chunk].  16-byte LDS
// accesses are served 8 lanes at a time over 128 bytes of banks, so a group
// of 8 lanes is conflict-free when it touches 8 distinct 16-byte slots mod 8.
// MFMA fragment reads (8 consecutive rows of one chunk) are, for any
// rotation; the rotations are chosen so that the stores, where 8 consecutive
// lanes hold consecutive (row, chunk) pairs of the global slab, are too.
template <int KIND, bool EXPAND>
__device__ __forceinline__ void split_item(const BatchDev &B, const Job &J, u4 *lds) {
  const PlanDev &P = J.P;
  int c = 0;
  if (EXPAND) {
    while (c + 1 < P.nclasses && J.local >= ld_const(&P.classes[c + 1].wg_exp_begin)) ++c;
  } else {
    while (c + 1 < P.nclasses && J.local >= ld_const(&P.classes[c + 1].wg_mom_begin)) ++c;
  }
  const ClassDev C = ld_const(P.classes + c);
  const int local = J.local - (EXPAND ? C.wg_exp_begin : C.wg_mom_begin);
  if ((EXPAND ? P.tm_exp : P.tm_mom) == 64)
    gemm_tile<KIND, EXPAND, 64>(B, P, C, J.io.phi, local, lds);
  else
    gemm_tile<KIND, EXPAND, 128>(B, P, C, J.io.phi, local, lds);
  if (EXPAND) stamp_done(B, J.f);
}

}  // namespace
}  // namespace mpole
