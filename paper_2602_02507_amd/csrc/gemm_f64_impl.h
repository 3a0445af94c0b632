// Device code of the two angular contractions of the solve in FP64 on MFMA (v_mfma_f64_16x16x4):
//
//   moment:  A[i][n]   = sum_b  P[i][b] T[b][n]   (Eq. AngularMomentsDiscrete;
//            P = dOmega_b S_ib packed per class, T = block-mean kernels)
//   expand:  Phi[i][b] = sum_n  C[i][n] T[b][n]   (Eq. Solution at the shell
//            centre with the assembled coefficients C)
//
// Both read the same kernel table T[b][n] (mode index fastest) staged through
// LDS; the moment contraction reads it row-wise (k = b), the expansion
// column-wise (k = n).  Tiles are 64 x 64 per workgroup of four waves, each
// wave owning a 32 x 32 corner as 2 x 2 MFMA 16x16 tiles; K advances 16 per
// LDS stage, double-buffered with register prefetch of the next stage.
//
// LDS layouts are chosen so that neither the stores of a stage nor the MFMA
// operand reads conflict on banks (8-byte accesses are served 16 lanes at a
// time over 128 bytes of banks): an operand whose rows are loaded with k
// contiguous is kept row-major with a pitch of BK + 1 doubles (16 lanes
// reading one k of 16 rows hit 16 distinct bank pairs, and a thread's 4
// consecutive k land in distinct banks from its 15 neighbours'); the moment
// table, loaded with n contiguous, is kept k-major and each lane loads and
// stores the n columns 16 apart, so 16 lanes always touch 128 contiguous
// bytes.
//
// The moment contraction is skinny (M = shells, N = modes, K = blocks up to
// ~1e5), so K is split across workgroups; each split writes its own FP64
// partial and a separate pass sums them in a fixed order (deterministic, no
// atomics).  Workgroup ids are remapped so that each XCD (8 per MI355X, with
// private L2) receives a contiguous run of tiles that share table panels.
//
// f64 MFMA 16x16x4 lane layout on gfx950 (checked on the device): lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; result element (i, j) sits in
// lane 16*(i%4) + j, accumulator register i/4.
#pragma once
#include "device_util.h"
#include "f64_mma.h"

namespace mpole {
namespace {


using namespace f64mma;

// 4 consecutive doubles from a 32-byte aligned address.  The load is
// unconditional (callers pass a valid address for rows outside the operand
// and zero them when storing to LDS), so the compiler need not wait for it
// before the store.
__device__ inline void load4(const double *p, double v[4]) {
  typedef double g2 __attribute__((ext_vector_type(2)));
  const auto q = gmem(reinterpret_cast<const g2 *>(p));
  const g2 x = q[0], y = q[1];
  v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
}

// LDS of one FP64 contraction tile, in doubles: two stages of each operand.
constexpr int F64_LDS = 4 * STAGE;

// Workgroup J.local of field J.f of a moment contraction launch.
__device__ __forceinline__ void moment_f64_item(const BatchDev &B, const Job &J, double *lds) {
  double(*As)[STAGE] = reinterpret_cast<double(*)[STAGE]>(lds);               // packed source, [row][k]
  double(*Bs)[STAGE] = reinterpret_cast<double(*)[STAGE]>(lds + 2 * STAGE);   // table, [k][n]
  const PlanDev &P = J.P;
  int c = 0;
  while (c + 1 < P.nclasses && J.local >= ld_const(&P.classes[c + 1].wg_mom_begin)) ++c;
  const ClassDev C = ld_const(P.classes + c);
  const int local = J.local - C.wg_mom_begin;
  const int mt = local % C.m_tiles_mom;
  const int rest = local / C.m_tiles_mom;
  const int nt = rest % C.n_tiles_mom;
  const int split = rest / C.n_tiles_mom;
  const int m0 = mt * BM, n0 = nt * BN;
  const int kbeg = split * C.kchunk;
  const int kend = min(kbeg + C.kchunk, C.npair_pad);
  // K = pairs, N = moment mode columns; odd columns contract the odd packed source
  const int nrows = C.nrows, ldp = C.npair_pad, namp = P.namp_m;
  const double *__restrict__ Pk = n0 >= P.odd_m0 ? C.pack_o : C.pack;
  const double *__restrict__ T = C.tm;

  const int tid = item_tid(), lane = tid & 63, w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;
  // loader roles: A rows (4 consecutive k of row ar); B row bk, columns
  // bn + 16 e (e < 4).  namp is a multiple of 16, so the column test is
  // uniform over each group of 16 lanes.
  const int ar = tid >> 2, ak = (tid & 3) * 4;
  const int bk = tid >> 4, bn = tid & 15;
  const bool a_ok = (m0 + ar) < nrows;
  bool b_ok[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) b_ok[e] = (n0 + bn + 16 * e) < namp;
  const double *abase = Pk + (size_t)(a_ok ? m0 + ar : 0) * ldp + ak;
  const auto bbase = gmem(T) + (size_t)bk * namp;

  d4 acc[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};

  double av[4], bv[4];
  auto load_b = [&](int k) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) bv[e] = bbase[(size_t)k * namp + (b_ok[e] ? n0 + bn + 16 * e : 0)];
  };
  auto store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) As[buf][ar * RK + ak + e] = a_ok ? av[e] : 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) Bs[buf][bk * KR + bn + 16 * e] = b_ok[e] ? bv[e] : 0.0;
  };
  const int nk = (kend - kbeg) / BK;
  if (nk > 0) {
    load4(abase + kbeg, av);
    load_b(kbeg);
    store(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) {
      const int k = kbeg + (kt + 1) * BK;
      load4(abase + k, av);
      load_b(k);
    }
    mfma_stage<true, false>(As[cur], Bs[cur], wm, wn, lane, acc);
    if (more) store(cur ^ 1);
    __syncthreads();
  }

  const auto out = gmem(C.partial) + (size_t)split * nrows * namp;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + t * 16 + 4 * r + (lane >> 4);
        const int col = n0 + wn * 32 + u * 16 + (lane & 15);
        if (row < nrows && col < namp) out[(size_t)row * namp + col] = acc[t][u][r];
      }
}

// Workgroup J.local of field J.f of an expansion contraction launch.
__device__ __forceinline__ void expand_f64_item(const BatchDev &B, const Job &J, double *lds) {
  double(*As)[STAGE] = reinterpret_cast<double(*)[STAGE]>(lds);               // coefficients, [shell row][k]
  double(*Bs)[STAGE] = reinterpret_cast<double(*)[STAGE]>(lds + 2 * STAGE);   // table, [pair][k]
  const PlanDev &P = J.P;
  double *__restrict__ phi = J.io.phi;
  int c = 0;
  while (c + 1 < P.nclasses && J.local >= ld_const(&P.classes[c + 1].wg_exp_begin)) ++c;
  const ClassDev C = ld_const(P.classes + c);
  const int local = J.local - C.wg_exp_begin;
  const int mt = local % C.m_tiles_exp;
  const int nt = local / C.m_tiles_exp;
  const int m0 = mt * BM, n0 = nt * BN;
  // N = pairs, K = expansion mode columns (even columns, then odd ones)
  const int nrows = C.nrows, namp = P.namp_e;
  const double *__restrict__ T = C.te;
  const double *__restrict__ coef = P.coef_e;

  const int tid = item_tid(), lane = tid & 63, w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;
  // both operands are rows with the mode index contiguous: 64 rows x 16 modes
  const int lr = tid >> 2, lk = (tid & 3) * 4;
  const bool a_ok = (m0 + lr) < nrows;
  const int shell_a = a_ok ? gmem(C.rows)[m0 + lr] : 0;
  const bool b_ok = (n0 + lr) < C.npair_pad;
  const double *arow = coef + (size_t)shell_a * namp;
  const double *brow = T + (size_t)(b_ok ? n0 + lr : 0) * namp;

  // even-column and odd-column sums (the odd ones stay 0 when unfolded)
  d4 acc[2][2], acco[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = acco[t][u] = d4{0.0, 0.0, 0.0, 0.0};

  double av[4], bv[4];
  const int nk = namp / BK, nk_even = P.odd_e0 / BK;
  load4(arow + lk, av);
  load4(brow + lk, bv);
#pragma unroll
  for (int e = 0; e < 4; ++e) As[0][lr * RK + lk + e] = a_ok ? av[e] : 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) Bs[0][lr * RK + lk + e] = b_ok ? bv[e] : 0.0;
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) {
      const int k = (kt + 1) * BK;
      load4(arow + k + lk, av);
      load4(brow + k + lk, bv);
    }
    if (kt < nk_even)
      mfma_stage<true, true>(As[cur], Bs[cur], wm, wn, lane, acc);
    else
      mfma_stage<true, true>(As[cur], Bs[cur], wm, wn, lane, acco);
    if (more) {
#pragma unroll
      for (int e = 0; e < 4; ++e) As[cur ^ 1][lr * RK + lk + e] = a_ok ? av[e] : 0.0;
#pragma unroll
      for (int e = 0; e < 4; ++e) Bs[cur ^ 1][lr * RK + lk + e] = b_ok ? bv[e] : 0.0;
    }
    __syncthreads();
  }

  // epilogue: a pair's potentials go to every member cell of its blocks,
  // even + odd sums to the rep block, even - odd to its mirror.  This lane's
  // two pairs are resolved once for all its rows ([.][0] rep, [.][1] mirror;
  // rect: first cell and extent; CSR: member range in bcell .. bnj); a block
  // of more than kLargeBlock cells only gets its first cell here,
  // launch_large copies it.
  bool bok[2], bmir[2] = {false, false};
  int bcell[2][2] = {}, bnj[2][2] = {}, bnk[2][2] = {};
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = n0 + wn * 32 + u * 16 + (lane & 15);
    bok[u] = q < C.npair;
    if (!bok[u]) continue;
    const i2v pr = gmem(reinterpret_cast<const i2v *>(C.pairs))[q];
    bmir[u] = pr.y != pr.x;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int b = h ? pr.y : pr.x;
      if (C.rect != nullptr) {
        const auto rect = gmem(reinterpret_cast<const int *>(C.rect));   // (j0, k0, nj, nk) per block
        bcell[u][h] = rect[4 * b] * P.nphi + rect[4 * b + 1];
        bnj[u][h] = rect[4 * b + 2];
        bnk[u][h] = rect[4 * b + 3];
        // first cell only: launch_large (past kLargeBlock cells) or the
        // broadcast phase (merged blocks of a banded class) writes the rest
        if (bnj[u][h] * bnk[u][h] > kLargeBlock || C.bands != nullptr) bnj[u][h] = bnk[u][h] = 1;
      } else {
        bcell[u][h] = gmem(C.moff)[b];
        bnj[u][h] = gmem(C.moff)[b + 1];
        if (bnj[u][h] - bcell[u][h] > kLargeBlock) bnj[u][h] = bcell[u][h] + 1;
      }
    }
  }
  const auto mem = gmem(C.mem);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m0 + wm * 32 + t * 16 + 4 * r + (lane >> 4);
      if (row >= nrows) continue;
      const auto dst = gmem(phi) + (size_t)gmem(C.rows)[row] * P.ncell;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (!bok[u]) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h == 1 && !bmir[u]) break;
          const double v = h ? acc[t][u][r] - acco[t][u][r] : acc[t][u][r] + acco[t][u][r];
          if (C.rect != nullptr) {
            if (bnj[u][h] == 1 && bnk[u][h] == 1) {
              __builtin_nontemporal_store(v, &dst[bcell[u][h]]);   // the potential streams out
            } else {
              for (int j = 0; j < bnj[u][h]; ++j)
                for (int k = 0; k < bnk[u][h]; ++k) dst[bcell[u][h] + j * P.nphi + k] = v;
            }
          } else {
            for (int e = bcell[u][h]; e < bnj[u][h]; ++e) dst[mem[e]] = v;
          }
        }
      }
    }
  stamp_done(B, J.f);
}

}  // namespace
}  // namespace mpole
