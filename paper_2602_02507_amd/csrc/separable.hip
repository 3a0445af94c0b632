// Separable form of the two angular contractions, in FP64.
//
// The cell-averaged kernels factor: <A_lma>_jk = <P~_lm>_j <trig_ma>_k, and
// so do the solid angles, dOmega_jk = dcos_j dphi_k (Eqs. AngularKernel_c /
// AngularKernel_s averaged over a theta-phi cell).  Within a shell:
//
//   moment   A_lma  = sum_j [4 pi G dcos_j P~_lm(j)] F_ma(j),
//            F_ma(j) = sum_k [dphi_k <trig_ma>_k] rhohat_jk,
//   potential Phihat_jk = sum_ma <trig_ma>_k G_ma(j),
//            G_ma(j) = sum_l C_lma P~_lm(j),
//
// where rhohat is the density with every coarsening block replaced by its
// solid-angle weighted mean, and a block's potential is the solid-angle
// weighted mean of Phihat over its members.  Both identities are exact
// (a reordering of the sums of Eq. AngularMomentsDiscrete and Eq. Solution
// with block-mean kernels), so this path computes the same result as the
// dense contractions over blocks x modes, in about (2L+1) nphi + (L+1)^2
// instead of 2 (L+1)^2 nphi multiply-adds per (shell, theta row).
//
// Trig modes are t = 0 (m = 0), 2m-1 (cos m phi), 2m (sin m phi), padded to
// tpad (a multiple of 16).  Per-shell intermediates are t-major:
// F[i][t][j], G[i][t][j].  Steps and kernels:
//   source     block means of rho on the rows that hold a merged block
//   phi_anal   F_i[t][j]  = sum_k TW[t][k] rhohat_i[j][k]       (batched over shells)
//   theta_anal A[i][lma]  = sum_j F[i][t][j] PW_m[j][l-m]       (batched over t)
//   (radial scans and coefficients as in the dense path)
//   theta_syn  G[i][t][j] = sum_l C[i][lma] PT_m[l-m][j]         (batched over t)
//   phi_syn    Phihat_i[j][k] = sum_t G_i[t][j] TT[t][k]        (batched over shells)
//   block_mean block means of Phihat written to the members of merged blocks
// All four contractions run on v_mfma_f64_16x16x4 with the 64 x 64 tiles
// and conflict-free LDS layouts of the dense FP64 kernels.
#include <algorithm>
#include <type_traits>

#include "device_util.h"
#include "f64_mma.h"

namespace mpole {
namespace {

using namespace f64mma;

// Operand of a tile.  K-contiguous operands (staged [row][k]) give the start
// of a row, row(b, r), and the offset of element k in it, off(k);
// row-contiguous operands (staged [k][row]) give the column start col(b, r)
// and the stride between k, ld.  Callers pass clamped, in-range rows and k;
// the tile zeroes elements outside (rows, K).
struct RowsK {   // element (r, k) at base + b*bs + r*ld + k
  const double *base;
  long bs, ld;
  __device__ const double *row(int b, int r) const { return base + b * bs + (long)r * ld; }
  __device__ int off(int k) const { return k; }
};
struct KRows {   // element (r, k) at base + b*bs + k*ld + r
  const double *base;
  long bs, ld;
  __device__ const double *col(int b, int r) const { return base + b * bs + r; }
};
// The density rows of shell b: rho, or the block means for rows with a merged block.
struct SourceRows {
  const double *rho, *shat;
  const uint8_t *alt;   // [nr][ntheta]
  int ntheta, nphi;
  long ncell;
  __device__ const double *row(int b, int r) const {
    const long o = b * ncell + (long)r * nphi;
    return (alt != nullptr && alt[(long)b * ntheta + r]) ? shat + o : rho + o;
  }
  __device__ int off(int k) const { return k; }
};
// Coefficients C[i][l m a] of one trig mode t = (m, a), element k at l = k + m.
struct CoefGather {
  const double *coef;
  int namp, m, a;
  __device__ const double *row(int, int r) const { return coef + (long)r * namp; }
  __device__ int off(int k) const {
    const int l = k + m;
    return m == 0 ? l * l : l * l + 2 * m - 1 + a;
  }
};

__device__ inline void trig_mode(int t, int &m, int &a) {
  m = (t + 1) >> 1;
  a = (t > 0 && (t & 1) == 0) ? 1 : 0;
}

// Loader of one operand of a 64-row tile (rows r0.., R rows in all, K deep):
// K-contiguous operands move 4 consecutive k of row tid/4, row-contiguous
// ones rows tid%16 + 16 e of k-row tid/16.  Row addresses are resolved once.
template <bool KC, class OP>
struct TileLoader {
  const double *p[4];
  long ld;
  int r[4], kk[4];
  OP op;
  __device__ TileLoader(const OP &o, int b, int r0, int R, long ld_) : ld(ld_), op(o) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      r[e] = KC ? (tid >> 2) : (tid & 15) + 16 * e;
      kk[e] = KC ? (tid & 3) * 4 + e : (tid >> 4);
      const int rc = min(r0 + r[e], max(R, 1) - 1);
      if constexpr (KC) p[e] = o.row(b, rc);
      else p[e] = o.col(b, rc);
    }
  }
  __device__ double load(int e, int k0, int K) const {
    const int k = min(k0 + kk[e], K - 1);
    if constexpr (KC) return *gmem(p[e] + op.off(k));
    else return *gmem(p[e] + (long)k * ld);
  }
  __device__ void store(double *S, int e, double v, bool ok) const {
    const double x = ok ? v : 0.0;
    if (KC) S[r[e] * RK + kk[e]] = x; else S[kk[e] * KR + r[e]] = x;
  }
};

// Accumulates the M x N x K product of one 64 x 64 output tile (rows m0..,
// columns n0..) of batch b into acc.
struct NoHook {
  __device__ void operator()(const double *, const double *, int) const {}
};

template <bool A_KC, bool B_KC, class OA, class OB, class HOOK = NoHook>
__device__ __forceinline__ void tile_product(const OA &A, long a_ld, const OB &B, long b_ld, int b, int M, int N,
                                             int K, int m0, int n0, d4 acc[2][2], double (*As)[STAGE],
                                             double (*Bs)[STAGE], const HOOK &hook = HOOK()) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;
  const TileLoader<A_KC, OA> la(A, b, m0, M, a_ld);
  const TileLoader<B_KC, OB> lb(B, b, n0, N, b_ld);
  double av[4], bv[4];
  auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      av[e] = la.load(e, k0, K);
      bv[e] = lb.load(e, k0, K);
    }
  };
  auto store = [&](int buf, int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      la.store(As[buf], e, av[e], m0 + la.r[e] < M && k0 + la.kk[e] < K);
      lb.store(Bs[buf], e, bv[e], n0 + lb.r[e] < N && k0 + lb.kk[e] < K);
    }
  };
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};
  const int nk = (K + BK - 1) / BK;
  load(0);
  store(0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) load((kt + 1) * BK);
    hook(As[cur], Bs[cur], kt * BK);   // the stage in LDS, before it is overwritten
    mfma_stage<A_KC, B_KC>(As[cur], Bs[cur], wm, wn, lane, acc);
    if (more) store(cur ^ 1, (kt + 1) * BK);
    __syncthreads();
  }
}

// tile_product for long K (the phi analysis, K = nphi): two register sets, so
// each load has two stages of MFMA work to hide behind.  For the short K of
// the other contractions the extra stage of an odd count and the deeper
// prologue cost more than they hide.
template <bool A_KC, bool B_KC, class OA, class OB, class HOOK = NoHook>
__device__ __forceinline__ void tile_product_deep(const OA &A, long a_ld, const OB &B, long b_ld, int b, int M,
                                                  int N, int K, int m0, int n0, d4 acc[2][2], double (*As)[STAGE],
                                                  double (*Bs)[STAGE], const HOOK &hook = HOOK()) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;
  const TileLoader<A_KC, OA> la(A, b, m0, M, a_ld);
  const TileLoader<B_KC, OB> lb(B, b, n0, N, b_ld);
  // two register sets: the loads of stage k + 2 are issued before stage k is
  // computed and reach LDS after stage k + 1 is, with no branch in the loop
  // (an odd stage count computes one more stage, of zeros: every element
  // past K is zeroed at the store, and loads past K read its last column).
  // The selects that zero elements outside (rows, K) stay behind each
  // stage's MFMAs (the scheduler would otherwise hoist them, and the wait for
  // their loads, to the top of the stage).
  double a0[4], b0[4], a1[4], b1[4];
  auto load = [&](double (&av)[4], double (&bv)[4], int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      av[e] = la.load(e, k0, K);
      bv[e] = lb.load(e, k0, K);
    }
  };
  auto store = [&](const double (&av)[4], const double (&bv)[4], int buf, int k0) __attribute__((always_inline)) {
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      la.store(As[buf], e, av[e], m0 + la.r[e] < M && k0 + la.kk[e] < K);
      lb.store(Bs[buf], e, bv[e], n0 + lb.r[e] < N && k0 + lb.kk[e] < K);
    }
  };
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};
  const int nk = (K + BK - 1) / BK;
  load(a0, b0, 0);
  load(a1, b1, BK);
  store(a0, b0, 0, 0);
  __syncthreads();
  load(a0, b0, 2 * BK);
  for (int kt = 0; kt < nk; kt += 2) {
    // stage kt in LDS 0; set 1 holds stage kt + 1, set 0 stage kt + 2
    hook(As[0], Bs[0], kt * BK);   // the stage in LDS, before it is overwritten
    mfma_stage<A_KC, B_KC>(As[0], Bs[0], wm, wn, lane, acc);
    store(a1, b1, 1, (kt + 1) * BK);
    __syncthreads();
    load(a1, b1, (kt + 3) * BK);
    hook(As[1], Bs[1], (kt + 1) * BK);
    mfma_stage<A_KC, B_KC>(As[1], Bs[1], wm, wn, lane, acc);
    store(a0, b0, 0, (kt + 2) * BK);
    __syncthreads();
    load(a0, b0, (kt + 4) * BK);
  }
}

// Row and column of accumulator element (t, u, r) of this lane.
__device__ inline void acc_pos(int t, int u, int r, int &row, int &col) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  row = (w & 1) * 32 + t * 16 + 4 * r + (lane >> 4);
  col = (w >> 1) * 32 + u * 16 + (lane & 15);
}

// ---- per-solve kernels ------------------------------------------------------

// Block means of rho for every block on a row that holds a merged block.
// Block means of the density on rows holding a merged block: thread x of
// shell blockIdx.y takes the x-th block of its class's source list (blocks
// of more than kLargeBlock cells are left to launch_large).
__global__ __launch_bounds__(256) void k_sep_source(PlanDev P, SepDev S, const double *rho_) {
  const int i = blockIdx.y;
  const int c = ld_const(P.shell_class + i);
  const SepClass L = ld_const(S.cls + c);
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= L.n_src) return;
  const ClassDev C = ld_const(P.classes + c);
  const int b = gmem(L.src)[x];
  double num = 0.0, den = 0.0;
  block_wsum(C, S.dom, rho_ + (long)i * P.ncell, P.nphi, b, num, den);
  block_fill(C, S.shat + (long)i * P.ncell, P.nphi, b, num / den);
}

// F_i[t][j] = sum_k TW[t][k] rhohat_i[j][k]; grid (t tiles x j tiles, shells).
// The MFMA tiles cover t = 1 .. 2L (cos and sin of m >= 1: 2L rows, whole
// 64-row tiles for even L); the m = 0 row, a dphi-weighted row sum, is added
// from the density stages in LDS by the workgroups of the first t tile.
struct RowSum {
  const double *dphi;   // TW row 0: dphi_k
  int j0, nphi;
  double *sum;          // this thread's running sum (row tid, tid < 64)
  __device__ void operator()(const double *, const double *Bs, int k0) const {
    if (threadIdx.x >= BN) return;
    double s = *sum;
    // dphi through scalar loads (the address is uniform): a vector load here
    // would wait behind the tile's staged operand loads
    if (k0 + BK <= nphi) {   // a whole stage: one batch of scalar loads
#pragma unroll
      for (int kk = 0; kk < BK; ++kk) s += ld_const(dphi + k0 + kk) * Bs[threadIdx.x * RK + kk];
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; ++kk)
        if (k0 + kk < nphi) s += ld_const(dphi + k0 + kk) * Bs[threadIdx.x * RK + kk];
    }
    *sum = s;
  }
};

__global__ __launch_bounds__(NTHREADS) void k_sep_phi_anal(PlanDev P, SepDev S, const double *rho) {
  __shared__ double As[2][STAGE], Bs[2][STAGE];
  const int i = blockIdx.y;
  const int ntj = (P.ntheta + BN - 1) / BN;
  const int m0 = (blockIdx.x / ntj) * BM, n0 = (blockIdx.x % ntj) * BN;
  const int M = 2 * P.lmax;   // t = 1 .. 2L
  const RowsK A{S.tw + P.nphi, 0, P.nphi};
  const SourceRows Bop{rho, S.shat, S.rowalt, P.ntheta, P.nphi, (long)P.ncell};
  d4 acc[2][2];
  double rs = 0.0;
  const auto F = gmem(S.f) + (long)i * S.tpad * P.ntheta;
  if (m0 == 0) {
    tile_product_deep<true, true>(A, 0, Bop, 0, i, M, P.ntheta, P.nphi, m0, n0, acc, As, Bs,
                                  RowSum{S.tw, n0, P.nphi, &rs});
    if (threadIdx.x < BN && n0 + (int)threadIdx.x < P.ntheta) F[n0 + threadIdx.x] = rs;
  } else {
    tile_product_deep<true, true>(A, 0, Bop, 0, i, M, P.ntheta, P.nphi, m0, n0, acc, As, Bs);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row, col;
        acc_pos(t, u, r, row, col);
        row += m0;
        col += n0;
        if (row < M && col < P.ntheta) F[(long)(row + 1) * P.ntheta + col] = acc[t][u][r];
      }
}

// A[i][l m a] = sum_j F[i][t][j] PW_m[j][l-m]; grid (shell tiles x l tiles, t).
__global__ __launch_bounds__(NTHREADS) void k_sep_theta_anal(PlanDev P, SepDev S, double *ang_out) {
  __shared__ double As[2][STAGE], Bs[2][STAGE];
  const int t = blockIdx.y;
  int m, a;
  trig_mode(t, m, a);
  const int L1 = P.lmax + 1, N = L1 - m;
  const int ntl = (L1 + BN - 1) / BN;
  const int m0 = (blockIdx.x / ntl) * BM, n0 = (blockIdx.x % ntl) * BN;
  if (n0 >= N) return;
  const RowsK A{S.f + (long)t * P.ntheta, 0, (long)S.tpad * P.ntheta};
  const KRows Bop{S.pw + (long)m * P.ntheta * L1, 0, L1};
  d4 acc[2][2];
  tile_product<true, false>(A, 0, Bop, Bop.ld, 0, P.nr, N, P.ntheta, m0, n0, acc, As, Bs);
#pragma unroll
  for (int tt = 0; tt < 2; ++tt)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row, col;
        acc_pos(tt, u, r, row, col);
        row += m0;
        col += n0;
        if (row >= P.nr || col >= N) continue;
        const int l = col + m;
        const int n = m == 0 ? l * l : l * l + 2 * m - 1 + a;
        gmem(P.ang)[(long)row * P.namp + n] = acc[tt][u][r];
        if (ang_out != nullptr) gmem(ang_out)[(long)row * P.nam + n] = acc[tt][u][r];
      }
}

// G[i][t][j] = sum_l C[i][l m a] PT_m[l-m][j]; grid (shell tiles x j tiles, t).
__global__ __launch_bounds__(NTHREADS) void k_sep_theta_syn(PlanDev P, SepDev S) {
  __shared__ double As[2][STAGE], Bs[2][STAGE];
  const int t = blockIdx.y;
  int m, a;
  trig_mode(t, m, a);
  const int L1 = P.lmax + 1, K = L1 - m;
  const int ntj = (P.ntheta + BN - 1) / BN;
  const int m0 = (blockIdx.x / ntj) * BM, n0 = (blockIdx.x % ntj) * BN;
  const CoefGather A{P.coef, P.namp, m, a};
  const KRows Bop{S.pt + (long)m * L1 * P.ntheta, 0, P.ntheta};
  d4 acc[2][2];
  tile_product<true, false>(A, 0, Bop, Bop.ld, 0, P.nr, P.ntheta, K, m0, n0, acc, As, Bs);
#pragma unroll
  for (int tt = 0; tt < 2; ++tt)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row, col;
        acc_pos(tt, u, r, row, col);
        row += m0;
        col += n0;
        if (row < P.nr && col < P.ntheta)
          gmem(S.g)[((long)row * S.tpad + t) * P.ntheta + col] = acc[tt][u][r];
      }
}

// ---- theta transforms with every operand load issued at once ---------------
//
// The tiled kernels above stream K through LDS 16 at a time, one stage
// ahead; the theta contractions are short (K = ntheta or L + 1 - m) and their
// grids hold about two workgroups per CU, so each stage's load latency is
// exposed in turn.  For the common shapes the forms below issue all of a
// workgroup's operand loads at once instead.  A workgroup takes 64 shells of
// one trig mode t, a wavefront 16 of them (the rows of its MFMA tiles); the
// per-shell operand goes straight into MFMA operand registers (loaded in the
// lane order of the f64 16x16x4 operand, no LDS), the per-mode table is
// staged once in LDS for the workgroup's four wavefronts.  The results are
// the same sums as the tiled kernels', in another order.

// k step s of a 128-wide chunk takes j = 8 (s / 2) + 2 q + s % 2 from the
// lanes of k slot q: every 16-byte load of the F rows then covers 64
// contiguous bytes per row.  Row s * 4 + q of the staged PW_m holds that j.
__device__ inline int anal_row(int jj) { return ((jj >> 3) * 2 + (jj & 1)) * 4 + ((jj >> 1) & 3); }

// A[i][l m a] = sum_j F[i][t][j] PW_m[j][l-m] for ntheta = 128 KCH and
// L + 1 - m <= 16 NB; grid (shell tiles of 64, t).  Lane (r, q) = (l % 16,
// l / 16) holds F[i0 + r][t][128 c + 8 h + 2 q + e] for h < 16, e < 2
// (16-byte loads), the A operands of k steps 2 h + e of chunk c.  Blocks of
// 16 columns wholly past L - m are skipped.
template <int KCH, int NB>
__global__ __launch_bounds__(NTHREADS) void k_sep_theta_anal_w(PlanDev P, SepDev S, double *ang_out) {
  extern __shared__ double Bs[];   // [KCH * 128][NB * 16 + 1]
  constexpr int PITCH = NB * 16 + 1, NBC = NB * 16, NLD = KCH * 128 * NBC / NTHREADS;
  static_assert(KCH * 128 * NBC % NTHREADS == 0, "table staging");
  const int t = blockIdx.y;
  int m, a;
  trig_mode(t, m, a);
  const int L1 = P.lmax + 1, N = L1 - m;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int r = lane & 15, q = lane >> 4;
  const int i0 = blockIdx.x * 64 + 16 * w;
  // PW_m[j][n], n = l - m (columns past N read column N - 1 and stage 0)
  const auto pw = gmem(S.pw + (long)m * P.ntheta * L1);
  double bv[NLD];
#pragma unroll
  for (int e = 0; e < NLD; ++e) {
    const int x = (int)threadIdx.x + NTHREADS * e, j = x / NBC, n = x % NBC;
    bv[e] = pw[(long)j * L1 + min(n, N - 1)];
  }
  // F[i][t][.]: this lane's 32 k of each chunk (shells past nr read shell nr - 1)
  typedef double dv2 __attribute__((ext_vector_type(2)));
  const dv2 *frow = reinterpret_cast<const dv2 *>(S.f + ((long)min(i0 + r, P.nr - 1) * S.tpad + t) * P.ntheta) + q;
  dv2 av[KCH][16];
#pragma unroll
  for (int c = 0; c < KCH; ++c)
#pragma unroll
    for (int h = 0; h < 16; ++h) av[c][h] = *gmem(frow + 64 * c + 4 * h);
#pragma unroll
  for (int e = 0; e < NLD; ++e) {
    const int x = (int)threadIdx.x + NTHREADS * e, j = x / NBC, n = x % NBC;
    Bs[((j >> 7) * 128 + anal_row(j & 127)) * PITCH + n] = n < N ? bv[e] : 0.0;
  }
  __syncthreads();
  d4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = d4{0.0, 0.0, 0.0, 0.0};
  // the live column blocks, chosen once per workgroup (a branch between
  // MFMAs would cost the hazard padding at every block boundary)
  auto product = [&](auto nlive) __attribute__((always_inline)) {
    constexpr int NL = decltype(nlive)::value;
#pragma unroll
    for (int c = 0; c < KCH; ++c)
#pragma unroll
      for (int s = 0; s < 32; ++s) {
        const double x = av[c][s >> 1][s & 1];
        const double *brow = Bs + (c * 128 + 4 * s + q) * PITCH + r;
#pragma unroll
        for (int nb = 0; nb < NL; ++nb) acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, brow[16 * nb], acc[nb], 0, 0, 0);
      }
  };
  if (NB >= 3 && N > 32) product(std::integral_constant<int, NB>{});
  else if (NB >= 2 && N > 16) product(std::integral_constant<int, (NB >= 2 ? 2 : NB)>{});
  else product(std::integral_constant<int, 1>{});
  // element (4 rr + q, r) of block nb: shell i0 + 4 rr + q, l = m + 16 nb + r
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int i = i0 + 4 * rr + q, lp = 16 * nb + r;
      if (i >= P.nr || lp >= N) continue;
      const int l = lp + m;
      const int n = m == 0 ? l * l : l * l + 2 * m - 1 + a;
      gmem(P.ang)[(long)i * P.namp + n] = acc[nb][rr];
      if (ang_out != nullptr) gmem(ang_out)[(long)i * P.nam + n] = acc[nb][rr];
    }
}

// G[i][t][j] = sum_l C[i][l m a] PT_m[l-m][j] for L + 1 <= 4 KS, over a
// column tile of 128 theta rows; grid (shell tiles of 64 x column tiles, t).
// Lane (r, q) holds the coefficient of l = m + 4 s + q of shell i0 + r for
// each k step s (a gather from the coefficient rows; l past L reads l = L,
// whose staged PT row is zero); PT_m is staged once, rows k < 4 KS.
template <int KS>
__global__ __launch_bounds__(NTHREADS) void k_sep_theta_syn_w(PlanDev P, SepDev S) {
  extern __shared__ double Bs[];   // [4 KS][128 + 1]
  constexpr int PITCH = 129, NLD = 4 * KS * 128 / NTHREADS;
  static_assert(4 * KS * 128 % NTHREADS == 0, "table staging");
  const int t = blockIdx.y;
  int m, a;
  trig_mode(t, m, a);
  const int L1 = P.lmax + 1, K = L1 - m;
  const int nct = P.ntheta / 128;
  const int i0w = (blockIdx.x / nct) * 64, j0 = (blockIdx.x % nct) * 128;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int r = lane & 15, q = lane >> 4;
  const int i0 = i0w + 16 * w;
  // PT_m[k][j0 + jj] (rows k >= K stage 0)
  const auto pt = gmem(S.pt + (long)m * L1 * P.ntheta + j0);
  double bv[NLD];
#pragma unroll
  for (int e = 0; e < NLD; ++e) {
    const int x = (int)threadIdx.x + NTHREADS * e, k = x >> 7, jj = x & 127;
    bv[e] = pt[(long)min(k, K - 1) * P.ntheta + jj];
  }
  const auto crow = gmem(P.coef + (long)min(i0 + r, P.nr - 1) * P.namp);
  double av[KS];
#pragma unroll
  for (int s2 = 0; s2 < KS; ++s2) {
    const int l = min(m + 4 * s2 + q, P.lmax);
    av[s2] = crow[m == 0 ? l * l : l * l + 2 * m - 1 + a];
  }
#pragma unroll
  for (int e = 0; e < NLD; ++e) {
    const int x = (int)threadIdx.x + NTHREADS * e, k = x >> 7, jj = x & 127;
    Bs[k * PITCH + jj] = k < K ? bv[e] : 0.0;
  }
  __syncthreads();
  d4 acc[8];
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) acc[nb] = d4{0.0, 0.0, 0.0, 0.0};
  // the k steps up to L - m, their count chosen once per workgroup (a branch
  // between MFMAs would cost the hazard padding at every block boundary)
  auto product = [&](auto nsteps) __attribute__((always_inline)) {
    constexpr int NS = decltype(nsteps)::value;
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      const double *brow = Bs + (4 * s2 + q) * PITCH + r;
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s2], brow[16 * nb], acc[nb], 0, 0, 0);
    }
  };
  using std::integral_constant;
  switch (min((K + 3) / 4, KS)) {
    case 1: product(integral_constant<int, 1>{}); break;
    case 2: product(integral_constant<int, 2 <= KS ? 2 : 1>{}); break;
    case 3: product(integral_constant<int, 3 <= KS ? 3 : 1>{}); break;
    case 4: product(integral_constant<int, 4 <= KS ? 4 : 1>{}); break;
    case 5: product(integral_constant<int, 5 <= KS ? 5 : 1>{}); break;
    case 6: product(integral_constant<int, 6 <= KS ? 6 : 1>{}); break;
    case 7: product(integral_constant<int, 7 <= KS ? 7 : 1>{}); break;
    case 8: product(integral_constant<int, 8 <= KS ? 8 : 1>{}); break;
    default: product(integral_constant<int, KS>{}); break;
  }
  // element (4 rr + q, r) of block nb: shell i0 + 4 rr + q, theta row j0 + 16 nb + r
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int i = i0 + 4 * rr + q;
    if (i >= P.nr) continue;
    const auto grow = gmem(S.g + ((long)i * S.tpad + t) * P.ntheta + j0 + r);
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) grow[16 * nb] = acc[nb][rr];
  }
}

// Phihat_i[j][k] = sum_t G_i[t][j] TT[t][k] for 2L + 1 <= 4 KS, ntheta and
// nphi multiples of 64; grid (j tiles x k tiles of 64, shells).  The same
// scheme as the theta forms above: lane (r, q) holds G_i[4 s + q][j0 + r]
// for each k step s (16 consecutive theta rows per trig mode; modes past 2L
// read mode 2L, whose staged TT row is zero, since G's padding modes are
// never written), and the 64 columns of TT the workgroup needs are staged
// once in LDS.
template <int KS>
__global__ __launch_bounds__(NTHREADS) void k_sep_phi_syn_w(PlanDev P, SepDev S, double *phi) {
  extern __shared__ double Bs[];   // [4 KS][64 + 1]
  constexpr int PITCH = 65, NLD = 4 * KS * 64 / NTHREADS;
  static_assert(4 * KS * 64 % NTHREADS == 0, "table staging");
  const int i = blockIdx.y;
  const int ntk = P.nphi / 64;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int r = lane & 15, q = lane >> 4;
  const int j0 = (blockIdx.x / ntk) * 64 + 16 * w, k0 = (blockIdx.x % ntk) * 64;
  const int K = 2 * P.lmax + 1;
  // TT[t][k0 + kk] (TT follows TW; its rows 2L < t < tpad are zero, and
  // tpad, a multiple of 16, exceeds the odd 2L + 1: rows past it read the
  // last, zero row)
  const auto tt = gmem(S.tw + (long)S.tpad * P.nphi + k0);
  double bv[NLD];
#pragma unroll
  for (int e = 0; e < NLD; ++e) {
    const int x = (int)threadIdx.x + NTHREADS * e, t = x >> 6, kk = x & 63;
    bv[e] = tt[(long)min(t, S.tpad - 1) * P.nphi + kk];
  }
  const auto g = gmem(S.g + (long)i * S.tpad * P.ntheta + j0 + r);
  double av[KS];
#pragma unroll
  for (int s2 = 0; s2 < KS; ++s2) av[s2] = g[(long)min(4 * s2 + q, K - 1) * P.ntheta];
#pragma unroll
  for (int e = 0; e < NLD; ++e) {
    const int x = (int)threadIdx.x + NTHREADS * e, t = x >> 6, kk = x & 63;
    Bs[t * PITCH + kk] = bv[e];
  }
  __syncthreads();
  d4 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s2 = 0; s2 < KS; ++s2) {
    const double *brow = Bs + (4 * s2 + q) * PITCH + r;
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s2], brow[16 * nb], acc[nb], 0, 0, 0);
  }
  // element (4 rr + q, r) of block nb: theta row j0 + 4 rr + q, phi column k0 + 16 nb + r
  const auto out = gmem(phi) + (long)i * P.ncell + k0 + r;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
      __builtin_nontemporal_store(acc[nb][rr], &out[(long)(j0 + 4 * rr + q) * P.nphi + 16 * nb]);   // streamed out
}

// Phihat_i[j][k] = sum_t G_i[t][j] TT[t][k]; grid (j tiles x k tiles, shells).
__global__ __launch_bounds__(NTHREADS) void k_sep_phi_syn(PlanDev P, SepDev S, double *phi) {
  __shared__ double As[2][STAGE], Bs[2][STAGE];
  const int i = blockIdx.y;
  const int ntk = (P.nphi + BN - 1) / BN;
  const int m0 = (blockIdx.x / ntk) * BM, n0 = (blockIdx.x % ntk) * BN;
  const KRows A{S.g, (long)S.tpad * P.ntheta, P.ntheta};
  const KRows Bop{S.tw + (long)S.tpad * P.nphi, 0, P.nphi};   // TT follows TW
  d4 acc[2][2];
  // K = the 2L + 1 trig modes G holds (its padding rows are never written)
  tile_product<false, false>(A, A.ld, Bop, Bop.ld, i, P.ntheta, P.nphi, 2 * P.lmax + 1, m0, n0, acc, As, Bs);
  const auto out = gmem(phi) + (long)i * P.ncell;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row, col;
        acc_pos(t, u, r, row, col);
        row += m0;
        col += n0;
        if (row < P.ntheta && col < P.nphi)
          __builtin_nontemporal_store(acc[t][u][r], &out[(long)row * P.nphi + col]);   // the potential streams out
      }
}

// Solid-angle weighted mean of Phihat over each merged block of shell
// blockIdx.y, written to its members (large blocks: launch_large).
__global__ __launch_bounds__(256) void k_sep_block_mean(PlanDev P, SepDev S, double *phi_) {
  const int i = blockIdx.y;
  const int c = ld_const(P.shell_class + i);
  const SepClass L = ld_const(S.cls + c);
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= L.n_avg) return;
  const ClassDev C = ld_const(P.classes + c);
  const int b = gmem(L.avg)[x];
  double num = 0.0, den = 0.0;
  block_wsum(C, S.dom, phi_ + (long)i * P.ncell, P.nphi, b, num, den);
  block_fill(C, phi_ + (long)i * P.ncell, P.nphi, b, num / den);
}

// ---- bind-time tables -------------------------------------------------------

// TW[t][k] = dphi_k <trig_t>_k and TT[t][k] = <trig_t>_k (zero for t > 2L);
// PW[m][j][l-m] = 4 pi G dcos_j <P~_lm>_j and PT[m][l-m][j] = <P~_lm>_j (zero for l > L).
__global__ __launch_bounds__(256) void k_sep_tables(PlanDev P, SepDev S) {
  const long x = (long)blockIdx.x * 256 + threadIdx.x;
  const int L1 = P.lmax + 1;
  const long ntw = (long)S.tpad * P.nphi;
  const long npw = (long)L1 * P.ntheta * L1;
  if (x < ntw) {
    const int t = (int)(x / P.nphi), k = (int)(x % P.nphi);
    int m, a;
    trig_mode(t, m, a);
    const double v = (t < 2 * L1 - 1) ? P.trig[(long)k * 2 * L1 + 2 * m + a] : 0.0;
    S.tw[x] = (P.phi_edges[k + 1] - P.phi_edges[k]) * v;
    S.tw[ntw + x] = v;
    return;
  }
  const long y = x - ntw;
  if (y >= 2 * npw) return;
  const int nplm = L1 * (L1 + 1) / 2;
  if (y < npw) {   // PW[m][j][lp]
    const int m = (int)(y / ((long)P.ntheta * L1));
    const int j = (int)(y / L1 % P.ntheta), lp = (int)(y % L1);
    const int l = lp + m;
    double v = 0.0;
    if (l <= P.lmax)
      v = 4.0 * kPi * P.G * cos_diff(P.theta_edges[j], P.theta_edges[j + 1]) *
          P.pavg[(long)j * nplm + l * (l + 1) / 2 + m];
    S.pw[y] = v;
  } else {         // PT[m][lp][j]
    const long z = y - npw;
    const int m = (int)(z / ((long)L1 * P.ntheta));
    const int lp = (int)(z / P.ntheta % L1), j = (int)(z % P.ntheta);
    const int l = lp + m;
    S.pt[z] = (l <= P.lmax) ? P.pavg[(long)j * nplm + l * (l + 1) / 2 + m] : 0.0;
  }
}

inline unsigned tiles(int n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_sep_tables(const PlanDev &P, const SepDev &S, hipStream_t s) {
  const long L1 = P.lmax + 1;
  const long n = (long)S.tpad * P.nphi + 2 * L1 * P.ntheta * L1;
  hipLaunchKernelGGL(k_sep_tables, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, S);
  return hipGetLastError();
}

hipError_t launch_sep_source(const PlanDev &P, const SepDev &S, const double *rho, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (S.max_src > 0) {
    hipLaunchKernelGGL(k_sep_source, dim3(tiles(S.max_src, 256), P.nr), dim3(256), 0, s, P, S, rho);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = launch_bands(P, kBandMean, rho, S.shat, s, S.fuse_nk);
  if (e == hipSuccess) e = launch_large(P, kLargeMean, rho, S.shat, s);
  return e;
}

hipError_t launch_sep_phi_anal(const PlanDev &P, const SepDev &S, const double *rho, hipStream_t s) {
  hipLaunchKernelGGL(k_sep_phi_anal, dim3(tiles(std::max(2 * P.lmax, 1), BM) * tiles(P.ntheta, BN), P.nr),
                     dim3(NTHREADS), 0, s, P, S, rho);
  return hipGetLastError();
}

hipError_t launch_sep_theta_anal(const PlanDev &P, const SepDev &S, double *ang_out, hipStream_t s) {
  // whole-K form: ntheta 128 with L + 1 <= 48, or 256 with L + 1 <= 16 (the
  // staged table within 64 KB of LDS)
  const int nb = (P.lmax + 16) / 16;
  const dim3 grid(tiles(P.nr, 64), 2 * P.lmax + 1);
  auto lds = [&](int kch, int n) { return (size_t)kch * 128 * (n * 16 + 1) * sizeof(double); };
  if (P.ntheta == 128 && nb == 1)
    hipLaunchKernelGGL((k_sep_theta_anal_w<1, 1>), grid, dim3(NTHREADS), lds(1, 1), s, P, S, ang_out);
  else if (P.ntheta == 128 && nb == 2)
    hipLaunchKernelGGL((k_sep_theta_anal_w<1, 2>), grid, dim3(NTHREADS), lds(1, 2), s, P, S, ang_out);
  else if (P.ntheta == 128 && nb == 3)
    hipLaunchKernelGGL((k_sep_theta_anal_w<1, 3>), grid, dim3(NTHREADS), lds(1, 3), s, P, S, ang_out);
  else if (P.ntheta == 256 && nb == 1)
    hipLaunchKernelGGL((k_sep_theta_anal_w<2, 1>), grid, dim3(NTHREADS), lds(2, 1), s, P, S, ang_out);
  else
    hipLaunchKernelGGL(k_sep_theta_anal, dim3(tiles(P.nr, BM) * tiles(P.lmax + 1, BN), 2 * P.lmax + 1),
                       dim3(NTHREADS), 0, s, P, S, ang_out);
  return hipGetLastError();
}

hipError_t launch_sep_theta_syn(const PlanDev &P, const SepDev &S, hipStream_t s) {
  // whole-K form: ntheta a multiple of 128 and L + 1 <= 36 (at most 9 k steps)
  const int ks = (P.lmax + 4) / 4;
  const dim3 grid(tiles(P.nr, 64) * (unsigned)(P.ntheta / 128), 2 * P.lmax + 1);
  auto lds = [&](int k) { return (size_t)4 * k * 129 * sizeof(double); };
  if (P.ntheta % 128 != 0 || ks > 9)
    hipLaunchKernelGGL(k_sep_theta_syn, dim3(tiles(P.nr, BM) * tiles(P.ntheta, BN), 2 * P.lmax + 1),
                       dim3(NTHREADS), 0, s, P, S);
  else if (ks <= 2)
    hipLaunchKernelGGL((k_sep_theta_syn_w<2>), grid, dim3(NTHREADS), lds(2), s, P, S);
  else if (ks <= 3)
    hipLaunchKernelGGL((k_sep_theta_syn_w<3>), grid, dim3(NTHREADS), lds(3), s, P, S);
  else if (ks <= 5)
    hipLaunchKernelGGL((k_sep_theta_syn_w<5>), grid, dim3(NTHREADS), lds(5), s, P, S);
  else
    hipLaunchKernelGGL((k_sep_theta_syn_w<9>), grid, dim3(NTHREADS), lds(9), s, P, S);
  return hipGetLastError();
}

hipError_t launch_sep_phi_syn(const PlanDev &P, const SepDev &S, double *phi, hipStream_t s) {
  // whole-K form: 64-row, 64-column tiles and 2L + 1 <= 100 (the staged TT
  // columns within 64 KB of LDS)
  const int ks = (2 * P.lmax + 4) / 4;
  const dim3 grid((unsigned)((P.ntheta / 64) * (P.nphi / 64)), (unsigned)P.nr);
  auto lds = [&](int k) { return (size_t)4 * k * 65 * sizeof(double); };
  if (P.ntheta % 64 != 0 || P.nphi % 64 != 0 || ks > 25)
    hipLaunchKernelGGL(k_sep_phi_syn, dim3(tiles(P.ntheta, BM) * tiles(P.nphi, BN), P.nr), dim3(NTHREADS), 0, s, P,
                       S, phi);
  else if (ks <= 5)
    hipLaunchKernelGGL((k_sep_phi_syn_w<5>), grid, dim3(NTHREADS), lds(5), s, P, S, phi);
  else if (ks <= 9)
    hipLaunchKernelGGL((k_sep_phi_syn_w<9>), grid, dim3(NTHREADS), lds(9), s, P, S, phi);
  else if (ks <= 13)
    hipLaunchKernelGGL((k_sep_phi_syn_w<13>), grid, dim3(NTHREADS), lds(13), s, P, S, phi);
  else if (ks <= 17)
    hipLaunchKernelGGL((k_sep_phi_syn_w<17>), grid, dim3(NTHREADS), lds(17), s, P, S, phi);
  else
    hipLaunchKernelGGL((k_sep_phi_syn_w<25>), grid, dim3(NTHREADS), lds(25), s, P, S, phi);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? launch_sep_block_means(P, S, phi, s) : e;
}

hipError_t launch_sep_block_means(const PlanDev &P, const SepDev &S, double *phi, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (S.max_avg > 0) {
    hipLaunchKernelGGL(k_sep_block_mean, dim3(tiles(S.max_avg, 256), P.nr), dim3(256), 0, s, P, S, phi);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = launch_bands(P, kBandMean, phi, phi, s, S.fuse_nk);
  if (e == hipSuccess) e = launch_large(P, kLargeMean, phi, phi, s);
  return e;
}

}  // namespace mpole
