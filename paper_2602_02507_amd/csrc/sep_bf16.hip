// Separable form with BF16 x3 phi transforms.
//
// The separable path (the cell-averaged kernels and solid angles factor in
// theta and phi, Eqs. AngularKernel_c / AngularKernel_s averaged over a cell)
// computes, per shell i and theta row j,
//   analysis   F_i[t][j]      = sum_k TW[t][k] rhohat_i[j][k],
//   synthesis  Phihat_i[j][k] = sum_t G_i[t][j] TT[t][k],
// with t the trig modes (t = 0: m = 0; 2m-1 / 2m: cos / sin m phi).  Here
// the m >= 1 rows of both transforms run on BF16 MFMA with every operand
// written as hi + mid + lo bfloat16 planes (split8 below) and the six
// products hi.hi, hi.mid, mid.hi, hi.lo, lo.hi, mid.mid accumulated in FP32;
// the m = 0 row (the density's dphi-weighted row sum, and the potential's
// m = 0 term), which carries the monopole, stays FP64.  The theta transforms
// and the radial sums are the FP64 kernels of the separable path.
//
// MFMA v_mfma_f32_16x16x32_bf16 (16-row tiles, 32-deep K steps: many short
// wavefronts to keep enough density loads in flight).  Each lane of a
// wavefront loads exactly the 8 values of its own density or G fragment and
// splits them in registers:
//   analysis:  the density fragment of lane l is row j0 + l % 16, phi cells
//              32 ks + 8 (l / 16) .. +7 (64 contiguous bytes; the four lanes
//              of a row cover its 256-byte run of the K step); the
//              trig-weight fragments come from a bind-time table in fragment
//              order, through LDS (one copy per workgroup and K step).
//   synthesis: the G fragment of lane l is theta row j0 + l % 16 at modes
//              1 + 32 ks + 8 (l / 16) .. +7 (each load coalesced across 16
//              rows); the trig fragments come from a table in fragment order.
// 16x16x32 lane layout (gfx950, checked on the device): lane l supplies
// X[l%16][8(l/16)..+7] and Y[l%16][same k]; result register r holds
// out[4(l/16) + r][l%16] of out[m][n] = sum_k X[m][k] Y[n][k].
//
// Both transforms are HBM-bound: the analysis reads the density once (8 B per
// cell) and the synthesis writes the potential once (8 B per cell).
#include <algorithm>

#include "device_util.h"
#include "split_util.h"

namespace mpole {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ inline f4 mma(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// hi, mid, lo bfloat16 planes of 8 FP64 values, packed two per dword
// (element e in the low half of dword e / 2 when e is even).  Each value is
// rounded to FP32 first (relative error 2^-24, the precision of the three
// planes together); the FP32 value is then exactly hi + mid + lo: hi is its
// nearest bfloat16, the remainders are exact FP32 differences, and the last
// one has at most 8 significant bits.
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
__device__ inline void split8(const double (&v)[8], u4 (&p)[3]) {
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    float x0 = (float)v[2 * d], x1 = (float)v[2 * d + 1];
    // keep the two roundings apart (FP64 -> FP32, then FP32 -> BF16)
    asm volatile("" : "+v"(x0), "+v"(x1));
    const f2 x = {x0, x1};
    const bf2 h = __builtin_convertvector(x, bf2);
    const f2 r = x - __builtin_convertvector(h, f2);
    const bf2 m = __builtin_convertvector(r, bf2);
    const f2 t = r - __builtin_convertvector(m, f2);
    p[0][d] = __builtin_bit_cast(uint32_t, h);
    p[1][d] = __builtin_bit_cast(uint32_t, m);
    p[2][d] = __builtin_bit_cast(uint32_t, __builtin_convertvector(t, bf2));
  }
}

// the six kept products of two split fragments (the other three are below
// 2^-24 of the product)
__device__ inline f4 mma6(const u4 (&a)[3], const u4 (&b)[3], f4 c) {
  c = mma(a[0], b[0], c);
  c = mma(a[0], b[1], c);
  c = mma(a[1], b[0], c);
  c = mma(a[0], b[2], c);
  c = mma(a[2], b[0], c);
  c = mma(a[1], b[1], c);
  return c;
}

__device__ inline u4 frag(const uint32_t *table, long entry, int lane) {
  return *(const __attribute__((address_space(1))) u4 *)(table + (entry * 64 + lane) * 4);
}

// ---- bind-time fragment tables ---------------------------------------------

// One thread per (K step, tile, lane) entry of either table: its 8 values,
// split, into the three planes.
__global__ __launch_bounds__(256) void k_sep_split_tables(PlanDev P, SepDev S) {
  const long x = (long)blockIdx.x * 256 + threadIdx.x;
  const long na = (long)S.ks_a * S.mt_a * 64, ns = (long)S.ks_s * S.nt_s * 64;
  const int tmax = 2 * P.lmax;
  const double *tw = S.tw, *tt = S.tw + (long)S.tpad * P.nphi;
  double v[8];
  uint32_t *dst;
  long entry;
  int lane;
  if (x < na) {
    lane = (int)(x % 64);
    const long e2 = x / 64;   // ks * mt_a + mt
    const int ks = (int)(e2 / S.mt_a), mt = (int)(e2 % S.mt_a);
    const int t = 1 + 16 * mt + lane % 16;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 32 * ks + 8 * (lane / 16) + e;
      v[e] = (t <= tmax && k < P.nphi) ? tw[(long)t * P.nphi + k] : 0.0;
    }
    dst = const_cast<uint32_t *>(S.twf);
    entry = e2 * 3;
  } else if (x < na + ns) {
    const long y = x - na;
    lane = (int)(y % 64);
    const long e2 = y / 64;   // ks * nt_s + nt
    const int ks = (int)(e2 / S.nt_s), nt = (int)(e2 % S.nt_s);
    const int k = 16 * nt + lane % 16;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int t = 1 + 32 * ks + 8 * (lane / 16) + e;
      v[e] = (t <= tmax && k < P.nphi) ? tt[(long)t * P.nphi + k] : 0.0;
    }
    dst = const_cast<uint32_t *>(S.ttf);
    entry = e2 * 3;
  } else {
    return;
  }
  u4 p[3];
  split8(v, p);
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int d = 0; d < 4; ++d) dst[((entry + q) * 64 + lane) * 4 + d] = p[q][d];
}

// ---- per-solve kernels ------------------------------------------------------

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) dv2 *gdv2;

// 8 consecutive doubles from a 16-byte aligned global address
__device__ inline void load8(const double *p, double (&v)[8]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const dv2 d = *(gdv2)(p + 2 * e);
    v[2 * e] = d[0];
    v[2 * e + 1] = d[1];
  }
}

// Analysis: a wavefront per (shell blockIdx.y, 16 theta rows), all m >= 1
// modes (MT tiles of 16); 4 wavefronts per workgroup on adjacent row tiles of
// one shell.  The workgroup copies each K step's trig-weight fragments
// (MT x 3 KB) to LDS once, one step ahead in registers, and its wavefronts
// read them from there.  Rows past the mesh read its row j0 and store nothing
// (each output row depends on its own density row only); a row tile wholly
// past the mesh only helps with the copies.  Full steps (32 cells inside the
// row) load without guards; a last partial step loads element by element.
// From 5 row tiles up (2L > 64) the compiler would settle for two waves per
// SIMD; three fit without spills and run the L = 64 analysis 8 % faster.
template <int MT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MT >= 5 ? 3 : 1))) void k_sep_phi_anal_bf16(
    PlanDev P, SepDev S, const double *rho, int rho16) {
  constexpr int NF = MT > 0 ? MT * 3 * 64 : 64;   // fragment entries (16 bytes) per K step
  constexpr int CP = (NF + 255) / 256;             // copied per thread
  __shared__ u4 As[2][NF];
  const int lane = threadIdx.x & 63, quad = lane >> 4;
  const int i = blockIdx.y;
  const int j0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  const bool tile_in = j0 < P.ntheta;   // wavefront-uniform
  const int j = j0 + (lane & 15);
  const bool jin = j < P.ntheta;
  const int jr = jin ? j : (tile_in ? j0 : 0);
  const long o = (long)i * P.ncell + (long)jr * P.nphi;
  // row code: 0 the density, 1 the block means (shat), 2 + log2(nk / 2)
  // one-row blocks of nk cells, averaged here in registers
  const int code = S.rowalt != nullptr ? S.rowalt[(long)i * P.ntheta + jr] : 0;
  const int fnk = code >= 2 ? 1 << (code - 1) : 1;
  const double *row = (code == 1 ? S.shat : rho) + o + 8 * quad;   // this lane's cells of step 0
  const double *dphi = S.tw + 8 * quad;                      // TW row 0: dphi_k
  const int np = P.nphi, nks = S.ks_a;
  const bool vec = rho16 && (np & 1) == 0;   // rows start 16-byte aligned

  f4 acc[MT > 0 ? MT : 1];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = f4{};
  double rs = 0.0;   // FP64 row sum of dphi_k rho over this lane's cells

  auto load = [&](double (&v)[8], double (&d)[8], int ks) __attribute__((always_inline)) {
    if (32 * ks + 32 <= np) {
      if (vec) {
        load8(row + 32 * ks, v);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = *gmem(row + 32 * ks + e);
      }
      load8(dphi + 32 * ks, d);
    } else {   // the partial last step
      const int k0 = 32 * ks + 8 * quad;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool in = k0 + e < np;
        v[e] = in ? *gmem(row + 32 * ks + e) : 0.0;
        d[e] = in ? *gmem(dphi + 32 * ks + e) : 0.0;
      }
    }
  };
  u4 fr[CP];   // this thread's share of a step's fragments, one step ahead
  auto fetch = [&](int ks) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < CP; ++c) {
      const int e = threadIdx.x + 256 * c;
      if (MT > 0 && e < NF) fr[c] = frag(S.twf, (long)ks * (NF / 64) + e / 64, e % 64);
    }
  };
  auto put = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < CP; ++c) {
      const int e = threadIdx.x + 256 * c;
      if (MT > 0 && e < NF) As[buf][e] = fr[c];
    }
  };
  double v[8], d[8], vn[8], dn[8];
  if (nks > 0) {
    fetch(0);
    if (tile_in) load(v, d, 0);
    put(0);
  }
  __syncthreads();
  for (int ks = 0; ks < nks; ++ks) {
    const bool more = ks + 1 < nks;
    if (more) {
      fetch(ks + 1);
      if (tile_in) load(vn, dn, ks + 1);
    }
    if (tile_in) {
      if (fnk > 1) {   // dphi-weighted means of the lane's aligned groups of fnk cells
        double g[8], dw[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          g[e] = d[e] * v[e];
          dw[e] = d[e];
        }
        // butterfly within the groups: every cell ends with its group's sums
#pragma unroll
        for (int m = 1; m < 8; m <<= 1)
          if (m < fnk) {
            double tg[8], tw[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              tg[e] = g[e] + g[e ^ m];
              tw[e] = dw[e] + dw[e ^ m];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              g[e] = tg[e];
              dw[e] = tw[e];
            }
          }
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = dw[e] > 0.0 ? g[e] / dw[e] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) rs += d[e] * v[e];
      if constexpr (MT > 0) {
        u4 b[3];
        split8(v, b);
        const u4 *st = As[ks & 1];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          u4 a[3];
#pragma unroll
          for (int q = 0; q < 3; ++q) a[q] = st[(m * 3 + q) * 64 + lane];
          acc[m] = mma6(a, b, acc[m]);
        }
      }
    }
    if (more) {
      put((ks + 1) & 1);   // that buffer was last read in step ks - 1
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        v[e] = vn[e];
        d[e] = dn[e];
      }
    }
    __syncthreads();
  }
  if (!tile_in) return;
  // a row's four quarters sit in lanes l, l + 16, l + 32, l + 48
  rs += __shfl_xor(rs, 16, 64);
  rs += __shfl_xor(rs, 32, 64);
  const auto F = gmem(S.f) + (long)i * S.tpad * P.ntheta;
  if (!jin) return;
  if (quad == 0) F[j] = rs;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = 1 + 16 * m + 4 * quad + r;
      if (t <= 2 * P.lmax) F[(long)t * P.ntheta + j] = (double)acc[m][r];
    }
}

// Synthesis: a wavefront per (shell blockIdx.y, 16 theta rows, a chunk of
// ntw phi tiles of 16); Phihat = G[0][j] TT[0][k] (FP64) + the m >= 1 sum.
// The wavefront loads and splits its rows' NKS K steps of G once, then walks
// its phi tiles two at a time, so the stores of one pair drain while the
// next is computed.  Rows past the
// mesh read its last row and store nothing.
template <int NKS>
__global__ __launch_bounds__(256) void k_sep_phi_syn_bf16(PlanDev P, SepDev S, double *phi, int ntw) {
  const int lane = threadIdx.x & 63, quad = lane >> 4;
  const int i = blockIdx.y;
  const int j0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (j0 >= P.ntheta) return;   // wavefront-uniform; no barrier
  const int nt0 = blockIdx.z * ntw, nt1 = min(nt0 + ntw, S.nt_s);
  const int ja = min(j0 + (lane & 15), P.ntheta - 1);   // this lane's G row
  const double *G = S.g + (long)i * S.tpad * P.ntheta;
  const int tmax = 2 * P.lmax;

  // the split G fragments of every K step (modes 1 + 32 ks + 8 quad .. +7)
  u4 a[NKS > 0 ? NKS : 1][3];
  {
    double v[NKS > 0 ? NKS : 1][8];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int t = 1 + 32 * ks + 8 * quad + e;
        v[ks][e] = t <= tmax ? *gmem(G + (long)t * P.ntheta + ja) : 0.0;
      }
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) split8(v[ks], a[ks]);
  }
  // m = 0 term of this lane's four output rows
  double g0[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) g0[r] = *gmem(G + min(j0 + 4 * quad + r, P.ntheta - 1));
  const auto tt0 = gmem(S.tw) + (long)S.tpad * P.nphi;   // TT row 0 (m = 0)
  const auto out = gmem(phi) + (long)i * P.ncell;

  auto load_b = [&](u4 (&b)[NKS > 0 ? NKS : 1][3], int nt) __attribute__((always_inline)) {
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
      for (int q = 0; q < 3; ++q) b[ks][q] = frag(S.ttf, ((long)ks * S.nt_s + nt) * 3 + q, lane);
  };
  // rows of one-row blocks of fnk cells (row code 2 + log2(fnk / 2)) get the
  // dphi-weighted block means here, over the fnk adjacent lanes that hold
  // the block's cells; the shuffles run on every lane
  int fnk[4];
  bool any_fused = false;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int jj = min(j0 + 4 * quad + r, P.ntheta - 1);
    const int code = S.rowalt != nullptr ? S.rowalt[(long)i * P.ntheta + jj] : 0;
    fnk[r] = code >= 2 ? 1 << (code - 1) : 1;
    any_fused = any_fused || fnk[r] > 1;
  }
  any_fused = __any(any_fused);   // wavefront-uniform
  auto store = [&](f4 acc, int nt) __attribute__((always_inline)) {
    const int k = 16 * nt + (lane & 15);
    const bool kin = k < P.nphi;
    const double c0 = kin ? tt0[k] : 0.0;
    double y[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) y[r] = g0[r] * c0 + (double)acc[r];
    if (any_fused) {
      const double w = kin ? *gmem(S.tw + k) : 0.0;   // TW row 0: dphi_k
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double num = w * y[r], den = w;
#pragma unroll
        for (int m = 1; m < 8; m <<= 1) {
          const double pn = __shfl_xor(num, m, 64), pd = __shfl_xor(den, m, 64);
          if (m < fnk[r]) {
            num += pn;
            den += pd;
          }
        }
        if (fnk[r] > 1) y[r] = den > 0.0 ? num / den : 0.0;
      }
    }
    if (kin) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jj = j0 + 4 * quad + r;
        if (jj < P.ntheta) __builtin_nontemporal_store(y[r], &out[(long)jj * P.nphi + k]);   // streamed out
      }
    }
  };
  // two tiles at a time, each product sum split over two accumulators (the
  // leading and the small products): four independent MFMA chains
  u4 ba[NKS > 0 ? NKS : 1][3], bb[NKS > 0 ? NKS : 1][3];
  for (int nt = nt0; nt < nt1; nt += 2) {
    const int nu = min(nt + 1, nt1 - 1);   // a single last tile is computed twice, stored once
    load_b(ba, nt);
    load_b(bb, nu);
    f4 p0 = f4{}, q0 = f4{}, p1 = f4{}, q1 = f4{};
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const u4(&x)[3] = a[ks];
      p0 = mma(x[0], ba[ks][0], p0);
      q0 = mma(x[0], ba[ks][2], q0);
      p1 = mma(x[0], bb[ks][0], p1);
      q1 = mma(x[0], bb[ks][2], q1);
      p0 = mma(x[0], ba[ks][1], p0);
      q0 = mma(x[2], ba[ks][0], q0);
      p1 = mma(x[0], bb[ks][1], p1);
      q1 = mma(x[2], bb[ks][0], q1);
      p0 = mma(x[1], ba[ks][0], p0);
      q0 = mma(x[1], ba[ks][1], q0);
      p1 = mma(x[1], bb[ks][0], p1);
      q1 = mma(x[1], bb[ks][1], q1);
    }
    store(p0 + q0, nt);
    if (nu != nt) store(p1 + q1, nu);
  }
}

// ---- whole-tile forms --------------------------------------------------------
//
// Vector memory counters retire in issue order, loads and stores alike, so a
// wait for a load also waits for every load and store issued before it, and
// at a join of branches the compiler waits for the longest count any path
// needs.  The two forms below (the host picks them when the mesh has whole K
// steps and tiles) keep every load a wait is for ahead of the stores and
// other loads that need not finish, and their steady state has no branch
// around a memory access, so each wait covers exactly the loads it needs.

// Analysis on whole K steps (nphi a multiple of 32, at most kAnalFullPhi;
// 16-byte aligned rows): the density and trig-fragment loads of step ks + 1
// are issued before step ks is computed, into the other of two register sets
// (no copies between them); dphi, the same for every row, comes from an LDS
// copy of the row (dynamic LDS, nphi doubles).  Every wavefront runs the same
// step sequence (a row tile past the mesh computes on row 0 of the shell and
// stores nothing).  Same arithmetic, in the same order, as
// k_sep_phi_anal_bf16.
constexpr int kAnalFullPhi = 1024;
template <int MT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MT >= 5 ? 3 : 4))) void k_sep_phi_anal_bf16_full(
    PlanDev P, SepDev S, const double *rho) {
  constexpr int NF = MT > 0 ? MT * 3 * 64 : 64;   // fragment entries (16 bytes) per K step
  constexpr int CP = (NF + 255) / 256;             // copied per thread
  // rounded up to whole copies of 256 entries: every thread stores its
  // entries unconditionally (a guarded LDS store would leave the wait for its
  // load in a branch, and the next fetch into the same registers would wait
  // for all loads in flight); the entries past NF are never read
  __shared__ u4 As[2][CP * 256];
  extern __shared__ double Ds[];                   // TW row 0: dphi_k
  const int lane = threadIdx.x & 63, quad = lane >> 4;
  const int i = blockIdx.y;
  const int j0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  const bool tile_in = j0 < P.ntheta;   // wavefront-uniform
  const int j = j0 + (lane & 15);
  const bool jin = j < P.ntheta;
  const int jr = jin ? j : (tile_in ? j0 : 0);
  const long o = (long)i * P.ncell + (long)jr * P.nphi;
  const int code = S.rowalt != nullptr ? S.rowalt[(long)i * P.ntheta + jr] : 0;
  const int fnk = code >= 2 ? 1 << (code - 1) : 1;
  const double *row = (code == 1 ? S.shat : rho) + o + 8 * quad;   // this lane's cells of step 0
  const int nks = S.ks_a;                                    // >= 1
  for (int k = threadIdx.x; k < P.nphi; k += 256) Ds[k] = S.tw[k];   // made visible by the first barrier

  f4 acc[MT > 0 ? MT : 1];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = f4{};
  double rs = 0.0;

  auto load = [&](double (&v)[8], int ks) __attribute__((always_inline)) { load8(row + 32 * ks, v); };
  u4 fr[CP];
  auto fetch = [&](int ks) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < CP; ++c) {
      const int e = min((int)threadIdx.x + 256 * c, NF - 1);
      if (MT > 0) fr[c] = frag(S.twf, (long)ks * (NF / 64) + e / 64, e % 64);
    }
  };
  auto put = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < CP; ++c)
      if (MT > 0) As[buf][threadIdx.x + 256 * c] = fr[c];
  };
  auto step = [&](double (&v)[8], int ks) __attribute__((always_inline)) {
    double d[8];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      const double2 w = *reinterpret_cast<const double2 *>(Ds + 32 * ks + 8 * quad + e);
      d[e] = w.x;
      d[e + 1] = w.y;
    }
    if (fnk > 1) {   // dphi-weighted means of the lane's aligned groups of fnk cells
      double g[8], dw[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        g[e] = d[e] * v[e];
        dw[e] = d[e];
      }
#pragma unroll
      for (int m = 1; m < 8; m <<= 1)
        if (m < fnk) {
          double tg[8], tw[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            tg[e] = g[e] + g[e ^ m];
            tw[e] = dw[e] + dw[e ^ m];
          }
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            g[e] = tg[e];
            dw[e] = tw[e];
          }
        }
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = dw[e] > 0.0 ? g[e] / dw[e] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) rs += d[e] * v[e];
    if constexpr (MT > 0) {
      u4 b[3];
      split8(v, b);
      const u4 *st = As[ks & 1];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        u4 a[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) a[q] = st[(m * 3 + q) * 64 + lane];
        acc[m] = mma6(a, b, acc[m]);
      }
    }
  };
  double va[8], vb[8];
  fetch(0);
  load(va, 0);
  put(0);
  // drain the vector memory counter once: with nothing in flight on entry,
  // the loop head needs no wait for registers the prologue loaded
  __builtin_amdgcn_s_waitcnt(0x0F70);   // gfx9 encoding: vmcnt(0), expcnt and lgkmcnt left free
  __syncthreads();
  // step ks reads buffer ks & 1; the fragments of step ks + 1 go to the other
  // buffer, last read in step ks - 1 (past the barrier).  The last step
  // fetches its own data again into the unused buffer and registers.
  for (int ks = 0;; ks += 2) {
    const int k1 = min(ks + 1, nks - 1);
    fetch(k1);
    load(vb, k1);
    step(va, ks);
    put((ks + 1) & 1);
    __syncthreads();
    if (ks + 1 >= nks) break;
    const int k2 = min(ks + 2, nks - 1);
    fetch(k2);
    load(va, k2);
    step(vb, ks + 1);
    put(ks & 1);
    __syncthreads();
    if (ks + 2 >= nks) break;
  }
  if (!tile_in) return;
  rs += __shfl_xor(rs, 16, 64);
  rs += __shfl_xor(rs, 32, 64);
  const auto F = gmem(S.f) + (long)i * S.tpad * P.ntheta;
  if (!jin) return;
  if (quad == 0) F[j] = rs;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = 1 + 16 * m + 4 * quad + r;
      if (t <= 2 * P.lmax) F[(long)t * P.ntheta + j] = (double)acc[m][r];
    }
}

// Synthesis on whole tiles (nphi a multiple of 32, ntheta a multiple of 64,
// an even number of phi tiles per wavefront): a workgroup's four wavefronts
// (64 rows of one shell) share each tile pair's trig fragments and the TT row
// 0 and dphi values of its 32 cells through LDS, two buffers deep.  The
// loads of pair p + 1 are issued before pair p is computed and stored, and
// written to LDS after the stores without waiting for them; the G loads of the
// prologue are unconditional.  Same arithmetic, in the same order, as
// k_sep_phi_syn_bf16.
template <int NKS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NKS >= 3 ? 3 : 4))) void k_sep_phi_syn_bf16_full(PlanDev P, SepDev S, double *phi, int ntw) {
  constexpr int NE = 2 * (NKS > 0 ? NKS : 1) * 3 * 64;   // fragment entries (16 bytes) of a tile pair
  constexpr int CP = (NE + 255) / 256;                    // staged per thread
  __shared__ u4 Bs[2][NE];
  __shared__ double Cs[2][64];   // per pair: TT row 0 of its 32 cells, then their dphi
  const int lane = threadIdx.x & 63, quad = lane >> 4;
  const int i = blockIdx.y;
  const int j0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  const int nt0 = blockIdx.z * ntw, npairs = (min(nt0 + ntw, S.nt_s) - nt0) / 2;
  const int ja = j0 + (lane & 15);   // this lane's G row (every row is in the mesh)
  const int np = P.nphi;
  const double *G = S.g + (long)i * S.tpad * P.ntheta;
  const int tmax = 2 * P.lmax;

  u4 a[NKS > 0 ? NKS : 1][3];
  {
    double v[NKS > 0 ? NKS : 1][8];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int t = 1 + 32 * ks + 8 * quad + e;
        const double x = *gmem(G + (long)min(t, tmax) * P.ntheta + ja);
        v[ks][e] = t <= tmax ? x : 0.0;
      }
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) split8(v[ks], a[ks]);
  }
  double g0[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) g0[r] = *gmem(G + j0 + 4 * quad + r);
  int fnk[4];
  bool any_fused = false;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int code = S.rowalt != nullptr ? S.rowalt[(long)i * P.ntheta + j0 + 4 * quad + r] : 0;
    fnk[r] = code >= 2 ? 1 << (code - 1) : 1;
    any_fused = any_fused || fnk[r] > 1;
  }
  any_fused = __any(any_fused);   // wavefront-uniform
  const auto out = gmem(phi) + (long)i * P.ncell + (long)j0 * np;

  // staging: entry e = ((ks * 2 + tile) * 3 + plane) * 64 + lane of the pair
  u4 sb[CP];
  double sc;
  const int cx = threadIdx.x & 63;
  const double *cbase = cx < 32 ? S.tw + (long)S.tpad * np + cx : S.tw + (cx - 32);   // TT row 0 / TW row 0
  auto stage_load = [&](int nt) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < CP; ++c) {
      const int e = min((int)threadIdx.x + 256 * c, NE - 1);
      const int ln = e % 64, q = (e / 64) % 3, tt = (e / 192) % 2, ks = e / 384;
      sb[c] = frag(S.ttf, ((long)ks * S.nt_s + nt + tt) * 3 + q, ln);
    }
    sc = *gmem(cbase + 16 * nt);
  };
  auto stage_put = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < CP; ++c) {
      const int e = threadIdx.x + 256 * c;
      if (e < NE) Bs[buf][e] = sb[c];
    }
    if (threadIdx.x < 64) Cs[buf][threadIdx.x] = sc;
  };
  auto store = [&](f4 acc, int nt, int tt, int buf) __attribute__((always_inline)) {
    const int k = 16 * nt + (lane & 15);
    const double c0 = Cs[buf][16 * tt + (lane & 15)];
    double y[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) y[r] = g0[r] * c0 + (double)acc[r];
    if (any_fused) {
      const double w = Cs[buf][32 + 16 * tt + (lane & 15)];   // dphi_k
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double num = w * y[r], den = w;
#pragma unroll
        for (int m = 1; m < 8; m <<= 1) {
          const double pn = __shfl_xor(num, m, 64), pd = __shfl_xor(den, m, 64);
          if (m < fnk[r]) {
            num += pn;
            den += pd;
          }
        }
        if (fnk[r] > 1) y[r] = den > 0.0 ? num / den : 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) __builtin_nontemporal_store(y[r], &out[(long)(4 * quad + r) * np + k]);   // streamed out
  };

  stage_load(nt0);
  stage_put(0);
  __syncthreads();
  for (int p = 0; p < npairs; ++p) {
    const int buf = p & 1, nt = nt0 + 2 * p;
    stage_load(nt0 + 2 * min(p + 1, npairs - 1));   // the last pair loads itself again, unused
    f4 p0 = f4{}, q0 = f4{}, p1 = f4{}, q1 = f4{};
    const u4 *st = Bs[buf];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      u4 ba[3], bb[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        ba[q] = st[((ks * 2 + 0) * 3 + q) * 64 + lane];
        bb[q] = st[((ks * 2 + 1) * 3 + q) * 64 + lane];
      }
      const u4(&x)[3] = a[ks];
      p0 = mma(x[0], ba[0], p0);
      q0 = mma(x[0], ba[2], q0);
      p1 = mma(x[0], bb[0], p1);
      q1 = mma(x[0], bb[2], q1);
      p0 = mma(x[0], ba[1], p0);
      q0 = mma(x[2], ba[0], q0);
      p1 = mma(x[0], bb[1], p1);
      q1 = mma(x[2], bb[0], q1);
      p0 = mma(x[1], ba[0], p0);
      q0 = mma(x[1], ba[1], q0);
      p1 = mma(x[1], bb[0], p1);
      q1 = mma(x[1], bb[1], q1);
    }
    store(p0 + q0, nt, 0, buf);
    store(p1 + q1, nt + 1, 1, buf);
    stage_put(buf ^ 1);   // buffer buf ^ 1 was last read in pair p - 1, past the barrier
    __syncthreads();
  }
}

inline unsigned cdiv(long n, long d) { return (unsigned)((n + d - 1) / d); }

}  // namespace

hipError_t launch_sep_split_tables(const PlanDev &P, const SepDev &S, hipStream_t s) {
  const long n = ((long)S.ks_a * S.mt_a + (long)S.ks_s * S.nt_s) * 64;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sep_split_tables, dim3(cdiv(n, 256)), dim3(256), 0, s, P, S);
  return hipGetLastError();
}

hipError_t launch_sep_phi_anal_bf16(const PlanDev &P, const SepDev &S, const double *rho, hipStream_t s) {
  const dim3 grid(cdiv(cdiv(P.ntheta, 16), 4), (unsigned)P.nr);
  // 16-byte density loads need 16-byte aligned rows (the block-mean copy is)
  const int rho16 = ((uintptr_t)rho % 16) == 0;
  if (rho16 && P.nphi % 32 == 0 && P.nphi <= kAnalFullPhi) {
    const size_t lds = (size_t)P.nphi * sizeof(double);
    switch (S.mt_a) {
#define MPOLE_ANAL_FULL(MT) \
  case MT: hipLaunchKernelGGL(k_sep_phi_anal_bf16_full<MT>, grid, dim3(256), lds, s, P, S, rho); break;
      MPOLE_ANAL_FULL(0) MPOLE_ANAL_FULL(1) MPOLE_ANAL_FULL(2) MPOLE_ANAL_FULL(3) MPOLE_ANAL_FULL(4)
      MPOLE_ANAL_FULL(5) MPOLE_ANAL_FULL(6) MPOLE_ANAL_FULL(7) MPOLE_ANAL_FULL(8)
#undef MPOLE_ANAL_FULL
      default: return hipErrorInvalidValue;   // 2L <= 128
    }
    return hipGetLastError();
  }
  switch (S.mt_a) {
#define MPOLE_ANAL(MT) \
  case MT: hipLaunchKernelGGL(k_sep_phi_anal_bf16<MT>, grid, dim3(256), 0, s, P, S, rho, rho16); break;
    MPOLE_ANAL(0) MPOLE_ANAL(1) MPOLE_ANAL(2) MPOLE_ANAL(3) MPOLE_ANAL(4)
    MPOLE_ANAL(5) MPOLE_ANAL(6) MPOLE_ANAL(7) MPOLE_ANAL(8)
#undef MPOLE_ANAL
    default: return hipErrorInvalidValue;   // 2L <= 128
  }
  return hipGetLastError();
}

hipError_t launch_sep_phi_syn_bf16(const PlanDev &P, const SepDev &S, double *phi, hipStream_t s) {
  // all phi tiles of a row tile in one wavefront (G read once), unless that
  // leaves fewer than 4096 wavefronts
  const long rows = (long)cdiv(P.ntheta, 16) * P.nr;
  const int chunks = (int)std::min<long>(std::max<long>(1, (4096 + rows - 1) / rows), std::max(S.nt_s, 1));
  if (P.nphi % 32 == 0 && P.ntheta % 64 == 0) {
    // whole tile pairs per wavefront: an even chunk of the (even) tile count
    const int ntw = 2 * (int)cdiv(S.nt_s / 2, chunks);
    const dim3 grid(cdiv(cdiv(P.ntheta, 16), 4), (unsigned)P.nr, cdiv(S.nt_s, ntw));
    switch (S.ks_s) {
#define MPOLE_SYN_FULL(NKS) \
  case NKS: hipLaunchKernelGGL(k_sep_phi_syn_bf16_full<NKS>, grid, dim3(256), 0, s, P, S, phi, ntw); break;
      MPOLE_SYN_FULL(0) MPOLE_SYN_FULL(1) MPOLE_SYN_FULL(2) MPOLE_SYN_FULL(3) MPOLE_SYN_FULL(4)
#undef MPOLE_SYN_FULL
      default: return hipErrorInvalidValue;   // 2L <= 128
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? launch_sep_block_means(P, S, phi, s) : e;
  }
  const int ntw = (int)cdiv(S.nt_s, chunks);
  const dim3 grid(cdiv(cdiv(P.ntheta, 16), 4), (unsigned)P.nr, cdiv(S.nt_s, std::max(ntw, 1)));
  switch (S.ks_s) {
#define MPOLE_SYN(NKS) \
  case NKS: hipLaunchKernelGGL(k_sep_phi_syn_bf16<NKS>, grid, dim3(256), 0, s, P, S, phi, ntw); break;
    MPOLE_SYN(0) MPOLE_SYN(1) MPOLE_SYN(2) MPOLE_SYN(3) MPOLE_SYN(4)
#undef MPOLE_SYN
    default: return hipErrorInvalidValue;   // 2L <= 128
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? launch_sep_block_means(P, S, phi, s) : e;
}

}  // namespace mpole
