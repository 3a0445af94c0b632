// Radial part of the solve in FP64 (GenASiS II Sec. 2.2, the edge
// recurrences after Eq. Solution):
//
//   k_reduce  angular moments A[i][n] = fixed-order sum of the split-K
//             partials of the moment contraction (split precisions: plus the
//             FP64 term of the mean source density the packing removed, and
//             the FP64 monopole from the packing kernel)
//   k_scan    regular moments by outward integration, M^R_0 = 0,
//             M^R_{i+1} = M^R_i + JR_l(i) A[i][n]; irregular moments by
//             inward integration, M^I_nr = 0, M^I_i = M^I_{i+1} + JI_l(i) A[i][n];
//             centre values (M_i + M_{i+1})/2 and the coefficients of Eq.
//             Solution C[i][n] = -Delta_m/(2l+1) (<r^l> M^I_c + <r^-(l+1)> M^R_c)
//
// The scan is a segmented prefix/suffix sum over radius, one segment per mode.
// A workgroup owns 16 or 8 consecutive modes (coalesced 128- or 64-byte row
// segments; the count is the plan's) and splits radius into 64 chunks: each thread sums one chunk of one mode, then one
// wavefront per mode scans the 64 chunk totals with lane shuffles (prefix for
// the outward sums, suffix for the inward ones), and a second pass writes
// edges and coefficients.  Chunk-boundary edges are always the scanned totals
// (never a thread's running sum), so the two chunks meeting at an edge use
// bitwise the same value.  Chunks of at most SG shells load their operands
// once, before the first pass, and keep them and the outward edges in
// registers: vector memory counters retire in issue order, so a load issued
// after a store would wait for the store.
#pragma once
#include "device_util.h"

namespace mpole {
namespace {


__device__ __forceinline__ void reduce_item(const Job &J) {
  const PlanDev &P = J.P;
  const auto ang_out = gmem(J.io.ang);
  const int gx = (P.namp + 255) / 256;
  const int i = J.local / gx;
  const int n = (J.local % gx) * 256 + item_tid();
  if (n >= P.namp) return;
  const ClassDev C = ld_const(P.classes + ld_const(P.shell_class + i));
  const int row = ld_const(P.shell_row + i);
  // the partials hold moment mode columns: natural mode n sits in column
  // pos_m[n] (padding modes past nam have none and sum to 0)
  const int col = P.pos_m ? gmem(P.pos_m)[n] : n;
  const size_t off = (size_t)row * P.namp_m + max(col, 0);
  const size_t stride = (size_t)C.nrows * P.namp_m;
  double s = 0.0;
  if (col < 0) {
  } else if (P.nplanes == 0) {
    const auto src = gmem(C.partial) + off;   // FP64 partials
#pragma unroll 8
    for (int q = 0; q < C.splits; ++q) s += src[q * stride];
  } else if (n == 0) {
    // split precisions: the monopole moment, summed in FP64 by the packing
    // workgroups of this shell, in workgroup order
    for (int q = 0; q < C.npack; ++q) s += gmem(P.mono_part)[(size_t)i * P.mono_stride + q];
  } else {
    const auto src = gmem(reinterpret_cast<const float *>(C.partial)) + off;   // FP32 partials
#pragma unroll 8
    for (int q = 0; q < C.splits; ++q) s += (double)src[q * stride];
    // the mean source density removed by the packing, times the column sum
    s += gmem(P.shift)[i] * gmem(C.tsum)[n];
  }
  gmem(P.ang)[(size_t)i * P.namp + n] = s;
  if (ang_out != nullptr && n < P.nam) ang_out[(size_t)i * P.nam + n] = s;
}

constexpr int SCAN_CHUNKS = 64;   // radial chunks per mode (one per lane of a wavefront)
constexpr int SG = 8;             // shells whose operands are loaded together

// Scan of one (mode, chunk) thread when the chunk holds at most SG shells: the
// arithmetic of scan_item below, in the same order, from registers.
template <int SCAN_MODES>
__device__ __forceinline__ void scan_chunk_in_registers(const Job &J, double *lds, bool live, int n, int l, int mode,
                                                        int c, int i0, int i1) {
  double(*tot_r)[SCAN_MODES] = reinterpret_cast<double(*)[SCAN_MODES]>(lds);
  double(*tot_i)[SCAN_MODES] = reinterpret_cast<double(*)[SCAN_MODES]>(lds + SCAN_CHUNKS * SCAN_MODES);
  double(*base_r)[SCAN_MODES] = reinterpret_cast<double(*)[SCAN_MODES]>(lds + 2 * SCAN_CHUNKS * SCAN_MODES);
  double(*base_i)[SCAN_MODES] =
      reinterpret_cast<double(*)[SCAN_MODES]>(lds + (2 * SCAN_CHUNKS + SCAN_CHUNKS + 1) * SCAN_MODES);
  const PlanDev &P = J.P;
  const auto er = gmem(J.io.interior ? J.io.interior : P.edge_r);
  const auto ei = gmem(J.io.exterior ? J.io.exterior : P.edge_i);
  const auto coef = gmem(P.coef);
  const auto A = gmem(P.ang);
  const auto jr = gmem(P.jr), ji = gmem(P.ji), rr = gmem(P.rr), ri = gmem(P.ri);
  const int ld_r = J.io.interior ? P.nam : P.namp;
  const int ld_i = J.io.exterior ? P.nam : P.namp;
  const int nr = P.nr, L1 = P.lmax + 1, namp = P.namp;
  const int nc = i1 - i0;   // shells of this chunk, 0 .. SG
  // every operand of the chunk, loaded together (entries past the chunk read
  // its first shell, or shell 0, and are not used)
  double av[SG], jrv[SG], jiv[SG], rrv[SG], riv[SG];
  const int ib = min(i0, nr - 1);
#pragma unroll
  for (int u = 0; u < SG; ++u) {
    const int i = u < nc ? i0 + u : ib;
    av[u] = A[(size_t)i * namp + n];
    jrv[u] = jr[i * L1 + l];
    jiv[u] = ji[i * L1 + l];
    rrv[u] = rr[i * L1 + l];
    riv[u] = ri[i * L1 + l];
  }
  // pass 1: chunk totals
  double sr = 0.0, si = 0.0;
  if (live) {
#pragma unroll
    for (int u = 0; u < SG; ++u) {
      if (u >= nc) break;
      sr += jrv[u] * av[u];
      si += jiv[u] * av[u];
    }
  }
  tot_r[c][mode] = sr;
  tot_i[c][mode] = si;
  __syncthreads();
  {
    const int t = item_tid(), w = t / 64, lane = t % 64;
    double x = tot_r[lane][w];
    double z = tot_i[lane][w];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const double xu = __shfl_up(x, d, 64);
      const double zd = __shfl_down(z, d, 64);
      if (lane >= d) x += xu;
      if (lane + d < 64) z += zd;
    }
    base_r[lane + 1][w] = x;
    base_i[lane][w] = z;
    if (lane == 0) base_r[0][w] = 0.0;
    if (lane == 63) base_i[SCAN_CHUNKS][w] = 0.0;
  }
  __syncthreads();
  if (!live) {
#pragma unroll
    for (int u = 0; u < SG; ++u)
      if (u < nc) coef[(size_t)(i0 + u) * namp + n] = 0.0;
    return;
  }
  // pass 2a: outward edges i0 .. i1-1, kept for pass 2b
  double ev[SG];
  double mr = base_r[c][mode];
#pragma unroll
  for (int u = 0; u < SG; ++u) {
    ev[u] = mr;
    if (u < nc) {
      er[(size_t)(i0 + u) * ld_r + n] = mr;
      mr += jrv[u] * av[u];
    }
  }
  const double mr_end = base_r[c + 1][mode];
  const double mi_end = base_i[c + 1][mode];
  if (i1 == nr && nc > 0) {
    er[(size_t)nr * ld_r + n] = mr_end;
    ei[(size_t)nr * ld_i + n] = mi_end;
  }
  // pass 2b: inward edges and the coefficients of Eq. Solution
  const double dm = (n == l * l) ? 1.0 : 2.0;
  const double f = -dm / (2.0 * l + 1.0);
  double mi = mi_end, mr_hi = mr_end;
#pragma unroll
  for (int u = SG - 1; u >= 0; --u) {
    if (u >= nc) continue;
    const int i = i0 + u;
    const double mi_hi = mi;
    mi = (u == 0) ? base_i[c][mode] : mi + jiv[u] * av[u];
    ei[(size_t)i * ld_i + n] = mi;
    const double mr_lo = ev[u];
    const double mic = 0.5 * (mi + mi_hi), mrc = 0.5 * (mr_lo + mr_hi);
    coef[(size_t)i * namp + n] = f * (rrv[u] * mic + riv[u] * mrc);
    mr_hi = mr_lo;
  }
}

// LDS of a scan item in doubles: chunk totals and chunk bases, both sums
template <int SCAN_MODES>
constexpr int scan_lds() {
  return (2 * SCAN_CHUNKS + 2 * (SCAN_CHUNKS + 1)) * SCAN_MODES;
}

// Scan workgroup J.local of field J.f: SCAN_MODES modes x SCAN_CHUNKS radial
// chunks, one thread each (the per-mode arithmetic does not depend on
// SCAN_MODES: the chunking of the radius is fixed).
template <int SCAN_MODES>
__device__ __forceinline__ void scan_item(const Job &J, double *lds) {
  double(*tot_r)[SCAN_MODES] = reinterpret_cast<double(*)[SCAN_MODES]>(lds);
  double(*tot_i)[SCAN_MODES] = reinterpret_cast<double(*)[SCAN_MODES]>(lds + SCAN_CHUNKS * SCAN_MODES);
  double(*base_r)[SCAN_MODES] = reinterpret_cast<double(*)[SCAN_MODES]>(lds + 2 * SCAN_CHUNKS * SCAN_MODES);
  double(*base_i)[SCAN_MODES] =
      reinterpret_cast<double(*)[SCAN_MODES]>(lds + (2 * SCAN_CHUNKS + SCAN_CHUNKS + 1) * SCAN_MODES);
  const PlanDev &P = J.P;
  // edge moments go to the caller's [nr+1][nAM] buffers, or to the workspace
  const auto er = gmem(J.io.interior ? J.io.interior : P.edge_r);
  const auto ei = gmem(J.io.exterior ? J.io.exterior : P.edge_i);
  const auto coef = gmem(P.coef);
  const auto rr = gmem(P.rr), ri = gmem(P.ri);
  const int ld_r = J.io.interior ? P.nam : P.namp;
  const int ld_i = J.io.exterior ? P.nam : P.namp;
  const int t = item_tid();
  const int mode = t % SCAN_MODES, c = t / SCAN_MODES;   // chunk c of mode n
  const int n = J.local * SCAN_MODES + mode;
  const int nr = P.nr, L1 = P.lmax + 1, namp = P.namp;
  const bool live = n < P.nam;
  int l = 0;
  if (live) {
    l = (int)sqrt((double)n);
    while ((l + 1) * (l + 1) <= n) ++l;
    while (l * l > n) --l;
  }
  const int cs = (nr + SCAN_CHUNKS - 1) / SCAN_CHUNKS;
  const int i0 = min(nr, c * cs), i1 = min(nr, i0 + cs);
  if (cs <= SG) {   // workgroup-uniform
    scan_chunk_in_registers<SCAN_MODES>(J, lds, live, n, l, mode, c, i0, i1);
    return;
  }
  const auto A = gmem(P.ang);
  const auto jr = gmem(P.jr), ji = gmem(P.ji);

  // pass 1: chunk totals of the regular and irregular increments
  double sr = 0.0, si = 0.0;
  if (live) {
#pragma unroll 8
    for (int i = i0; i < i1; ++i) {
      const double a = A[(size_t)i * namp + n];
      sr += jr[i * L1 + l] * a;
      si += ji[i * L1 + l] * a;
    }
  }
  tot_r[c][mode] = sr;
  tot_i[c][mode] = si;
  __syncthreads();

  // wavefront w scans the 64 chunk totals of mode w with lane = chunk:
  // inclusive prefix (outward) and inclusive suffix (inward) by shuffles
  {
    const int w = t / 64, lane = t % 64;
    double x = tot_r[lane][w];
    double z = tot_i[lane][w];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const double xu = __shfl_up(x, d, 64);
      const double zd = __shfl_down(z, d, 64);
      if (lane >= d) x += xu;
      if (lane + d < 64) z += zd;
    }
    base_r[lane + 1][w] = x;    // M^R at the first edge of chunk lane+1
    base_i[lane][w] = z;        // M^I at the first edge of chunk lane
    if (lane == 0) base_r[0][w] = 0.0;
    if (lane == 63) base_i[SCAN_CHUNKS][w] = 0.0;
  }
  __syncthreads();

  if (!live) {
    for (int i = i0; i < i1; ++i) coef[(size_t)i * namp + n] = 0.0;
    return;
  }
  // pass 2a: outward edges i0 .. i1-1; chunk boundaries come from base_r only.
  // Both passes load SG shells' operands before the group's stores, so the
  // loads of a group are in flight together (the stores could alias them,
  // which would otherwise order every load behind the previous shell's
  // store); the arithmetic order is the plain sequential one.
  double mr = base_r[c][mode];
  for (int g0 = i0; g0 < i1; g0 += SG) {
    double av[SG], jv[SG];
#pragma unroll
    for (int u = 0; u < SG; ++u) {
      const int i = min(g0 + u, i1 - 1);
      av[u] = A[(size_t)i * namp + n];
      jv[u] = jr[i * L1 + l];
    }
#pragma unroll
    for (int u = 0; u < SG; ++u) {
      if (g0 + u >= i1) break;
      er[(size_t)(g0 + u) * ld_r + n] = mr;
      mr += jv[u] * av[u];
    }
  }
  const double mr_end = base_r[c + 1][mode];
  const double mi_end = base_i[c + 1][mode];
  if (i1 == nr && i0 < i1) {
    er[(size_t)nr * ld_r + n] = mr_end;
    ei[(size_t)nr * ld_i + n] = mi_end;
  }
  // pass 2b: inward edges and the coefficients of Eq. Solution
  const double dm = (n == l * l) ? 1.0 : 2.0;
  const double f = -dm / (2.0 * l + 1.0);
  double mi = mi_end, mr_hi = mr_end;
  for (int g1 = i1 - 1; g1 >= i0; g1 -= SG) {
    double av[SG], jv[SG], ev[SG], rv[SG], qv[SG];
#pragma unroll
    for (int u = 0; u < SG; ++u) {
      const int i = max(g1 - u, i0);
      av[u] = A[(size_t)i * namp + n];
      jv[u] = ji[i * L1 + l];
      ev[u] = er[(size_t)i * ld_r + n];   // written by this thread in pass 2a
      rv[u] = rr[i * L1 + l];
      qv[u] = ri[i * L1 + l];
    }
#pragma unroll
    for (int u = 0; u < SG; ++u) {
      const int i = g1 - u;
      if (i < i0) break;
      const double mi_hi = mi;
      mi = (i == i0) ? base_i[c][mode] : mi + jv[u] * av[u];
      ei[(size_t)i * ld_i + n] = mi;
      const double mr_lo = ev[u];
      const double mic = 0.5 * (mi + mi_hi), mrc = 0.5 * (mr_lo + mr_hi);
      coef[(size_t)i * namp + n] = f * (rv[u] * mic + qv[u] * mrc);
      mr_hi = mr_lo;
    }
  }
}

}  // namespace
}  // namespace mpole
