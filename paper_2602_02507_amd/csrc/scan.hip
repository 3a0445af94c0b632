// Radial part of the solve in FP64 (GenASiS II Sec. 2.2, the edge
// recurrences after Eq. Solution):
//
//   k_reduce  angular moments A[i][n] = fixed-order sum of the split-K
//             partials of the moment contraction
//   k_scan    regular moments by outward integration, M^R_0 = 0,
//             M^R_{i+1} = M^R_i + JR_l(i) A[i][n]; irregular moments by
//             inward integration, M^I_nr = 0, M^I_i = M^I_{i+1} + JI_l(i) A[i][n];
//             centre values (M_i + M_{i+1})/2 and the coefficients of Eq.
//             Solution C[i][n] = -Delta_m/(2l+1) (<r^l> M^I_c + <r^-(l+1)> M^R_c)
//
// The scan is a segmented prefix/suffix sum over radius, one segment per mode.
// A wavefront owns 16 consecutive modes (coalesced 128-byte rows) split into
// 4 radial chunks, one per 16-lane group: each lane sums its chunk, the four
// chunk totals are exchanged with wavefront shuffles, and a second pass writes
// edges and coefficients.  Chunk-boundary edges are always taken from the
// shuffled totals (never from a lane's running sum), so the two chunks that
// meet at an edge use bitwise the same value.
#include "mpole_internal.h"

namespace mpole {
namespace {

__global__ __launch_bounds__(256) void k_reduce(PlanDev P, double *__restrict__ ang_out) {
  const int i = blockIdx.y;
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= P.namp) return;
  const ClassDev C = P.classes[P.shell_class[i]];
  const int row = P.shell_row[i];
  const double *__restrict__ src = C.partial + (size_t)row * P.namp + n;
  const size_t stride = (size_t)C.nrows * P.namp;
  double s = 0.0;
  for (int q = 0; q < C.splits; ++q) s += src[q * stride];
  P.ang[(size_t)i * P.namp + n] = s;
  if (ang_out != nullptr && n < P.nam) ang_out[(size_t)i * P.nam + n] = s;
}

__global__ __launch_bounds__(256) void k_scan(PlanDev P, double *__restrict__ er, int ld_r,
                                              double *__restrict__ ei, int ld_i) {
  const int lane = threadIdx.x & 63;
  const int slab = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int n = slab * 16 + (lane & 15);
  if (slab * 16 >= P.namp) return;          // whole wavefront idle
  const int g = lane >> 4;                  // radial chunk of this lane
  const int nr = P.nr, L1 = P.lmax + 1, namp = P.namp;
  const bool live = n < P.nam;
  int l = 0;
  if (live) {
    l = (int)sqrt((double)n);
    while ((l + 1) * (l + 1) <= n) ++l;
    while (l * l > n) --l;
  }
  const int cs = (nr + 3) / 4;
  const int i0 = min(nr, g * cs), i1 = min(nr, i0 + cs);
  const double *__restrict__ A = P.ang;

  // pass 1: chunk totals of the regular and irregular increments
  double sr = 0.0, si = 0.0;
  if (live)
    for (int i = i0; i < i1; ++i) {
      const double a = A[(size_t)i * namp + n];
      sr += P.jr[i * L1 + l] * a;
      si += P.ji[i * L1 + l] * a;
    }
  // exchange the four chunk totals of this mode (lanes n%16 + 16 q)
  double tr[4], ti[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    tr[q] = __shfl(sr, (lane & 15) + 16 * q, 64);
    ti[q] = __shfl(si, (lane & 15) + 16 * q, 64);
  }
  double base_r = 0.0, base_i = 0.0;      // M^R at edge i0, M^I at edge i1
  for (int q = 0; q < g; ++q) base_r += tr[q];
  for (int q = 3; q > g; --q) base_i += ti[q];
  if (!live) {
    for (int i = i0; i < i1; ++i) P.coef[(size_t)i * namp + n] = 0.0;
    return;
  }
  // pass 2a: outward edges i0 .. i1-1 (edge i1 belongs to the next chunk)
  double mr = base_r;
  for (int i = i0; i < i1; ++i) {
    er[(size_t)i * ld_r + n] = mr;
    mr += P.jr[i * L1 + l] * A[(size_t)i * namp + n];
  }
  const double mr_end = base_r + sr;        // = base_r of the next chunk, same order
  if (i1 == nr && i0 < i1) er[(size_t)nr * ld_r + n] = mr_end;
  // pass 2b: inward edges and the coefficients of Eq. Solution
  const double dm = (n == l * l) ? 1.0 : 2.0;
  const double f = -dm / (2.0 * l + 1.0);
  double mi = base_i;
  if (i1 == nr && i0 < i1) ei[(size_t)nr * ld_i + n] = mi;
  double mr_hi = mr_end;
  for (int i = i1 - 1; i >= i0; --i) {
    const double mi_hi = mi;
    // edge i0 is the previous chunk's base: take it from the shuffled totals
    mi = (i == i0) ? base_i + si : mi + P.ji[i * L1 + l] * A[(size_t)i * namp + n];
    ei[(size_t)i * ld_i + n] = mi;
    const double mr_lo = er[(size_t)i * ld_r + n];
    const double mic = 0.5 * (mi + mi_hi), mrc = 0.5 * (mr_lo + mr_hi);
    P.coef[(size_t)i * namp + n] = f * (P.rr[i * L1 + l] * mic + P.ri[i * L1 + l] * mrc);
    mr_hi = mr_lo;
  }
}

}  // namespace

hipError_t launch_reduce(const PlanDev &P, double *ang_out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3((P.namp + 255) / 256, P.nr), dim3(256), 0, s, P, ang_out);
  return hipGetLastError();
}

hipError_t launch_scan(const PlanDev &P, double *interior, double *exterior, hipStream_t s) {
  double *er = interior ? interior : P.edge_r;
  double *ei = exterior ? exterior : P.edge_i;
  const int ldr = interior ? P.nam : P.namp;
  const int ldi = exterior ? P.nam : P.namp;
  const int slabs = P.namp / 16;
  hipLaunchKernelGGL(k_scan, dim3((slabs + 3) / 4), dim3(256), 0, s, P, er, ldr, ei, ldi);
  return hipGetLastError();
}

}  // namespace mpole
