// One-time FP64 tables of a plan (GenASiS II Sec. 2.2: the cell-averaged
// angular and radial kernels are computed once at the beginning of a run).
//
//   k_theta_avg   solid-angle weighted theta-cell averages of P~_l^m, by
//                 composite 16-point Gauss-Legendre quadrature in theta of
//                 P~_l^m(cos th) sin th (the paper uses Romberg; any quadrature
//                 exact to rounding gives the same table)
//   k_trig        phi-cell averages of cos m ph and sin m ph (exact antiderivative)
//   k_weight      dOmega and 4 pi G dOmega per angular cell (S = 4 pi G rho)
//   k_block_table solid-angle weighted block means of A_iAM = <P~> x <trig>
//   k_radial      exact shell integrals of r^(2+l), r^(1-l) and the volume
//                 averages of r^l, r^-(l+1) used by the radial sums
#include <algorithm>

#include "device_util.h"

namespace mpole {
namespace {

// P~_l^m(x) at x = cos th, s = sin th, by the m-seeded three-term recurrence in l.
__device__ double ptilde(int l, int m, double x, double s) {
  double pmm = sqrt((2.0 * m + 1.0) / (4.0 * kPi));
  for (int i = 1; i <= m; ++i) pmm *= -sqrt((2.0 * i - 1.0) / (2.0 * i)) * s;
  if (l == m) return pmm;
  double p1 = x * sqrt(2.0 * m + 3.0) * pmm;
  double p0 = pmm;
  for (int k = m + 2; k <= l; ++k) {
    const double dk = (double)k, dm = (double)m;
    const double a = sqrt((4.0 * dk * dk - 1.0) / (dk * dk - dm * dm));
    const double b = sqrt(((dk - 1.0) * (dk - 1.0) - dm * dm) / (4.0 * (dk - 1.0) * (dk - 1.0) - 1.0));
    const double p = a * (x * p1 - b * p0);
    p0 = p1;
    p1 = p;
  }
  return p1;
}

__global__ void k_theta_avg(PlanDev P, GaussRule g) {
  const int nplm = (P.lmax + 1) * (P.lmax + 2) / 2;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)P.ntheta * nplm) return;
  const int j = (int)(t / nplm), p = (int)(t % nplm);
  int l = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while ((l + 1) * (l + 2) / 2 <= p) ++l;
  while (l * (l + 1) / 2 > p) --l;
  const int m = p - l * (l + 1) / 2;
  const double t0 = P.theta_edges[j], t1 = P.theta_edges[j + 1];
  // sub-intervals short enough that 16 nodes resolve degree lmax+1 to rounding
  const int nsub = max(1, (int)ceil((P.lmax + 1) * (t1 - t0) * 0.5));
  const double h = (t1 - t0) / nsub;
  double acc = 0.0;
  for (int s = 0; s < nsub; ++s) {
    const double mid = t0 + (s + 0.5) * h;
    double part = 0.0;
    for (int q = 0; q < kGaussNodes; ++q) {
      const double th = mid + 0.5 * h * g.x[q];
      double sn, cs;
      sincos(th, &sn, &cs);
      part += g.w[q] * sn * ptilde(l, m, cs, sn);
    }
    acc += 0.5 * h * part;
  }
  P.pavg[(size_t)j * nplm + p] = acc / cos_diff(t0, t1);
}

__global__ void k_trig(PlanDev P) {
  const int L1 = P.lmax + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P.nphi * L1) return;
  const int k = t / L1, m = t % L1;
  const double p0 = P.phi_edges[k], p1 = P.phi_edges[k + 1];
  double c = 1.0, s = 0.0;
  if (m > 0) {
    // (sin m p1 - sin m p0)/(m dp) and (cos m p0 - cos m p1)/(m dp) as products
    const double half = 0.5 * m * (p1 - p0);
    const double f = sin(half) / half;
    double sm, cm;
    sincos(0.5 * m * (p0 + p1), &sm, &cm);
    c = cm * f;
    s = sm * f;
  }
  P.trig[(size_t)k * 2 * L1 + 2 * m] = c;
  P.trig[(size_t)k * 2 * L1 + 2 * m + 1] = s;
}

// dOmega and the source weight 4 pi G dOmega of each cell; the weight is the
// product of a row factor 4 pi G (cos th_j - cos th_j+1) and the column
// width dph_k, both kept, so that kernels can form it from the two factors
// bitwise equal to the table.
__global__ void k_weight(PlanDev P) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P.ncell) return;
  const int j = q / P.nphi, k = q % P.nphi;
  const double dc = cos_diff(P.theta_edges[j], P.theta_edges[j + 1]);
  const double dp = P.phi_edges[k + 1] - P.phi_edges[k];
  const double wr = 4.0 * kPi * P.G * dc;
  P.dom[q] = dc * dp;
  P.weight[q] = wr * dp;
  if (k == 0) P.wrow[j] = wr;
  if (j == 0) P.dphi[k] = dp;
}

__global__ void k_block_table(PlanDev P, ClassDev C) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)C.nblocks_pad * P.namp) return;
  const int b = (int)(t / P.namp), n = (int)(t % P.namp);
  double v = 0.0;
  if (b < C.nblocks && n < P.nam) {
    int l = (int)sqrt((double)n);
    while ((l + 1) * (l + 1) <= n) ++l;
    while (l * l > n) --l;
    const int d = n - l * l;
    const int m = (d + 1) >> 1;
    const int a = (d > 0 && (d & 1) == 0) ? 1 : 0;
    const int nplm = (P.lmax + 1) * (P.lmax + 2) / 2;
    const int p = l * (l + 1) / 2 + m;
    const int L1 = P.lmax + 1;
    double num = 0.0, den = 0.0;
    for (int e = C.moff[b]; e < C.moff[b + 1]; ++e) {
      const int q = C.mem[e];
      const int j = q / P.nphi, k = q % P.nphi;
      const double dom = cos_diff(P.theta_edges[j], P.theta_edges[j + 1]) * (P.phi_edges[k + 1] - P.phi_edges[k]);
      num += dom * (P.pavg[(size_t)j * nplm + p] * P.trig[(size_t)k * 2 * L1 + 2 * m + a]);
      den += dom;
    }
    v = num / den;
  }
  C.table[t] = v;
}

// Per pair q: tcol0[q] (l = 0 kernel) and, folded FP64, tm[q][column] and
// te[q][column] over the moment and expansion mode columns.
__global__ void k_pair_tables(PlanDev P, ClassDev C) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nm = (long)C.npair_pad * P.namp_m, ne = (long)C.npair_pad * P.namp_e;
  if (t < C.npair_pad) C.tcol0[t] = pair_kernel(P, C, (int)t, 0);
  if (!P.fold || P.nplanes != 0) return;
  if (t < nm) {
    const int q = (int)(t / P.namp_m), col = (int)(t % P.namp_m);
    C.tm[t] = pair_kernel(P, C, q, P.perm_m[col]);
  }
  if (t < ne) {
    const int q = (int)(t / P.namp_e), col = (int)(t % P.namp_e);
    C.te[t] = pair_kernel(P, C, q, P.perm_e[col]);
  }
}

// 4 pi G dOmega of each block: the cell weights of its members, in CSR order.
__global__ void k_block_wsum(PlanDev P, ClassDev C) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= C.nblocks) return;
  double w = 0.0;
  for (int e = C.moff[b]; e < C.moff[b + 1]; ++e) w += P.weight[C.mem[e]];
  C.wsum[b] = w;
}

// Column sums tsum[n] = sum_b wsum[b] table[b][n] (the integral of each
// kernel over the sphere, 4 pi G sqrt(4 pi) for n = 0 and 0 otherwise up to
// quadrature error), in two fixed-order passes: kTsumChunks contiguous block
// ranges, then the chunk totals in chunk order.
__global__ void k_tsum_part(PlanDev P, ClassDev C) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P.namp) return;
  const int ch = blockIdx.y;
  const int span = (C.nblocks + kTsumChunks - 1) / kTsumChunks;
  const int b0 = ch * span, b1 = min(C.nblocks, b0 + span);
  double s = 0.0;
  for (int b = b0; b < b1; ++b) s += C.wsum[b] * C.table[(size_t)b * P.namp + n];
  P.tsum_part[(size_t)ch * P.namp + n] = s;
}

__global__ void k_tsum_final(PlanDev P, ClassDev C) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P.namp) return;
  double s = 0.0;
  for (int ch = 0; ch < kTsumChunks; ++ch) s += P.tsum_part[(size_t)ch * P.namp + n];
  C.tsum[n] = s;
}

// b^p - a^p for 0 < a < b without cancellation for thin shells
__device__ double pow_span(double a, double b, double p) {
  const double lr = log1p((b - a) / a);
  const double x = p * lr;
  if (fabs(x) < 1.0) return pow(a, p) * expm1(x);
  return pow(b, p) - pow(a, p);
}

__global__ void k_radial(PlanDev P) {
  const int L1 = P.lmax + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P.nr * L1) return;
  const int i = t / L1, l = t % L1;
  const double a = P.r_edges[i], b = P.r_edges[i + 1];
  double v3, jr, ji;
  if (a > 0.0) {
    v3 = pow_span(a, b, 3.0) / 3.0;
    jr = pow_span(a, b, l + 3.0) / (l + 3.0);
    ji = (l == 2) ? log1p((b - a) / a) : pow_span(a, b, 2.0 - l) / (2.0 - l);
  } else {
    // shell containing the origin: r^2 r^-(l+1) is integrable only for l = 0, 1
    v3 = b * b * b / 3.0;
    jr = pow(b, l + 3.0) / (l + 3.0);
    ji = (l == 0) ? 0.5 * b * b : (l == 1) ? b : 0.0;
  }
  P.jr[t] = jr;
  P.ji[t] = ji;
  P.rr[t] = jr / v3;
  P.ri[t] = ji / v3;
}

__global__ void k_fill_word(uint4 *p, size_t n16, uint32_t w) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(w, w, w, w);
}

__global__ void k_fill_value(double *p, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

inline unsigned grid_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_fill_word(void *p, size_t bytes, uint32_t word, hipStream_t s) {
  // callers pass 16-byte multiples of 256-byte aligned workspace regions
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<size_t>((n16 + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_word, dim3(g), dim3(256), 0, s, (uint4 *)p, n16, word);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) { return launch_fill_word(p, bytes, 0u, s); }

hipError_t launch_fill_value(double *p, size_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_value, dim3(g), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_tables(const PlanDev &P, const ClassDev *host_classes, const GaussRule &g, bool dense,
                         hipStream_t s) {
  const int nplm = (P.lmax + 1) * (P.lmax + 2) / 2;
  hipLaunchKernelGGL(k_theta_avg, dim3(grid_for((long)P.ntheta * nplm, 64)), dim3(64), 0, s, P, g);
  hipLaunchKernelGGL(k_trig, dim3(grid_for((long)P.nphi * (P.lmax + 1), 256)), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_weight, dim3(grid_for(P.ncell, 256)), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_radial, dim3(grid_for((long)P.nr * (P.lmax + 1), 256)), dim3(256), 0, s, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int c = 0; c < P.nclasses; ++c) {
    const ClassDev &C = host_classes[c];
    hipLaunchKernelGGL(k_block_wsum, dim3(grid_for(C.nblocks, 256)), dim3(256), 0, s, P, C);
    if (dense) {   // block-mean kernel table and its weighted column sums
      hipLaunchKernelGGL(k_block_table, dim3(grid_for((long)C.nblocks_pad * P.namp, 256)), dim3(256), 0, s, P, C);
      hipLaunchKernelGGL(k_tsum_part, dim3(grid_for(P.namp, 256), kTsumChunks), dim3(256), 0, s, P, C);
      hipLaunchKernelGGL(k_tsum_final, dim3(grid_for(P.namp, 256)), dim3(256), 0, s, P, C);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_pair_tables(const PlanDev &P, const ClassDev *host_classes, hipStream_t s) {
  for (int c = 0; c < P.nclasses; ++c) {
    const ClassDev &C = host_classes[c];
    const long n = (long)C.npair_pad * std::max(std::max(P.namp_m, P.namp_e), 1);
    hipLaunchKernelGGL(k_pair_tables, dim3(grid_for(n, 256)), dim3(256), 0, s, P, C);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mpole
