// Synthetic density of the repeated-solve workload: a radial profile times
// (1 + eps * a low-order real-harmonic perturbation) whose pattern is rotated
// by R, i.e. the perturbation is evaluated at R^T n for the cell-centre
// direction n.  A generator of input, not part of the multipole method; it
// runs on the device so that a sequence of solves on an advected density can
// be captured in one HIP graph.
//
// The harmonics are the orthonormal real ones with the Condon-Shortley
// phase: Y_l0 = Pn_l^0(cos t), and for m > 0 sqrt(2) Pn_l^m(cos t) cos(m p)
// ("c") and sqrt(2) Pn_l^m(cos t) sin(m p) ("s"), where Pn_l^m is the
// associated Legendre function normalised so that Pn_l^m(cos t) e^{i m p} is
// the complex orthonormal harmonic.  Pn is evaluated by the standard
// three-term recurrence in l at fixed m, started from the sectoral values
// Pn_m^m = -sqrt((2m+1)/(2m)) sin t Pn_{m-1}^{m-1}, Pn_0^0 = 1/sqrt(4 pi),
// and cos(m p), sin(m p) by repeated complex multiplication, so neither the
// rotated angles nor any inverse trigonometric function is formed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "mpole_workload.h"

namespace {

constexpr int kMaxL = 16;
constexpr int kShellsPerWg = 64;
constexpr double kPi = 3.14159265358979323846264338327950288;

struct Args {
  int nr, nt, np, lpert;
  const double *radial, *theta_c, *phi_c, *coef, *rot;
  double eps;
  double *rho;
};

__global__ __launch_bounds__(256) void k_rotated_density(Args a) {
  const int ncell = a.nt * a.np;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= ncell) return;
  const int j = q / a.np, k = q % a.np;
  // cell-centre direction and its image under R^T
  double st, ct, sp, cp;
  sincos(a.theta_c[j], &st, &ct);
  sincos(a.phi_c[k], &sp, &cp);
  const double n[3] = {st * cp, st * sp, ct};
  const double *R = a.rot;   // row-major
  const double vx = R[0] * n[0] + R[3] * n[1] + R[6] * n[2];
  const double vy = R[1] * n[0] + R[4] * n[1] + R[7] * n[2];
  const double vz = R[2] * n[0] + R[5] * n[1] + R[8] * n[2];
  const double x = fmin(1.0, fmax(-1.0, vz));   // cos t'
  const double s = sqrt(vx * vx + vy * vy);     // sin t' >= 0
  double c1 = 1.0, s1 = 0.0;                    // cos p', sin p'
  if (s > 0.0) {
    c1 = vx / s;
    s1 = vy / s;
  }
  const int L = a.lpert;
  double sum = 0.0;
  double pmm = 1.0 / sqrt(4.0 * kPi);   // Pn_m^m
  double cm = 1.0, sm = 0.0;            // cos m p', sin m p'
  for (int m = 0; m <= L; ++m) {
    if (m > 0) {
      pmm *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
      const double c = cm * c1 - sm * s1;
      sm = sm * c1 + cm * s1;
      cm = c;
    }
    double p2 = 0.0, p1 = pmm;   // Pn_{l-2}^m, Pn_{l-1}^m
    for (int l = m; l <= L; ++l) {
      double p;
      if (l == m) {
        p = pmm;
      } else if (l == m + 1) {
        p = sqrt(2.0 * m + 3.0) * x * pmm;
      } else {
        const double al = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
        const double bl = sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
        p = al * (x * p1 - bl * p2);
      }
      if (l > m) {
        p2 = p1;
        p1 = p;
      }
      const int base = l * l;
      if (m == 0) {
        sum += a.coef[base] * p;
      } else {
        const double f = sqrt(2.0) * p;
        sum += a.coef[base + 2 * m - 1] * f * cm + a.coef[base + 2 * m] * f * sm;
      }
    }
  }
  const double ang = 1.0 + a.eps * sum;
  const int i0 = blockIdx.y * kShellsPerWg, i1 = min(a.nr, i0 + kShellsPerWg);
  for (int i = i0; i < i1; ++i) a.rho[(size_t)i * ncell + q] = a.radial[i] * ang;
}

}  // namespace

extern "C" int mpole_wl_rotated_density(int32_t nr, int32_t ntheta, int32_t nphi, const double *radial,
                                        const double *theta_c, const double *phi_c, int32_t lpert,
                                        const double *coef, double eps, const double *rot, double *rho,
                                        void *stream) {
  if (nr < 1 || ntheta < 1 || nphi < 1 || (int64_t)ntheta * nphi > (1 << 30)) return 1;
  if (lpert < 0 || lpert > kMaxL) return 1;
  if (!radial || !theta_c || !phi_c || !coef || !rot || !rho) return 1;
  Args a{nr, ntheta, nphi, lpert, radial, theta_c, phi_c, coef, rot, eps, rho};
  const int ncell = ntheta * nphi;
  const dim3 grid((ncell + 255) / 256, (nr + kShellsPerWg - 1) / kShellsPerWg);
  hipLaunchKernelGGL(k_rotated_density, grid, dim3(256), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? 0 : 4;
}
