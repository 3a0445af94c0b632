// Coordinate gradient of the potential for the gravitational source terms
// of the balance equations (Sec. 3: the -rho grad Phi and -rho v . grad Phi
// sources, each derivative the simplest centred difference over the two
// nearest neighbours).
//
// dPhi/dr, dPhi/dtheta and dPhi/dphi at cell centres (edge midpoints):
// (Phi(next) - Phi(previous)) / (x(next) - x(previous)); the first and last
// shell and theta row use the cell itself in place of the missing neighbour
// (one-sided), phi wraps around when its edges close the circle (else
// one-sided too), and a single-cell dimension has zero derivative.
//
// One thread per cell (grid x: cells of a shell, y: shells), phi fastest, so
// every neighbour load of a wavefront
// is a coalesced run; neighbours along theta (+-nphi) and radius (+-ncell)
// are re-read from L2 by the workgroups of the adjacent rows and shells.
// HBM-bound: about 8 B read and 24 B written per cell.
#include "device_util.h"

namespace mpole {
namespace {

__device__ inline double centre(const double *e, int i) { return 0.5 * (e[i] + e[i + 1]); }

__global__ __launch_bounds__(256) void k_gradient(PlanDev P, const double *phi_, double *d_r, double *d_th,
                                                  double *d_ph, int periodic) {
  const long ncell = (long)P.ntheta * P.nphi;
  const int i = blockIdx.y;                       // shell
  const int c = blockIdx.x * 256 + threadIdx.x;   // cell within the shell
  if (c >= ncell) return;
  const long q = (long)i * ncell + c;
  const int j = c / P.nphi, k = c - j * P.nphi;
  const auto phi = gmem(phi_);
  if (d_r != nullptr) {
    double v = 0.0;
    if (P.nr > 1) {
      const int lo = i > 0 ? i - 1 : i, hi = i < P.nr - 1 ? i + 1 : i;
      v = (phi[(long)hi * ncell + c] - phi[(long)lo * ncell + c]) / (centre(P.r_edges, hi) - centre(P.r_edges, lo));
    }
    gmem(d_r)[q] = v;
  }
  if (d_th != nullptr) {
    double v = 0.0;
    if (P.ntheta > 1) {
      const int lo = j > 0 ? j - 1 : j, hi = j < P.ntheta - 1 ? j + 1 : j;
      v = (phi[q + (long)(hi - j) * P.nphi] - phi[q + (long)(lo - j) * P.nphi]) /
          (centre(P.theta_edges, hi) - centre(P.theta_edges, lo));
    }
    gmem(d_th)[q] = v;
  }
  if (d_ph != nullptr) {
    double v = 0.0;
    if (P.nphi > 1) {
      int lo, hi;
      double xl, xh;
      if (periodic) {
        lo = k > 0 ? k - 1 : P.nphi - 1;
        hi = k < P.nphi - 1 ? k + 1 : 0;
        xl = centre(P.phi_edges, lo) - (k == 0 ? 2.0 * kPi : 0.0);
        xh = centre(P.phi_edges, hi) + (k == P.nphi - 1 ? 2.0 * kPi : 0.0);
      } else {
        lo = k > 0 ? k - 1 : k;
        hi = k < P.nphi - 1 ? k + 1 : k;
        xl = centre(P.phi_edges, lo);
        xh = centre(P.phi_edges, hi);
      }
      v = (phi[q + (hi - k)] - phi[q + (lo - k)]) / (xh - xl);
    }
    gmem(d_ph)[q] = v;
  }
}

}  // namespace

hipError_t launch_gradient(const PlanDev &P, const double *phi, double *d_r, double *d_th, double *d_ph, int periodic,
                           hipStream_t s) {
  const long ncell = (long)P.ntheta * P.nphi;
  hipLaunchKernelGGL(k_gradient, dim3((unsigned)((ncell + 255) / 256), (unsigned)P.nr), dim3(256), 0, s, P, phi, d_r, d_th,
                     d_ph, periodic);
  return hipGetLastError();
}

}  // namespace mpole
