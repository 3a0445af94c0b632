/*
 * Device-side input generator for the repeated-solve workload (a separate
 * library, libmpole_workload.so; not part of the multipole method).
 *
 * mpole_wl_rotated_density: writes, on hip_stream,
 *     rho[i][j][k] = radial[i] * (1 + eps * sum_n coef[n] Y_n(R^T u_jk))
 * where u_jk is the unit vector of the cell centre (theta_c[j], phi_c[k]),
 * R the 3 x 3 rotation rot[9] (row-major), and Y_n the orthonormal real
 * spherical harmonics with the Condon-Shortley phase in the collapsed order of
 * the multipole library: n = l^2 for m = 0, l^2 + 2m - 1 for (m, cos),
 * l^2 + 2m for (m, sin), l <= lpert.  A rotation of the pattern by R is the
 * advection of the perturbation by a rigid rotation.
 *
 * All pointers are device pointers owned by the caller: radial [nr],
 * theta_c [ntheta], phi_c [nphi], coef [(lpert+1)^2], rot [9], rho
 * [nr][ntheta][nphi] (phi fastest).  Returns 0, 1 for invalid arguments
 * (sizes < 1, ntheta*nphi > 2^30, lpert outside [0, 16], a null pointer;
 * nothing is enqueued), 4 for a launch failure.  One kernel launch, no
 * allocation or host synchronisation: capturable in a HIP graph.
 */
#ifndef MPOLE_WORKLOAD_H
#define MPOLE_WORKLOAD_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

int mpole_wl_rotated_density(int32_t nr, int32_t ntheta, int32_t nphi, const double *radial,
                             const double *theta_c, const double *phi_c, int32_t lpert, const double *coef,
                             double eps, const double *rot, double *rho, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
