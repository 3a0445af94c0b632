/*
 * Plain FP64 CPU oracle for the multipole Poisson solve (GenASiS II, Sec. 2.2
 * "Poisson Solver"; coarsening blocks from Sec. 2.1 "Mesh").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the HIP library, and the
 * library never calls it.
 *
 * Every step follows the paper's description in its own order:
 *   - renormalised associated Legendre functions by the m-seeded recurrence
 *     in l (Sec. 2.2, the seed and three-term recurrence equations);
 *   - angular kernels A^c_lm = P~_l^m(cos th) cos(m ph), A^s_lm = P~ sin(m ph)
 *     (Eqs. AngularKernel_c, AngularKernel_s), averaged over each angular cell
 *     by Romberg integration in theta (the paper names Romberg) and by the
 *     exact antiderivative in phi;
 *   - discrete angular moments (Eq. AngularMomentsDiscrete);
 *   - outward / inward radial integration at shell edges with cell-averaged
 *     radial kernels R^R = r^l, R^I = r^-(l+1) (Eqs. RadialRegular,
 *     RadialIrregular and the edge recurrences that follow them);
 *   - linear interpolation of edge moments to the shell centre and the
 *     cell-averaged evaluation of Eq. Solution.
 * Sums run in ascending index order in plain FP64; OpenMP only splits
 * independent shells (or angular cells) between threads and never reorders a
 * sum.
 *
 * Conventions where the paper is silent (each is a documented reading):
 *   - mode set: 0 <= m <= l <= L, a in {c, s}, dropping the identically zero
 *     A^s_l0, so nAM = (L+1)^2; collapsed index iAM = l^2 for m = 0,
 *     l^2 + 2m - 1 for (m, c) and l^2 + 2m for (m, s);
 *   - cell averages are solid-angle weighted in angle and volume (r^2 dr)
 *     weighted in radius, so (solid angle) x (average) is the exact integral;
 *   - a shell whose inner edge is r = 0 gets zero irregular increment and
 *     zero <R^I> for l >= 2, where the r^2-weighted average of r^-(l+1)
 *     diverges (l = 0, 1 stay finite and are kept);
 *   - a merged (coarsened) block is one cell of the solve: its density is
 *     the solid-angle weighted mean of its members (the volume-weighted block
 *     average of Sec. 2.3 within one shell), its kernel is the solid-angle
 *     weighted mean of its members' kernels, and the block's potential is
 *     written to every member cell.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_PI 3.14159265358979323846264338327950288

/* index of (l, m) in a triangular [(L+1)(L+2)/2] array */
static inline int plm_index(int l, int m) { return l * (l + 1) / 2 + m; }

int oracle_n_modes(int lmax) { return (lmax + 1) * (lmax + 1); }

/* collapsed angular-moment index of (l, m, a); a = 0 cosine, a = 1 sine */
int oracle_mode_index(int l, int m, int a) {
  if (m == 0) return l * l;
  return l * l + 2 * m - 1 + a;
}

/*
 * Renormalised associated Legendre functions P~_l^m(cos th) for all
 * 0 <= m <= l <= lmax at polar angle th (Sec. 2.2).  Seeds:
 *   P~_m^m = (-1)^m sqrt((2m+1)/(4 pi (2m)!)) (2m-1)!! (1-x^2)^(m/2)
 * evaluated as (-1)^m sqrt((2m+1)/(4 pi)) prod_{i=1..m} sqrt((2i-1)/(2i)) sin th
 * (the same number: (2m-1)!!/sqrt((2m)!) = sqrt(prod (2i-1)/(2i)), and
 * (1-x^2)^(1/2) = sin th on [0, pi]);
 *   P~_{m+1}^m = x sqrt(2m+3) P~_m^m;
 *   P~_l^m = sqrt((4l^2-1)/(l^2-m^2)) [x P~_{l-1}^m
 *            - sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)) P~_{l-2}^m].
 */
void oracle_legendre(int lmax, double th, double *out) {
  const double x = cos(th), s = sin(th);
  for (int m = 0; m <= lmax; ++m) {
    double pmm = sqrt((2.0 * m + 1.0) / (4.0 * ORACLE_PI));
    for (int i = 1; i <= m; ++i) pmm *= sqrt((2.0 * i - 1.0) / (2.0 * i)) * s;
    if (m % 2 == 1) pmm = -pmm;
    out[plm_index(m, m)] = pmm;
    if (m + 1 > lmax) continue;
    double pm1 = x * sqrt(2.0 * m + 3.0) * pmm;
    out[plm_index(m + 1, m)] = pm1;
    double p2 = pmm, p1 = pm1;
    for (int l = m + 2; l <= lmax; ++l) {
      double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
      double b = sqrt(((double)(l - 1) * (l - 1) - (double)m * m) /
                      (4.0 * (l - 1) * (l - 1) - 1.0));
      double p = a * (x * p1 - b * p2);
      out[plm_index(l, m)] = p;
      p2 = p1;
      p1 = p;
    }
  }
}

/* cos th0 - cos th1 written without cancellation (trigonometric identity) */
static double dcos(double th0, double th1) {
  return 2.0 * sin(0.5 * (th0 + th1)) * sin(0.5 * (th1 - th0));
}

/*
 * Solid-angle weighted theta-cell average of every P~_l^m:
 *   <P~>_j = int_{th0}^{th1} P~(cos th) sin th dth / (cos th0 - cos th1),
 * integrated by Romberg: trapezoid rules on 2^k panels followed by
 * Richardson extrapolation, stopping when the diagonal changes by at most
 * 1e-14 of the bound sqrt((2l+1)/4pi)*(cos th0 - cos th1) for every (l, m)
 * (k >= 4), or at k = 20.  Returns the number of levels used.
 */
#define ROMBERG_KMAX 20
int oracle_theta_average(int lmax, double th0, double th1, double *out) {
  const int np = (lmax + 1) * (lmax + 2) / 2;
  double *R = (double *)malloc(sizeof(double) * (ROMBERG_KMAX + 1) * (ROMBERG_KMAX + 1) * np);
  double *f = (double *)malloc(sizeof(double) * np);
  double *tol = (double *)malloc(sizeof(double) * np);
  const double h0 = th1 - th0, w = dcos(th0, th1);
  for (int l = 0; l <= lmax; ++l)
    for (int m = 0; m <= l; ++m)
      tol[plm_index(l, m)] = 1e-14 * sqrt((2.0 * l + 1.0) / (4.0 * ORACLE_PI)) * w;
#define RR(k, j, p) R[((k) * (ROMBERG_KMAX + 1) + (j)) * np + (p)]
  /* level 0: trapezoid with one panel */
  oracle_legendre(lmax, th0, f);
  for (int p = 0; p < np; ++p) RR(0, 0, p) = 0.5 * h0 * f[p] * sin(th0);
  oracle_legendre(lmax, th1, f);
  for (int p = 0; p < np; ++p) RR(0, 0, p) += 0.5 * h0 * f[p] * sin(th1);
  int kused = ROMBERG_KMAX;
  for (int k = 1; k <= ROMBERG_KMAX; ++k) {
    const long npan = 1L << k;
    const double h = h0 / (double)npan;
    for (int p = 0; p < np; ++p) RR(k, 0, p) = 0.5 * RR(k - 1, 0, p);
    for (long q = 1; q < npan; q += 2) {
      const double th = th0 + h * (double)q;
      oracle_legendre(lmax, th, f);
      const double st = sin(th);
      for (int p = 0; p < np; ++p) RR(k, 0, p) += h * f[p] * st;
    }
    double pow4 = 1.0;
    for (int j = 1; j <= k; ++j) {
      pow4 *= 4.0;
      for (int p = 0; p < np; ++p)
        RR(k, j, p) = RR(k, j - 1, p) + (RR(k, j - 1, p) - RR(k - 1, j - 1, p)) / (pow4 - 1.0);
    }
    if (k >= 4) {
      int done = 1;
      for (int p = 0; p < np && done; ++p)
        if (fabs(RR(k, k, p) - RR(k - 1, k - 1, p)) > tol[p]) done = 0;
      if (done) {
        kused = k;
        break;
      }
    }
  }
  for (int p = 0; p < np; ++p) out[p] = RR(kused, kused, p) / w;
#undef RR
  free(R);
  free(f);
  free(tol);
  return kused;
}

/*
 * phi-cell averages of cos(m ph) and sin(m ph) over [ph0, ph1] from the
 * antiderivative: <cos> = (sin m ph1 - sin m ph0)/(m dph),
 * <sin> = (cos m ph0 - cos m ph1)/(m dph), both differences written as
 * products (trigonometric identities) so thin cells lose no digits;
 * m = 0 gives 1 and 0.
 */
void oracle_phi_average(int lmax, double ph0, double ph1, double *cavg, double *savg) {
  const double d = ph1 - ph0, mid = 0.5 * (ph0 + ph1);
  cavg[0] = 1.0;
  savg[0] = 0.0;
  for (int m = 1; m <= lmax; ++m) {
    const double half = sin(0.5 * m * d);
    cavg[m] = 2.0 * cos(m * mid) * half / (m * d);
    savg[m] = 2.0 * sin(m * mid) * half / (m * d);
  }
}

/*
 * b^p - a^p for 0 < a < b.  For a thin shell (|p ln(b/a)| < 1) the plain
 * difference cancels, so it is taken as a^p expm1(p log1p((b-a)/a)); for a
 * thick shell the rounding of the large exponent argument would dominate
 * instead, and the plain difference loses at most a factor 1/(1 - 1/e).
 */
static double pow_diff(double a, double b, double p) {
  const double x = p * log1p((b - a) / a);
  if (fabs(x) < 1.0) return pow(a, p) * expm1(x);
  return pow(b, p) - pow(a, p);
}

/*
 * Exact shell integrals for shell [r0, r1] and every l <= lmax:
 *   JR_l = int r^2 r^l dr = (r1^(l+3) - r0^(l+3))/(l+3),
 *   JI_l = int r^2 r^-(l+1) dr = (r1^(2-l) - r0^(2-l))/(2-l)   (ln(r1/r0) at l = 2),
 *   V3   = (r1^3 - r0^3)/3,
 * so that V3 <R^R>_l = JR_l and V3 <R^I>_l = JI_l are the Delta(r^3/3)-times-
 * cell-averaged kernel products of the edge recurrences.  For r0 = 0 the
 * irregular integral is finite only for l = 0, 1; JI_l for l >= 2 is set to 0
 * (documented convention).
 */
void oracle_radial(int lmax, double r0, double r1, double *JR, double *JI, double *V3) {
  if (r0 > 0.0) {
    *V3 = pow_diff(r0, r1, 3.0) / 3.0;
    for (int l = 0; l <= lmax; ++l) {
      JR[l] = pow_diff(r0, r1, l + 3.0) / (l + 3.0);
      if (l == 2)
        JI[l] = log1p((r1 - r0) / r0);
      else
        JI[l] = pow_diff(r0, r1, 2.0 - l) / (2.0 - l);
    }
  } else {
    *V3 = r1 * r1 * r1 / 3.0;
    for (int l = 0; l <= lmax; ++l) {
      JR[l] = pow(r1, l + 3.0) / (l + 3.0);
      JI[l] = (l == 0) ? 0.5 * r1 * r1 : (l == 1) ? r1 : 0.0;
    }
  }
}

/* number of blocks of class c (max block id + 1) */
static int class_nblocks(const int32_t *cb, int ncell) {
  int mx = -1;
  for (int q = 0; q < ncell; ++q)
    if (cb[q] > mx) mx = cb[q];
  return mx + 1;
}

/*
 * Angular tables for a mesh.  Outputs (any may be NULL):
 *   pavg  [ntheta][(L+1)(L+2)/2]   theta-cell averages of P~_l^m
 *   cavg, savg [nphi][L+1]          phi-cell averages of cos, sin (m ph)
 *   domega [ntheta*nphi]            cell solid angles
 *   akern [ntheta*nphi][nAM]        cell-averaged A_iAM
 * Returns the maximum number of Romberg levels used.
 */
int oracle_angular_tables(int ntheta, int nphi, int lmax, const double *th, const double *ph,
                          double *pavg, double *cavg, double *savg, double *domega,
                          double *akern) {
  const int np = (lmax + 1) * (lmax + 2) / 2, nam = oracle_n_modes(lmax);
  double *P = (double *)malloc(sizeof(double) * (size_t)ntheta * np);
  double *Cs = (double *)malloc(sizeof(double) * (size_t)nphi * (lmax + 1));
  double *Sn = (double *)malloc(sizeof(double) * (size_t)nphi * (lmax + 1));
  int kmax = 0;
#pragma omp parallel for schedule(dynamic) reduction(max : kmax)
  for (int j = 0; j < ntheta; ++j) {
    int k = oracle_theta_average(lmax, th[j], th[j + 1], P + (size_t)j * np);
    if (k > kmax) kmax = k;
  }
  for (int k = 0; k < nphi; ++k)
    oracle_phi_average(lmax, ph[k], ph[k + 1], Cs + (size_t)k * (lmax + 1), Sn + (size_t)k * (lmax + 1));
  if (pavg) memcpy(pavg, P, sizeof(double) * (size_t)ntheta * np);
  if (cavg) memcpy(cavg, Cs, sizeof(double) * (size_t)nphi * (lmax + 1));
  if (savg) memcpy(savg, Sn, sizeof(double) * (size_t)nphi * (lmax + 1));
  if (domega)
    for (int j = 0; j < ntheta; ++j)
      for (int k = 0; k < nphi; ++k)
        domega[(size_t)j * nphi + k] = dcos(th[j], th[j + 1]) * (ph[k + 1] - ph[k]);
  if (akern) {
#pragma omp parallel for
    for (int j = 0; j < ntheta; ++j)
      for (int k = 0; k < nphi; ++k) {
        double *row = akern + ((size_t)j * nphi + k) * nam;
        for (int l = 0; l <= lmax; ++l)
          for (int m = 0; m <= l; ++m) {
            const double p = P[(size_t)j * np + plm_index(l, m)];
            row[oracle_mode_index(l, m, 0)] = p * Cs[(size_t)k * (lmax + 1) + m];
            if (m > 0) row[oracle_mode_index(l, m, 1)] = p * Sn[(size_t)k * (lmax + 1) + m];
          }
      }
  }
  free(P);
  free(Cs);
  free(Sn);
  return kmax;
}

/*
 * Full solve.  Mesh: edges r[nr+1], th[ntheta+1], ph[nphi+1]; lmax; G.
 * Merging: nclasses = 0 means every angular cell is its own block; otherwise
 * shell_class[nr] selects a class and class_block[c][ntheta*nphi] gives each
 * angular cell's block id within class c.
 * rho and phi are [nr][ntheta][nphi] (phi fastest).  Optional outputs (may
 * be NULL): ang [nr][nAM] angular moments, interior / exterior [nr+1][nAM]
 * edge radial moments, coef [nr][nAM] the assembled expansion coefficients,
 * seconds[2] wall time of the table construction and of the solve proper.
 */
int oracle_solve(int nr, int ntheta, int nphi, int lmax, const double *r, const double *th,
                 const double *ph, double G, int nclasses, const int32_t *shell_class,
                 const int32_t *class_block, const double *rho, double *phi, double *ang,
                 double *interior, double *exterior, double *coef, double *seconds) {
  const int nam = oracle_n_modes(lmax), ncell = ntheta * nphi;
  const double fourpiG = 4.0 * ORACLE_PI * G;
  const double t_start = omp_get_wtime();

  /* angular tables on the fine cells */
  double *dom = (double *)malloc(sizeof(double) * ncell);
  double *afine = (double *)malloc(sizeof(double) * (size_t)ncell * nam);
  oracle_angular_tables(ntheta, nphi, lmax, th, ph, NULL, NULL, NULL, dom, afine);

  /* block tables per class: solid angle and solid-angle weighted mean kernel */
  const int ncls = nclasses > 0 ? nclasses : 1;
  int *nblk = (int *)malloc(sizeof(int) * ncls);
  int32_t **bmap = (int32_t **)malloc(sizeof(int32_t *) * ncls);
  double **bdom = (double **)malloc(sizeof(double *) * ncls);
  double **bker = (double **)malloc(sizeof(double *) * ncls);
  for (int c = 0; c < ncls; ++c) {
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * ncell);
    if (nclasses > 0)
      memcpy(map, class_block + (size_t)c * ncell, sizeof(int32_t) * ncell);
    else
      for (int q = 0; q < ncell; ++q) map[q] = q;
    const int nb = class_nblocks(map, ncell);
    double *bd = (double *)calloc((size_t)nb, sizeof(double));
    double *bk = (double *)calloc((size_t)nb * nam, sizeof(double));
    for (int q = 0; q < ncell; ++q) {
      const int b = map[q];
      bd[b] += dom[q];
      for (int n = 0; n < nam; ++n) bk[(size_t)b * nam + n] += dom[q] * afine[(size_t)q * nam + n];
    }
    for (int b = 0; b < nb; ++b)
      for (int n = 0; n < nam; ++n) bk[(size_t)b * nam + n] /= bd[b];
    nblk[c] = nb;
    bmap[c] = map;
    bdom[c] = bd;
    bker[c] = bk;
  }
  free(afine);
  const double t_tables = omp_get_wtime();

  /* angular moments: A[i][n] = sum_b dOmega_b <A_n>_b S_ib, S = 4 pi G rho_b */
  double *A = (double *)calloc((size_t)nr * nam, sizeof(double));
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < nr; ++i) {
    const int c = nclasses > 0 ? shell_class[i] : 0;
    const int nb = nblk[c];
    double *rb = (double *)calloc((size_t)nb, sizeof(double));
    for (int q = 0; q < ncell; ++q) rb[bmap[c][q]] += dom[q] * rho[(size_t)i * ncell + q];
    for (int b = 0; b < nb; ++b) rb[b] /= bdom[c][b]; /* block density */
    double *acc = A + (size_t)i * nam;
    for (int b = 0; b < nb; ++b) {
      const double w = bdom[c][b] * fourpiG * rb[b];
      const double *kb = bker[c] + (size_t)b * nam;
      for (int n = 0; n < nam; ++n) acc[n] += w * kb[n];
    }
    free(rb);
  }

  /* radial integrals and cell-averaged radial kernels */
  double *JR = (double *)malloc(sizeof(double) * (size_t)nr * (lmax + 1));
  double *JI = (double *)malloc(sizeof(double) * (size_t)nr * (lmax + 1));
  double *V3 = (double *)malloc(sizeof(double) * nr);
  for (int i = 0; i < nr; ++i)
    oracle_radial(lmax, r[i], r[i + 1], JR + (size_t)i * (lmax + 1), JI + (size_t)i * (lmax + 1), V3 + i);

  /* edge radial moments: outward (regular) and inward (irregular) */
  double *MR = (double *)calloc((size_t)(nr + 1) * nam, sizeof(double));
  double *MI = (double *)calloc((size_t)(nr + 1) * nam, sizeof(double));
  for (int l = 0; l <= lmax; ++l)
    for (int n = l * l; n < (l + 1) * (l + 1); ++n) {
      for (int i = 0; i < nr; ++i)
        MR[(size_t)(i + 1) * nam + n] = MR[(size_t)i * nam + n] + JR[(size_t)i * (lmax + 1) + l] * A[(size_t)i * nam + n];
      for (int i = nr - 1; i >= 0; --i)
        MI[(size_t)i * nam + n] = MI[(size_t)(i + 1) * nam + n] + JI[(size_t)i * (lmax + 1) + l] * A[(size_t)i * nam + n];
    }

  /* centre values and expansion coefficients of Eq. Solution */
  double *C = (double *)malloc(sizeof(double) * (size_t)nr * nam);
  for (int i = 0; i < nr; ++i)
    for (int l = 0; l <= lmax; ++l) {
      const double rr = JR[(size_t)i * (lmax + 1) + l] / V3[i];
      const double ri = JI[(size_t)i * (lmax + 1) + l] / V3[i];
      for (int n = l * l; n < (l + 1) * (l + 1); ++n) {
        const int m = (n == l * l) ? 0 : (n - l * l + 1) / 2;
        const double dm = (m == 0) ? 1.0 : 2.0;
        const double mic = 0.5 * (MI[(size_t)i * nam + n] + MI[(size_t)(i + 1) * nam + n]);
        const double mrc = 0.5 * (MR[(size_t)i * nam + n] + MR[(size_t)(i + 1) * nam + n]);
        C[(size_t)i * nam + n] = -dm / (2.0 * l + 1.0) * (rr * mic + ri * mrc);
      }
    }

  /* potential: Phi_ib = sum_n C[i][n] <A_n>_b, written to every member cell */
  if (phi) {
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < nr; ++i) {
      const int c = nclasses > 0 ? shell_class[i] : 0;
      const int nb = nblk[c];
      double *pb = (double *)malloc(sizeof(double) * nb);
      const double *ci = C + (size_t)i * nam;
      for (int b = 0; b < nb; ++b) {
        const double *kb = bker[c] + (size_t)b * nam;
        double s = 0.0;
        for (int n = 0; n < nam; ++n) s += ci[n] * kb[n];
        pb[b] = s;
      }
      for (int q = 0; q < ncell; ++q) phi[(size_t)i * ncell + q] = pb[bmap[c][q]];
      free(pb);
    }
  }

  if (seconds) {
    seconds[0] = t_tables - t_start;
    seconds[1] = omp_get_wtime() - t_tables;
  }
  if (ang) memcpy(ang, A, sizeof(double) * (size_t)nr * nam);
  if (interior) memcpy(interior, MR, sizeof(double) * (size_t)(nr + 1) * nam);
  if (exterior) memcpy(exterior, MI, sizeof(double) * (size_t)(nr + 1) * nam);
  if (coef) memcpy(coef, C, sizeof(double) * (size_t)nr * nam);

  for (int c = 0; c < ncls; ++c) {
    free(bmap[c]);
    free(bdom[c]);
    free(bker[c]);
  }
  free(nblk);
  free(bmap);
  free(bdom);
  free(bker);
  free(dom);
  free(A);
  free(JR);
  free(JI);
  free(V3);
  free(MR);
  free(MI);
  free(C);
  return 0;
}

/* Gradient of the potential for the gravitational source terms (Sec. 3, the
 * source vector of the balance equations with its -rho grad Phi and
 * -rho v . grad Phi entries, and the sentence after it: each component is
 * the simplest centred difference, from the two nearest neighbours).
 *
 * Readings: the components are the coordinate derivatives dPhi/dr,
 * dPhi/dtheta, dPhi/dphi at cell centres (the covariant components that the
 * covector momentum source uses); a cell's coordinate is the midpoint of its
 * edges; the difference is (Phi(next) - Phi(previous)) / (x(next) -
 * x(previous)); where a neighbour is missing (first or last shell, first or
 * last theta row, phi when the phi edges do not close the circle) the cell
 * itself takes its place (one-sided difference); phi wraps around when its
 * edges span 2 pi; a dimension with a single cell has zero derivative. */
static double mid(const double *e, int i) { return 0.5 * (e[i] + e[i + 1]); }

static void neighbours(int i, int n, int *lo, int *hi) {
  *lo = i > 0 ? i - 1 : i;
  *hi = i < n - 1 ? i + 1 : i;
}

void oracle_gradient(int nr, int ntheta, int nphi, const double *r, const double *th, const double *ph,
                     const double *phi, double *d_r, double *d_th, double *d_ph) {
  const double two_pi = 2.0 * ORACLE_PI;
  const int periodic = fabs((ph[nphi] - ph[0]) - two_pi) <= 1e-12 * two_pi;
  const long ncell = (long)ntheta * nphi;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < nr; ++i) {
    for (int j = 0; j < ntheta; ++j) {
      for (int k = 0; k < nphi; ++k) {
        const long q = (long)i * ncell + (long)j * nphi + k;
        int lo, hi;
        /* radius */
        if (nr == 1) {
          d_r[q] = 0.0;
        } else {
          neighbours(i, nr, &lo, &hi);
          d_r[q] = (phi[(long)hi * ncell + (long)j * nphi + k] - phi[(long)lo * ncell + (long)j * nphi + k]) /
                   (mid(r, hi) - mid(r, lo));
        }
        /* polar angle */
        if (ntheta == 1) {
          d_th[q] = 0.0;
        } else {
          neighbours(j, ntheta, &lo, &hi);
          d_th[q] = (phi[(long)i * ncell + (long)hi * nphi + k] - phi[(long)i * ncell + (long)lo * nphi + k]) /
                    (mid(th, hi) - mid(th, lo));
        }
        /* azimuth */
        if (nphi == 1) {
          d_ph[q] = 0.0;
        } else if (periodic) {
          const int kl = (k + nphi - 1) % nphi, kh = (k + 1) % nphi;
          double xl = mid(ph, kl), xh = mid(ph, kh);
          if (k == 0) xl -= two_pi;
          if (k == nphi - 1) xh += two_pi;
          d_ph[q] = (phi[(long)i * ncell + (long)j * nphi + kh] - phi[(long)i * ncell + (long)j * nphi + kl]) / (xh - xl);
        } else {
          neighbours(k, nphi, &lo, &hi);
          d_ph[q] = (phi[(long)i * ncell + (long)j * nphi + hi] - phi[(long)i * ncell + (long)j * nphi + lo]) /
                    (mid(ph, hi) - mid(ph, lo));
        }
      }
    }
  }
}

/* Threads of the OpenMP regions above (n >= 1); returns the count in effect.
   Used by the benchmark's CPU baseline to time the oracle single-threaded. */
int oracle_set_threads(int n) {
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
}
