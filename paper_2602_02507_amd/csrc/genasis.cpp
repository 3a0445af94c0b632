// GenASiS mesh with automatic angular coarsening (Sec. 2.1), host side.
//
// Radial law: N_core shells of uniform width dr_min = r_core / N_core inside
// r_core, then each shell wider than the previous one by the factor
// (1 + 1/N_core) (dr proportional to r, constant polar/radial aspect ratio);
// N_core = N_theta / core_ratio to the nearest integer, N_r = floor(R_radial
// N_theta).  Angular cells of a shell narrower than the coarsening width are
// grouped into aligned power-of-two blocks: the theta group from r dtheta,
// then, per theta block, the phi group from r sin(theta) dphi of its row
// nearest the axis; both at the cell centre and capped at the largest power
// of two dividing the cell count.  Shells with equal patterns share a class.
#include <cmath>
#include <map>
#include <vector>

#include "../../include/mpole.h"
#include "mpole_internal.h"

using namespace mpole;

namespace {

struct Pattern {
  int ct = 1;                // theta group size
  std::vector<int> cp;       // phi group size of each theta block
  bool operator<(const Pattern &o) const { return ct != o.ct ? ct < o.ct : cp < o.cp; }
};

struct Layout {
  int nr = 0, nt = 0, np = 0, ncore = 0;
  double r_core = 0.0, dr = 0.0;
  std::vector<double> r, th, ph;
  std::vector<int> shell_class;
  std::vector<const Pattern *> shell_pattern;
  std::vector<Pattern> classes;   // in order of first shell
};

int pow2_cap(int n) {
  int c = 1;
  while (n % (2 * c) == 0) c *= 2;
  return c;
}

// smallest power of two c with c * width >= dr, at most cap
int group_size(double width, double dr, int cap) {
  int c = 1;
  while ((double)c * width < dr && c < cap) c *= 2;
  return c;
}

int layout(const mpole_genasis *g, Layout &o) {
  if (!g) return fail(MPOLE_ERR_INVALID, "genasis parameters are null");
  if (g->dims < 1 || g->dims > 3) return fail(MPOLE_ERR_INVALID, "dims %d not in 1..3", g->dims);
  if (g->ntheta < 1 || g->ntheta > 65536) return fail(MPOLE_ERR_INVALID, "ntheta %d not in 1..65536", g->ntheta);
  if (!std::isfinite(g->r_core) || !(g->r_core > 0.0)) return fail(MPOLE_ERR_INVALID, "r_core must be finite and > 0");
  if (!std::isfinite(g->r_radial) || !(g->r_radial > 0.0))
    return fail(MPOLE_ERR_INVALID, "r_radial must be finite and > 0");
  if (!std::isfinite(g->core_ratio) || g->core_ratio < 0.0)
    return fail(MPOLE_ERR_INVALID, "core_ratio must be finite and >= 0");
  if (!std::isfinite(g->dr_coarsen) || g->dr_coarsen < 0.0)
    return fail(MPOLE_ERR_INVALID, "dr_coarsen must be finite and >= 0");
  const double ratio = g->core_ratio > 0.0 ? g->core_ratio : 32.0 / 25.0;
  const double ncore = std::floor((double)g->ntheta / ratio + 0.5);
  const double nr = std::floor(g->r_radial * (double)g->ntheta + 1e-9);
  if (!(ncore >= 1.0) || ncore > (double)(1 << 20)) return fail(MPOLE_ERR_INVALID, "N_core = %.0f not in 1..2^20", ncore);
  if (!(nr >= 1.0) || nr > (double)(1 << 20)) return fail(MPOLE_ERR_INVALID, "N_r = %.0f not in 1..2^20", nr);
  o.ncore = (int)ncore;
  o.nr = (int)nr;
  o.nt = g->dims >= 2 ? g->ntheta : 1;
  o.np = g->dims == 3 ? 2 * g->ntheta : 1;
  o.r_core = g->r_core;
  o.dr = g->dr_coarsen > 0.0 ? g->dr_coarsen : g->r_core / (double)o.ncore;

  o.r.resize(o.nr + 1);
  for (int i = 0; i <= o.nr; ++i)
    o.r[i] = i <= o.ncore ? g->r_core * (double)i / (double)o.ncore
                          : g->r_core * std::pow(1.0 + 1.0 / (double)o.ncore, (double)(i - o.ncore));
  if (!std::isfinite(o.r[o.nr]) || o.r[o.nr] > 1e290)
    return fail(MPOLE_ERR_RANGE, "outer radius overflows (N_r %d, N_core %d)", o.nr, o.ncore);
  o.th.resize(o.nt + 1);
  for (int j = 0; j <= o.nt; ++j) o.th[j] = kPi * (double)j / (double)o.nt;
  o.ph.resize(o.np + 1);
  for (int k = 0; k <= o.np; ++k) o.ph[k] = 2.0 * kPi * (double)k / (double)o.np;

  const double dth = kPi / (double)o.nt, dph = 2.0 * kPi / (double)o.np;
  const int cap_t = pow2_cap(o.nt), cap_p = pow2_cap(o.np);
  std::vector<double> sin_c(o.nt);
  for (int j = 0; j < o.nt; ++j) {
    const double thc = 0.5 * (kPi * (double)j / (double)o.nt + kPi * (double)(j + 1) / (double)o.nt);
    sin_c[j] = std::sin(thc);
  }
  std::map<Pattern, int> index;
  std::vector<Pattern> pats(o.nr);
  o.shell_class.resize(o.nr);
  for (int i = 0; i < o.nr; ++i) {
    const double rc = 0.5 * (o.r[i] + o.r[i + 1]);
    Pattern &p = pats[i];
    p.ct = group_size(rc * dth, o.dr, cap_t);
    for (int j0 = 0; j0 < o.nt; j0 += p.ct) {
      int need = 1;
      for (int j = j0; j < j0 + p.ct; ++j) need = std::max(need, group_size(rc * sin_c[j] * dph, o.dr, cap_p));
      p.cp.push_back(need);
    }
    auto it = index.find(p);
    if (it == index.end()) {
      it = index.emplace(p, (int)o.classes.size()).first;
      o.classes.push_back(p);
    }
    o.shell_class[i] = it->second;
  }
  return MPOLE_OK;
}

}  // namespace

extern "C" {

int mpole_genasis_shape(const mpole_genasis *g, int32_t *nr, int32_t *ntheta, int32_t *nphi, int32_t *ncore,
                        int32_t *nclasses) {
  Layout o;
  const int rc = layout(g, o);
  if (rc != MPOLE_OK) return rc;
  if (nr) *nr = o.nr;
  if (ntheta) *ntheta = o.nt;
  if (nphi) *nphi = o.np;
  if (ncore) *ncore = o.ncore;
  if (nclasses) *nclasses = (int32_t)o.classes.size();
  return ok();
}

int mpole_genasis_build(const mpole_genasis *g, double *r_edges, double *theta_edges, double *phi_edges,
                        int32_t *shell_class, int32_t *class_block, int32_t *c_theta, int32_t *c_phi) {
  if (!r_edges || !theta_edges || !phi_edges || !shell_class || !class_block)
    return fail(MPOLE_ERR_INVALID, "an output array is null");
  Layout o;
  const int rc = layout(g, o);
  if (rc != MPOLE_OK) return rc;
  std::copy(o.r.begin(), o.r.end(), r_edges);
  std::copy(o.th.begin(), o.th.end(), theta_edges);
  std::copy(o.ph.begin(), o.ph.end(), phi_edges);
  std::copy(o.shell_class.begin(), o.shell_class.end(), shell_class);
  const size_t ncell = (size_t)o.nt * o.np;
  for (size_t c = 0; c < o.classes.size(); ++c) {
    const Pattern &p = o.classes[c];
    int32_t *m = class_block + c * ncell;
    int nb = 0;
    for (int jb = 0, j0 = 0; j0 < o.nt; ++jb, j0 += p.ct)
      for (int k0 = 0; k0 < o.np; k0 += p.cp[jb], ++nb)
        for (int j = j0; j < j0 + p.ct; ++j)
          for (int k = k0; k < k0 + p.cp[jb]; ++k) m[(size_t)j * o.np + k] = nb;
  }
  for (int i = 0; i < o.nr; ++i) {
    const Pattern &p = o.classes[o.shell_class[i]];
    if (c_theta) c_theta[i] = p.ct;
    if (c_phi)
      for (int j = 0; j < o.nt; ++j) c_phi[(size_t)i * o.nt + j] = p.cp[j / p.ct];
  }
  return ok();
}

}  // extern "C"
