// Host side of the C ABI declared in include/mpole.h: mesh validation, the
// per-class block maps (CSR), workspace layout, table construction at bind
// time and the kernel sequence of one solve.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mpole.h"
#include "mpole_internal.h"

using namespace mpole;

namespace mpole {

// Per-solve scratch of mpole_solve_static: one copy of this array on every
// device the library runs on, held until the process ends.  Every static
// solve on a device uses it from the start (it keeps the last solve's
// contents; the solve writes everything before reading it), so static
// solves that overlap on one device race.
constexpr size_t kScratchBytes = size_t(256) << 20;
__device__ __align__(256) char scratch[kScratchBytes];

}  // namespace mpole

namespace mpole {

// fixed-size per-thread message buffer: setting it never allocates
thread_local char g_error[512];

int fail(int code, const char *fmt, ...) {
  char buf[sizeof g_error];   // formatted apart, so that g_error may be an argument
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  std::memcpy(g_error, buf, sizeof buf);
  return code;
}

int ok() {
  g_error[0] = '\0';
  return MPOLE_OK;
}

}  // namespace mpole

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
int round_up(int x, int m) { return (x + m - 1) / m * m; }

// 16-point Gauss-Legendre rule on [-1, 1] by Newton iteration on P_16.
GaussRule make_gauss_rule() {
  GaussRule g{};
  const int n = kGaussNodes;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    g.x[i] = x;
    g.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return g;
}

struct ClassHost {
  std::vector<int32_t> rows, moff, mem;
  std::vector<int32_t> rect;  // 4 per block when every block is a rectangle in (j, k)
  std::vector<int32_t> span0;  // per block span: first cell when the span is a run of single cells, else -1
  std::vector<int32_t> pspan0; // the same per packing span of pairs (rep cells)
  std::vector<int32_t> sep_src, sep_avg;   // separable path: blocks on merged rows, blocks with > 1 member
  std::vector<int32_t> large, lidx;        // blocks of more than kLargeBlock cells; index in `large` per block
  std::vector<int32_t> bands;              // theta bands (j0, nj, nk, kind), or empty
  std::vector<int32_t> bcast;              // indices of the bands of merged blocks (kind 1)
  std::vector<int32_t> mirb;               // mirror block of each block (theta -> pi - theta), or empty
  std::vector<int32_t> pairs;              // (rep, mir) per pair
  std::vector<int32_t> ptasks;             // band packing tasks (j0, nj, nk, q0), or empty
  int npair = 0, npair_pad = 0, npack = 0;
  size_t off_ptasks = 0;
  size_t off_pairs = 0, off_tm = 0, off_te = 0, off_pack_o = 0, off_ppacks_o = 0;
  size_t off_lidx = 0, off_bands = 0, off_bcast = 0;
  size_t off_sep_src = 0, off_sep_avg = 0;
  size_t off_span0 = 0, off_pspan0 = 0;
  size_t off_rect = 0;
  int nblocks = 0, nblocks_pad = 0, splits = 1, kchunk = 0;
  int m_tiles_mom = 0, m_tiles_exp = 0, n_tiles_mom = 0, n_tiles_exp = 0, wg_mom_begin = 0, wg_exp_begin = 0;
  size_t off_rows = 0, off_moff = 0, off_mem = 0, off_table = 0, off_pack = 0, off_partial = 0;
  size_t off_tplanes = 0, off_ttplanes = 0, off_ppacks = 0, off_pscale = 0, off_tcol0 = 0, off_wsum = 0, off_tsum = 0;
};

// planes of a split precision (0 for FP64)
int n_planes(int precision) {
  return precision == MPOLE_BF16X3 ? 3 : precision == MPOLE_FP16X2 ? 2 : 0;
}

}  // namespace

struct mpole_plan_t {
  int nr = 0, nt = 0, np = 0, L = 0, nam = 0, namp = 0, ncell = 0, ncls = 0, precision = 0;
  double G = 1.0;
  std::vector<double> r, th, ph;
  std::vector<int32_t> shell_class, shell_row;
  std::vector<ClassHost> cls;
  size_t ws_bytes = 0;
  size_t off_r = 0, off_th = 0, off_ph = 0, off_shell_class = 0, off_shell_row = 0, off_classes = 0;
  size_t off_wrow = 0, off_dphi = 0;
  size_t off_pavg = 0, off_trig = 0, off_weight = 0, off_jr = 0, off_ji = 0, off_rr = 0, off_ri = 0;
  size_t off_ang = 0, off_coef = 0, off_edge_r = 0, off_edge_i = 0, off_cplanes = 0, off_cscale = 0, off_mono = 0, off_max = 0;
  int mono_stride = 1;
  int phi_periodic = 0;   // phi edges close the circle (gradient wraps around)
  bool sep = false;       // separable contractions
  bool sep_bf16 = false;  // separable with BF16 x3 phi transforms
  int tpad = 0;           // separable: trig modes 2L+1 padded to 16
  bool any_alt = false;   // separable: some row holds a merged block
  std::vector<uint8_t> rowalt;   // separable: [nr][ntheta] rows read from the block means
  size_t off_tw = 0, off_pw = 0, off_pt = 0, off_shat = 0, off_rowalt = 0, off_f = 0, off_g = 0, off_dom = 0;
  size_t off_twf = 0, off_ttf = 0;
  int ks_a = 0, mt_a = 0, ks_s = 0, nt_s = 0;   // BF16 x3 separable: fragment table shapes
  SepDev sdev{};
  std::vector<SepClass> scls;
  size_t off_scls = 0;
  int max_src = 0, max_avg = 0;   // separable: longest per-class block lists
  // blocks of more than kLargeBlock cells over all shells: (shell, block) items and each shell's first item
  std::vector<int32_t> litems, lbase, lchunks;
  size_t off_litems = 0, off_lbase = 0, off_lsum = 0, off_lchunks = 0, off_lpart = 0;
  size_t off_shift = 0, off_tsum_part = 0;
  int nplanes = 0, tm_mom = 64, tm_exp = 64, tile_n = 64, kpad = 16, moment_target = 0;
  // mirror fold of the dense contractions: mode columns of both contractions
  bool fold = false;
  int namp_m = 0, odd_m0 = 0, namp_e = 0, odd_e0 = 0;
  std::vector<int32_t> pos_m, perm_m, perm_e;
  size_t off_pos_m = 0, off_perm_m = 0, off_perm_e = 0, off_coef_e = 0;
  int scan_modes = kScanModesWide;   // modes per radial-scan workgroup
  size_t off_plandev = 0, off_prefix = 0, off_bcast_items = 0;
  size_t solve_off = 0, solve_bytes = 0;        // per-solve region: start in the workspace, size
  size_t off_plandev_s = 0, off_classes_s = 0;  // device views of the static-scratch solve
  int wg_mom = 0, wg_exp = 0;
  GaussRule rule{};
  // per-phase timing events (host objects), recorded while timing is on
  bool timing = false;
  std::vector<hipEvent_t> ev;  // pairs: [2k] before, [2k+1] after launch k
  std::vector<int> ev_phase;
  size_t ev_used = 0;
  // bound state
  bool bound = false;
  char *ws = nullptr;
  PlanDev dev{};
  std::vector<ClassDev> cdev;
  // mpole_solve_static: the same views with the per-solve region in the
  // static scratch array of the bound device (valid when static_ok)
  bool static_ok = false;
  int static_dev = -1;
  PlanDev dev_s{};
  std::vector<ClassDev> cdev_s;
  SepDev sdev_s{};
  std::vector<int32_t> prefix;   // [PH_COUNT][2] single-plan phase prefix sums
  std::vector<int32_t> bcast_items; // broadcast workgroups: (shell, first band) pairs
};

namespace {

int check_edges(const char *name, const double *e, int n, double lo, double hi) {
  if (!e) return fail(MPOLE_ERR_INVALID, "%s is null", name);
  for (int i = 0; i <= n; ++i)
    if (!std::isfinite(e[i])) return fail(MPOLE_ERR_INVALID, "%s[%d] is not finite", name, i);
  for (int i = 0; i < n; ++i)
    if (!(e[i + 1] > e[i])) return fail(MPOLE_ERR_INVALID, "%s is not strictly increasing at %d", name, i);
  if (e[0] < lo || e[n] > hi) return fail(MPOLE_ERR_INVALID, "%s leaves [%g, %g]", name, lo, hi);
  return MPOLE_OK;
}

// Split-K choice for the moment contraction: spread about `target` workgroups
// over the classes in proportion to their work, at least one K step (kpad)
// per split.
constexpr int kMaxSplitChunk = 2048;

void choose_splits(mpole_plan_t &p, int target) {
  double total = 0.0;
  for (auto &c : p.cls) total += (double)c.rows.size() * c.npair_pad;
  for (auto &c : p.cls) {
    const int tiles = c.m_tiles_mom * c.n_tiles_mom;
    const double share = total > 0 ? target * (double)c.rows.size() * c.npair_pad / total : 1.0;
    int s = (int)std::lround(share / std::max(tiles, 1));
    // FP32-accumulated contractions: no split longer than kMaxSplitChunk
    // pairs, so the rounding of one accumulator chain stays bounded; the
    // partials are summed in FP64
    if (p.precision != MPOLE_FP64) s = std::max(s, (c.npair_pad + kMaxSplitChunk - 1) / kMaxSplitChunk);
    s = std::max(1, std::min(s, c.npair_pad / p.kpad));
    c.kchunk = round_up((c.npair_pad + s - 1) / s, p.kpad);
    c.splits = (c.npair_pad + c.kchunk - 1) / c.kchunk;
  }
}

void layout_plan(mpole_plan_t *p, int target);
void bcast_layout(mpole_plan_t *p);
int default_target(const mpole_plan_t *p);

// Band packing tasks of a class whose blocks form theta bands of merged
// blocks (at most kLargeBlock cells) and single-cell rows: one task per
// merged band that is its own rep (north of its mirror, or its own mirror),
// and per run of up to kBandCopyRows single-cell rows that are all north of
// their mirror rows or one row that is its own mirror (unfolded: every band,
// rows as they come).  Each task's pairs must be consecutive: q0 + k / nk for
// a merged band, q0 + (j - j0) nphi + k for single-cell rows; any other map
// keeps the span path (empty list).
void build_pack_tasks(const mpole_plan_t *p, ClassHost &C) {
  C.ptasks.clear();
  if (C.bands.empty()) return;
  std::vector<int32_t> id(p->ncell), qb(C.nblocks, -1);
  for (int b = 0; b < C.nblocks; ++b)
    for (int e = C.moff[b]; e < C.moff[b + 1]; ++e) id[C.mem[e]] = b;
  for (int q = 0; q < C.npair; ++q) qb[C.pairs[2 * q]] = q;
  const int nt = p->nt, np = p->np;
  std::vector<int32_t> t;
  auto pair_at = [&](int j, int k) { return qb[id[(size_t)j * np + k]]; };
  for (size_t x = 0; x + 3 < C.bands.size(); x += 4) {
    const int j0 = C.bands[x], nj = C.bands[x + 1], nk = C.bands[x + 2], kind = C.bands[x + 3];
    if (kind == 2) return;
    if (kind == 1) {
      const int mj0 = nt - j0 - nj;   // first row of the mirror band
      if (p->fold && mj0 < j0) continue;
      const int q0 = pair_at(j0, 0);
      for (int k = 0; k < np; ++k)
        if (q0 < 0 || pair_at(j0, k) != q0 + k / nk) return;
      t.insert(t.end(), {j0, nj, nk, q0});
      continue;
    }
    // single-cell rows: runs of rows that are reps of pairs (or their own mirror)
    for (int j = j0; j < j0 + nj;) {
      const int mj = nt - 1 - j;
      if (p->fold && mj < j) { ++j; continue; }
      int n = 1;
      if (!p->fold || mj > j)
        while (j + n < j0 + nj && n < kBandCopyRows && (!p->fold || nt - 1 - (j + n) > j + n)) ++n;
      const int q0 = pair_at(j, 0);
      for (int r = 0; r < n; ++r)
        for (int k = 0; k < np; ++k)
          if (q0 < 0 || pair_at(j + r, k) != q0 + r * np + k) return;
      t.insert(t.end(), {j, n, 1, q0});
      j += n;
    }
  }
  C.ptasks = t;
}

int build_plan(const mpole_mesh *m, mpole_plan_t *p) {
  if (!m) return fail(MPOLE_ERR_INVALID, "mesh is null");
  if (m->nr < 1 || m->ntheta < 1 || m->nphi < 1)
    return fail(MPOLE_ERR_INVALID, "mesh sizes must be >= 1 (nr=%d ntheta=%d nphi=%d)", m->nr, m->ntheta, m->nphi);
  if (m->lmax < 0) return fail(MPOLE_ERR_INVALID, "lmax must be >= 0");
  if (m->lmax > MPOLE_LMAX_MAX) return fail(MPOLE_ERR_UNSUPPORTED, "lmax %d above %d", m->lmax, MPOLE_LMAX_MAX);
  if (m->precision != MPOLE_FP64 && m->precision != MPOLE_BF16X3 && m->precision != MPOLE_FP16X2 &&
      m->precision != MPOLE_FP64_SEPARABLE && m->precision != MPOLE_BF16X3_SEPARABLE)
    return fail(MPOLE_ERR_UNSUPPORTED, "unknown precision %d", m->precision);
  if (!std::isfinite(m->G)) return fail(MPOLE_ERR_INVALID, "G is not finite");
  const long long ncell = (long long)m->ntheta * m->nphi;
  if (ncell > (1LL << 30) || (long long)m->nr * ncell > (1LL << 40))
    return fail(MPOLE_ERR_INVALID, "mesh too large");
  int rc;
  if ((rc = check_edges("r_edges", m->r_edges, m->nr, 0.0, INFINITY))) return rc;
  if ((rc = check_edges("theta_edges", m->theta_edges, m->ntheta, 0.0, kPi * (1 + 1e-15)))) return rc;
  if ((rc = check_edges("phi_edges", m->phi_edges, m->nphi, -INFINITY, INFINITY))) return rc;
  if (m->phi_edges[m->nphi] - m->phi_edges[0] > 2 * kPi * (1 + 1e-15))
    return fail(MPOLE_ERR_INVALID, "phi_edges span more than 2 pi");
  // FP64 range of r^(l+3) and r^(2-l) for l <= lmax on every nonzero edge
  const double pmax = std::max(m->lmax + 3.0, std::fabs(2.0 - m->lmax));
  for (int i = 0; i <= m->nr; ++i) {
    const double r = m->r_edges[i];
    if (r > 0.0 && std::fabs(std::log10(r)) * pmax > 290.0)
      return fail(MPOLE_ERR_RANGE, "r_edges[%d] = %g: r^%g leaves the FP64 range", i, r, pmax);
  }
  if (m->nclasses < 0) return fail(MPOLE_ERR_INVALID, "nclasses < 0");
  if (m->nclasses > 0 && (!m->shell_class || !m->class_block))
    return fail(MPOLE_ERR_INVALID, "shell_class and class_block are required when nclasses > 0");

  p->nr = m->nr;
  p->nt = m->ntheta;
  p->np = m->nphi;
  p->L = m->lmax;
  p->nam = (m->lmax + 1) * (m->lmax + 1);
  p->kpad = kPadF64;
  p->namp = round_up(p->nam, p->kpad);
  p->scan_modes = p->namp / kScanModesWide >= kScanWideMinWgs ? kScanModesWide : kScanModesNarrow;
  p->ncell = (int)ncell;
  p->precision = m->precision;
  p->nplanes = n_planes(m->precision);
  p->sep = m->precision == MPOLE_FP64_SEPARABLE || m->precision == MPOLE_BF16X3_SEPARABLE;
  p->sep_bf16 = m->precision == MPOLE_BF16X3_SEPARABLE;
  p->tpad = round_up(2 * m->lmax + 1, 16);
  // theta edges symmetric about the equator (the mirror fold's first condition)
  bool theta_sym = true;
  for (int j = 0; j <= m->ntheta && theta_sym; ++j)
    theta_sym = std::fabs(m->theta_edges[j] + m->theta_edges[m->ntheta - j] - kPi) <= 1e-13 * kPi;
  // output tiles of the contraction kernels: 64 x 64 (f64 MFMA); 128 x 128
  // (split; the height may be tuned to 64)
  p->tm_mom = p->tm_exp = p->nplanes ? 128 : 64;
  p->tile_n = p->nplanes ? 128 : 64;
  p->G = m->G;
  p->r.assign(m->r_edges, m->r_edges + m->nr + 1);
  p->th.assign(m->theta_edges, m->theta_edges + m->ntheta + 1);
  p->ph.assign(m->phi_edges, m->phi_edges + m->nphi + 1);
  p->phi_periodic = std::fabs((p->ph[p->np] - p->ph[0]) - 2.0 * kPi) <= 1e-12 * 2.0 * kPi;
  p->ncls = m->nclasses > 0 ? m->nclasses : 1;
  p->cls.assign(p->ncls, ClassHost{});
  p->shell_class.assign(p->nr, 0);
  p->shell_row.assign(p->nr, 0);
  for (int i = 0; i < p->nr; ++i) {
    const int c = m->nclasses > 0 ? m->shell_class[i] : 0;
    if (c < 0 || c >= p->ncls) return fail(MPOLE_ERR_INVALID, "shell_class[%d] = %d out of range", i, c);
    p->shell_class[i] = c;
    p->shell_row[i] = (int)p->cls[c].rows.size();
    p->cls[c].rows.push_back(i);
  }
  for (int c = 0; c < p->ncls; ++c) {
    ClassHost &C = p->cls[c];
    std::vector<int32_t> id(p->ncell);
    if (m->nclasses > 0) {
      std::memcpy(id.data(), m->class_block + (size_t)c * p->ncell, sizeof(int32_t) * p->ncell);
    } else {
      for (int q = 0; q < p->ncell; ++q) id[q] = q;
    }
    int nb = 0;
    for (int q = 0; q < p->ncell; ++q) {
      if (id[q] < 0 || id[q] >= p->ncell)
        return fail(MPOLE_ERR_INVALID, "class_block[%d][%d] = %d out of range", c, q, id[q]);
      nb = std::max(nb, id[q] + 1);
    }
    std::vector<int32_t> count(nb, 0);
    for (int q = 0; q < p->ncell; ++q) ++count[id[q]];
    for (int b = 0; b < nb; ++b)
      if (count[b] == 0) return fail(MPOLE_ERR_INVALID, "class %d: block id %d unused (ids must be dense)", c, b);
    C.nblocks = nb;
    C.nblocks_pad = round_up(nb, p->kpad);
    C.moff.assign(nb + 1, 0);
    for (int b = 0; b < nb; ++b) C.moff[b + 1] = C.moff[b] + count[b];
    C.mem.assign(p->ncell, 0);
    std::vector<int32_t> fillp(C.moff.begin(), C.moff.end() - 1);
    for (int q = 0; q < p->ncell; ++q) C.mem[fillp[id[q]]++] = q;   // ascending q per block
    // rectangle descriptors: a block is a rectangle when its member count
    // equals the area of its bounding box in (theta row, phi column)
    C.rect.assign(4 * (size_t)nb, 0);
    bool rect_ok = true;
    for (int b = 0; b < nb && rect_ok; ++b) {
      int j0 = p->nt, j1 = -1, k0 = p->np, k1 = -1;
      for (int e = C.moff[b]; e < C.moff[b + 1]; ++e) {
        const int j = C.mem[e] / p->np, k = C.mem[e] % p->np;
        j0 = std::min(j0, j); j1 = std::max(j1, j);
        k0 = std::min(k0, k); k1 = std::max(k1, k);
      }
      if ((j1 - j0 + 1) * (k1 - k0 + 1) != C.moff[b + 1] - C.moff[b]) rect_ok = false;
      C.rect[4 * b] = j0;
      C.rect[4 * b + 1] = k0;
      C.rect[4 * b + 2] = j1 - j0 + 1;
      C.rect[4 * b + 3] = k1 - k0 + 1;
    }
    if (!rect_ok) C.rect.clear();
    // theta bands (the layout power-of-two coarsening produces): rows
    // [j, j + nj) whose blocks are all nj x nk rectangles at phi columns that
    // are multiples of nk; single-cell rows are merged into copy bands
    C.bands.clear();
    if (!C.rect.empty()) {
      bool ok = true;
      for (int j = 0; j < p->nt && ok;) {
        const int b = id[(size_t)j * p->np];
        const int nj = C.rect[4 * b + 2], nk = C.rect[4 * b + 3];
        ok = C.rect[4 * b] == j && C.rect[4 * b + 1] == 0 && p->np % nk == 0 && j + nj <= p->nt;
        for (int jj = j; jj < j + nj && ok; ++jj)
          for (int k = 0; k < p->np && ok; ++k) {
            const int bb = id[(size_t)jj * p->np + k];
            ok = C.rect[4 * bb] == j && C.rect[4 * bb + 1] == k / nk * nk && C.rect[4 * bb + 2] == nj &&
                 C.rect[4 * bb + 3] == nk;
          }
        const int kind = nj * nk == 1 ? 0 : nj * nk > kLargeBlock ? 2 : 1;
        if (kind == 1 && (nk > 64 || (nk & (nk - 1)) != 0)) ok = false;
        if (!ok) break;
        const size_t nb4 = C.bands.size();
        if (kind == 0 && nb4 > 0 && C.bands[nb4 - 1] == 0 && C.bands[nb4 - 3] < kBandRows &&
            C.bands[nb4 - 4] + C.bands[nb4 - 3] == j) {
          ++C.bands[nb4 - 3];
        } else {
          C.bands.insert(C.bands.end(), {j, nj, nk, kind});
        }
        j += nj;
      }
      if (!ok) C.bands.clear();
    }
    C.bcast.clear();
    for (size_t x = 0; x + 3 < C.bands.size(); x += 4)
      if (C.bands[x + 3] == 1) C.bcast.push_back((int32_t)(x / 4));
    // mirror image of every block about the equator (row j -> ntheta-1-j),
    // when the map is symmetric: the mirror cells of a block's members are
    // exactly the members of one block
    C.mirb.clear();
    if (theta_sym) {
      C.mirb.assign(nb, -1);
      auto mcell = [&](int q) { return (p->nt - 1 - q / p->np) * p->np + q % p->np; };
      for (int b = 0; b < nb; ++b) C.mirb[b] = id[mcell(C.mem[C.moff[b]])];
      bool sym = true;
      for (int q = 0; q < p->ncell && sym; ++q) sym = id[mcell(q)] == C.mirb[id[q]];
      if (!sym) C.mirb.clear();
    }
    // blocks too large for one thread: a workgroup each (launch_large)
    C.large.clear();
    for (int b = 0; b < nb; ++b)
      if (C.moff[b + 1] - C.moff[b] > kLargeBlock) C.large.push_back(b);
    C.lidx.clear();
    if (!C.large.empty()) {
      C.lidx.assign(nb, -1);
      for (size_t l = 0; l < C.large.size(); ++l) C.lidx[C.large[l]] = (int32_t)l;
    }
  }
  // the mirror fold: dense precisions, every class symmetric (MPOLE_FOLD=0
  // turns it off, for comparisons)
  p->fold = !p->sep && theta_sym;
  for (const auto &C : p->cls) p->fold = p->fold && !C.mirb.empty();
  if (const char *env = std::getenv("MPOLE_FOLD")) p->fold = p->fold && std::atoi(env) != 0;
  for (int c = 0; c < p->ncls; ++c) {
    ClassHost &C = p->cls[c];
    C.pairs.clear();
    for (int b = 0; b < C.nblocks; ++b) {
      const int mb = p->fold ? C.mirb[b] : b;
      if (mb >= b) C.pairs.insert(C.pairs.end(), {b, mb});
    }
    C.npair = (int)(C.pairs.size() / 2);
    C.npair_pad = round_up(C.npair, p->kpad);
    // spans of kPackSpan blocks that are single cells at consecutive cell
    // indices (coarsening): span0[s] = cell of the span's first block, else -1
    const int nbspan = (C.nblocks + kPackSpan - 1) / kPackSpan;
    C.span0.assign(nbspan, -1);
    for (int sp = 0; sp < nbspan; ++sp) {
      const int bb = sp * kPackSpan, be = std::min(C.nblocks, bb + kPackSpan);
      const int first = C.mem[C.moff[bb]];
      bool affine = true;
      for (int b = bb; b < be && affine; ++b)
        affine = C.moff[b + 1] - C.moff[b] == 1 && C.mem[C.moff[b]] == first + (b - bb);
      if (affine) C.span0[sp] = first;
    }
    // packing spans of pairs whose rep blocks are single cells at consecutive
    // cell indices: pspan0[s] = cell of the span's first rep, else -1 (their
    // mirror blocks are then the single mirror cells)
    const int nspan = (C.npair + kPackSpan - 1) / kPackSpan;
    C.pspan0.assign(nspan, -1);
    for (int sp = 0; sp < nspan; ++sp) {
      const int qb = sp * kPackSpan, qe = std::min(C.npair, qb + kPackSpan);
      const int first = C.mem[C.moff[C.pairs[2 * qb]]];
      bool affine = true;
      for (int q = qb; q < qe && affine; ++q) {
        const int b = C.pairs[2 * q], mb = C.pairs[2 * q + 1];
        affine = C.moff[b + 1] - C.moff[b] == 1 && C.mem[C.moff[b]] == first + (q - qb) &&
                 C.moff[mb + 1] - C.moff[mb] == 1;
      }
      if (affine) C.pspan0[sp] = first;
    }
    build_pack_tasks(p, C);
    C.npack = C.ptasks.empty() ? nspan : (int)(C.ptasks.size() / 4);
  }
  // mode columns: folded, even parity (l + m) first, then odd
  p->pos_m.clear();
  p->perm_m.clear();
  p->perm_e.clear();
  if (p->fold) {
    std::vector<int32_t> ev, od;
    for (int l = 0; l <= p->L; ++l)
      for (int d = 0; d <= 2 * l; ++d) {
        const int mm = (d + 1) / 2;
        ((l + mm) % 2 == 0 ? ev : od).push_back(l * l + d);
      }
    p->odd_m0 = round_up((int)ev.size(), p->tile_n);
    p->namp_m = p->odd_m0 + round_up((int)od.size(), p->kpad);
    p->odd_e0 = round_up((int)ev.size(), p->kpad);
    p->namp_e = p->odd_e0 + round_up((int)od.size(), p->kpad);
    p->perm_m.assign(p->namp_m, -1);
    p->perm_e.assign(p->namp_e, -1);
    p->pos_m.assign(p->namp, -1);
    for (size_t t = 0; t < ev.size(); ++t) {
      p->perm_m[t] = p->perm_e[t] = ev[t];
      p->pos_m[ev[t]] = (int32_t)t;
    }
    for (size_t t = 0; t < od.size(); ++t) {
      p->perm_m[p->odd_m0 + t] = od[t];
      p->perm_e[p->odd_e0 + t] = od[t];
      p->pos_m[od[t]] = (int32_t)(p->odd_m0 + t);
    }
  } else {
    p->namp_m = p->odd_m0 = p->namp_e = p->odd_e0 = p->namp;
  }
  for (auto &C : p->cls) {
    C.n_tiles_mom = (p->namp_m + p->tile_n - 1) / p->tile_n;
    C.n_tiles_exp = (C.npair + p->tile_n - 1) / p->tile_n;
  }
  p->litems.clear();
  p->lbase.assign(p->nr + 1, 0);
  for (int i = 0; i < p->nr; ++i) {
    p->lbase[i] = (int32_t)(p->litems.size() / 2);
    for (int b : p->cls[p->shell_class[i]].large) {
      p->litems.push_back(i);
      p->litems.push_back(b);
    }
  }
  p->lbase[p->nr] = (int32_t)(p->litems.size() / 2);
  // chunks of at most kLargeChunk members: (item, chunk, chunks of the item, first chunk of the item)
  p->lchunks.clear();
  for (size_t it = 0; it < p->litems.size() / 2; ++it) {
    const ClassHost &C = p->cls[p->shell_class[p->litems[2 * it]]];
    const int b = p->litems[2 * it + 1];
    const int n = (C.moff[b + 1] - C.moff[b] + kLargeChunk - 1) / kLargeChunk;
    const int first = (int)(p->lchunks.size() / 4);
    for (int c = 0; c < n; ++c) {
      p->lchunks.push_back((int32_t)it);
      p->lchunks.push_back(c);
      p->lchunks.push_back(n);
      p->lchunks.push_back(first);
    }
  }
  if (p->sep) {
    // rows holding a merged block read the block-mean density; their blocks
    // are averaged on the way in, blocks of several cells on the way out
    p->rowalt.assign((size_t)p->nr * p->nt, 0);
    std::vector<std::vector<uint8_t>> merged(p->ncls, std::vector<uint8_t>(p->nt, 0));
    for (int c = 0; c < p->ncls; ++c) {
      ClassHost &C = p->cls[c];
      for (int b = 0; b < C.nblocks; ++b)
        if (C.moff[b + 1] - C.moff[b] > 1)
          for (int e = C.moff[b]; e < C.moff[b + 1]; ++e) merged[c][C.mem[e] / p->np] = 1;
      C.sep_src.clear();
      C.sep_avg.clear();
      for (int b = 0; b < C.nblocks && C.bands.empty(); ++b) {   // banded classes: launch_bands
        const int n = C.moff[b + 1] - C.moff[b];
        if (n > kLargeBlock) continue;   // launch_large
        if (n > 1) C.sep_avg.push_back(b);
        if (merged[c][C.mem[C.moff[b]] / p->np]) C.sep_src.push_back(b);
      }
      p->max_src = std::max(p->max_src, (int)C.sep_src.size());
      p->max_avg = std::max(p->max_avg, (int)C.sep_avg.size());
    }
    // BF16 x3: rows of one-row blocks of 2, 4 or 8 cells (bands with nj = 1)
    // are averaged inside the phi transforms, code 1 + log2 nk
    for (int c = 0; c < p->ncls && p->sep_bf16; ++c) {
      const ClassHost &C = p->cls[c];
      for (size_t q = 0; q + 3 < C.bands.size(); q += 4) {
        const int j0 = C.bands[q], nj = C.bands[q + 1], nk = C.bands[q + 2], kind = C.bands[q + 3];
        if (kind == 1 && nj == 1 && nk >= 2 && nk <= kSepFuseNk)
          merged[c][j0] = (uint8_t)(nk == 2 ? 2 : nk == 4 ? 3 : 4);
      }
    }
    for (int i = 0; i < p->nr; ++i)
      for (int j = 0; j < p->nt; ++j) {
        p->rowalt[(size_t)i * p->nt + j] = merged[p->shell_class[i]][j];
        p->any_alt = p->any_alt || merged[p->shell_class[i]][j];
      }
  }
  p->rule = make_gauss_rule();
  // about one full round of resident workgroups: 4 per CU (f64 kernel), 3 per CU (split kernel)
  layout_plan(p, default_target(p));
  return MPOLE_OK;
}

// Tuning validation: tile heights 0 (default), 64 or 128 for the split
// contractions, 0 or 64 for the FP64 ones; moment workgroups >= 0.
int check_tuning(const mpole_plan_t *p, const mpole_tuning *t) {
  if (t->moment_wgs < 0) return fail(MPOLE_ERR_INVALID, "moment_wgs %d < 0", t->moment_wgs);
  const int hs[2] = {t->moment_tile_m, t->expand_tile_m};
  for (int h : hs) {
    const bool okh = h == 0 || h == 64 || (h == 128 && p->nplanes > 0);
    if (!okh) return fail(MPOLE_ERR_UNSUPPORTED, "tile height %d (64%s)", h, p->nplanes ? " or 128" : " only for FP64");
  }
  return MPOLE_OK;
}

int default_target(const mpole_plan_t *p) {
  int target = p->nplanes ? 768 : 1024;
  if (const char *env = std::getenv("MPOLE_MOMENT_WGS")) target = std::max(1, std::atoi(env));
  return target;
}

void apply_tuning(mpole_plan_t *p, const mpole_tuning *t, int target) {
  const int def = p->nplanes ? 128 : 64;
  p->tm_mom = t->moment_tile_m ? t->moment_tile_m : def;
  p->tm_exp = t->expand_tile_m ? t->expand_tile_m : def;
  layout_plan(p, target);
}

// Split-K choice, workgroup counts and workspace layout for a moment
// workgroup target (host only; may be redone before bind).
void layout_plan(mpole_plan_t *p, int target) {
  p->moment_target = target;
  for (auto &C : p->cls) {
    C.m_tiles_mom = std::max(1, ((int)C.rows.size() + p->tm_mom - 1) / p->tm_mom);
    C.m_tiles_exp = std::max(1, ((int)C.rows.size() + p->tm_exp - 1) / p->tm_exp);
  }
  choose_splits(*p, target);
  int wm = 0, we = 0;
  for (auto &C : p->cls) {
    C.wg_mom_begin = wm;
    C.wg_exp_begin = we;
    if (!C.rows.empty()) {
      wm += C.m_tiles_mom * C.n_tiles_mom * C.splits;
      we += C.m_tiles_exp * C.n_tiles_exp;
    }
  }
  p->wg_mom = wm;
  p->wg_exp = we;

  // workspace layout: the bind-time region (tables, maps, device views)
  // first, then the per-solve region (everything a solve writes before it
  // reads it: packed operands, partials, moments, coefficients, edge sums);
  // per-solve offsets are relative to the start of their region
  size_t off = 0, soff = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  auto stake = [&](size_t bytes) {
    const size_t o = soff;
    soff = align256(soff + bytes);
    return o;
  };
  const int nplm = (p->L + 1) * (p->L + 2) / 2;
  p->off_r = take(sizeof(double) * (p->nr + 1));
  p->off_th = take(sizeof(double) * (p->nt + 1));
  p->off_ph = take(sizeof(double) * (p->np + 1));
  p->off_shell_class = take(sizeof(int32_t) * p->nr);
  p->off_shell_row = take(sizeof(int32_t) * p->nr);
  p->off_classes = take(sizeof(ClassDev) * p->ncls);
  p->off_pavg = take(sizeof(double) * (size_t)p->nt * nplm);
  p->off_trig = take(sizeof(double) * (size_t)p->np * 2 * (p->L + 1));
  p->off_weight = take(sizeof(double) * (size_t)p->ncell);
  p->off_wrow = take(sizeof(double) * (size_t)p->nt);
  p->off_dphi = take(sizeof(double) * (size_t)p->np);
  p->off_dom = take(sizeof(double) * (size_t)p->ncell);
  p->off_jr = take(sizeof(double) * (size_t)p->nr * (p->L + 1));
  p->off_ji = take(sizeof(double) * (size_t)p->nr * (p->L + 1));
  p->off_rr = take(sizeof(double) * (size_t)p->nr * (p->L + 1));
  p->off_ri = take(sizeof(double) * (size_t)p->nr * (p->L + 1));
  p->off_ang = stake(sizeof(double) * (size_t)p->nr * p->namp);
  p->off_coef = stake(sizeof(double) * (size_t)p->nr * p->namp);
  p->off_edge_r = stake(sizeof(double) * (size_t)(p->nr + 1) * p->namp);
  p->off_edge_i = stake(sizeof(double) * (size_t)(p->nr + 1) * p->namp);
  p->off_cplanes = stake(sizeof(uint16_t) * (size_t)p->nplanes * p->nr * p->namp_e);
  // FP64 folded expansion: coefficients in expansion columns
  p->off_coef_e = stake(p->fold && p->nplanes == 0 ? sizeof(double) * (size_t)p->nr * p->namp_e : 0);
  p->off_pos_m = take(sizeof(int32_t) * p->pos_m.size());
  p->off_perm_m = take(sizeof(int32_t) * p->perm_m.size());
  p->off_perm_e = take(sizeof(int32_t) * p->perm_e.size());
  p->off_cscale = stake(sizeof(double) * (size_t)p->nr);
  {
    int maxb = 0;
    for (auto &C : p->cls) maxb = std::max(maxb, C.npack);
    p->mono_stride = std::max(maxb, 1);
  }
  p->off_mono = stake(sizeof(double) * (size_t)p->nr * p->mono_stride);
  p->off_max = stake(sizeof(double) * (size_t)p->nr * p->mono_stride);
  p->off_shift = stake(sizeof(double) * (size_t)p->nr);
  p->off_tsum_part = take(sizeof(double) * (size_t)kTsumChunks * p->namp);
  p->off_litems = take(sizeof(int32_t) * p->litems.size());
  p->off_lbase = take(sizeof(int32_t) * p->lbase.size());
  p->off_lsum = stake(p->sep ? 0 : sizeof(double) * (p->litems.size() / 2));
  p->off_lchunks = take(sizeof(int32_t) * p->lchunks.size());
  p->off_lpart = stake(sizeof(double) * 2 * (p->lchunks.size() / 4));
  for (auto &C : p->cls) {
    const size_t nrows = C.rows.size();
    C.off_rows = take(sizeof(int32_t) * std::max<size_t>(nrows, 1));
    C.off_moff = take(sizeof(int32_t) * (C.nblocks + 1));
    C.off_mem = take(sizeof(int32_t) * p->ncell);
    C.off_rect = take(sizeof(int32_t) * C.rect.size());
    C.off_span0 = take(sizeof(int32_t) * C.span0.size());
    C.off_pspan0 = take(sizeof(int32_t) * C.pspan0.size());
    C.off_lidx = take(sizeof(int32_t) * C.lidx.size());
    C.off_bands = take(sizeof(int32_t) * C.bands.size());
    C.off_bcast = take(sizeof(int32_t) * C.bcast.size());
    const size_t dense = p->sep ? 0 : 1;   // the separable path has no block x mode tables
    C.off_table = take(dense * sizeof(double) * (size_t)C.nblocks_pad * p->namp);
    C.off_pairs = take(sizeof(int32_t) * C.pairs.size());
    C.off_ptasks = take(sizeof(int32_t) * C.ptasks.size());
    // FP64 folded operands over pairs (unfolded: the table itself)
    const size_t f64fold = (dense && p->fold && p->nplanes == 0) ? 1 : 0;
    C.off_tm = take(f64fold * sizeof(double) * (size_t)C.npair_pad * p->namp_m);
    C.off_te = take(f64fold * sizeof(double) * (size_t)C.npair_pad * p->namp_e);
    C.off_tcol0 = take(dense * sizeof(double) * (size_t)C.npair_pad);
    C.off_wsum = take(sizeof(double) * (size_t)C.nblocks_pad);
    C.off_tsum = take(dense * sizeof(double) * (size_t)p->namp);
    const size_t odd = p->fold ? 1 : 0;
    C.off_pack = stake(dense * sizeof(double) * nrows * C.npair_pad);
    C.off_pack_o = stake(dense * odd * sizeof(double) * nrows * C.npair_pad);
    // split-K partials: FP64 for the f64 kernel, FP32 (the accumulator type) for split precisions
    C.off_partial = stake(dense * (p->nplanes ? sizeof(float) : sizeof(double)) * (size_t)C.splits * nrows * p->namp_m);
    C.off_sep_src = take(sizeof(int32_t) * C.sep_src.size());
    C.off_sep_avg = take(sizeof(int32_t) * C.sep_avg.size());
    C.off_tplanes = take(sizeof(uint16_t) * (size_t)p->nplanes * C.npair_pad * p->namp_e);
    C.off_ttplanes = take(sizeof(uint16_t) * (size_t)p->nplanes * C.npair_pad * p->namp_m);
    C.off_ppacks = stake(sizeof(uint16_t) * (size_t)p->nplanes * nrows * C.npair_pad);
    C.off_ppacks_o = stake(odd * sizeof(uint16_t) * (size_t)p->nplanes * nrows * C.npair_pad);
    C.off_pscale = stake(sizeof(double) * std::max<size_t>(nrows, 1));
  }
  if (p->sep) {
    const size_t L1 = p->L + 1, nrt = (size_t)p->nr * p->nt;
    p->off_tw = take(sizeof(double) * 2 * (size_t)p->tpad * p->np);
    p->off_pw = take(sizeof(double) * L1 * p->nt * L1);
    p->off_pt = take(sizeof(double) * L1 * L1 * p->nt);
    p->off_shat = stake(p->any_alt ? sizeof(double) * (size_t)p->nr * p->ncell : 0);
    p->off_rowalt = take(nrt);
    p->off_f = stake(sizeof(double) * nrt * p->tpad);
    p->off_g = stake(sizeof(double) * nrt * p->tpad);
    p->off_scls = take(sizeof(SepClass) * p->ncls);
    // fragment-order split tables (64 lanes x 16 bytes per K step, tile and plane)
    p->ks_a = (p->np + 31) / 32;
    p->mt_a = (2 * p->L + 15) / 16;
    p->ks_s = (2 * p->L + 31) / 32;
    p->nt_s = (p->np + 15) / 16;
    const size_t frag = 3 * 64 * 16;
    p->off_twf = take(p->sep_bf16 ? frag * p->ks_a * p->mt_a : 0);
    p->off_ttf = take(p->sep_bf16 ? frag * p->ks_s * p->nt_s : 0);
  }
  // the single-plan view of the batched kernels: one device plan, phase prefix
  // sums; and the view of mpole_solve_static (per-solve region in the static
  // scratch array): its own device plan and class views
  p->off_plandev = take(sizeof(PlanDev));
  p->off_prefix = take(sizeof(int32_t) * PH_COUNT * 2);
  bcast_layout(p);
  p->off_bcast_items = take(sizeof(int32_t) * p->bcast_items.size());
  p->off_plandev_s = take(sizeof(PlanDev));
  p->off_classes_s = take(sizeof(ClassDev) * p->ncls);
  p->solve_off = off;
  p->solve_bytes = soff;
  p->ws_bytes = off + soff;
}

// Runs one phase launch, bracketed by timing events when timing is on.
template <class F>
hipError_t timed(mpole_plan_t *p, int phase, hipStream_t s, F &&launch) {
  if (!p->timing) return launch();
  if (p->ev_used * 2 + 2 > p->ev.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      p->ev.push_back(e);
    }
    p->ev_phase.push_back(0);
  }
  const size_t k = p->ev_used++;
  p->ev_phase[k] = phase;
  hipError_t r = hipEventRecord(p->ev[2 * k], s);
  if (r == hipSuccess) r = launch();
  if (r == hipSuccess) r = hipEventRecord(p->ev[2 * k + 1], s);
  return r;
}

hipError_t upload(char *ws, size_t off, const void *src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  return hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, s);
}

}  // namespace

extern "C" {

int mpole_abi_version(void) { return MPOLE_ABI_VERSION; }

const char *mpole_last_error(void) { return g_error; }

int mpole_plan_create(const mpole_mesh *mesh, mpole_plan *out) {
  if (!out) return fail(MPOLE_ERR_INVALID, "out is null");
  try {
    mpole_plan_t *p = new mpole_plan_t();
    const int rc = build_plan(mesh, p);
    if (rc != MPOLE_OK) {
      delete p;
      return rc;
    }
    *out = p;
    return ok();
  } catch (const std::bad_alloc &) {
    return fail(MPOLE_ERR_INVALID, "host allocation failed");
  } catch (...) {
    return fail(MPOLE_ERR_INVALID, "unexpected host exception");
  }
}

size_t mpole_plan_workspace_bytes(mpole_plan p) { return p ? p->ws_bytes : 0; }

int mpole_plan_nmodes(mpole_plan p) { return p ? p->nam : 0; }

int mpole_plan_folded(mpole_plan p) { return p && p->fold ? 1 : 0; }

}  // extern "C"

namespace {

// Broadcast workgroups of a dense plan: kBcastBands merged-block bands of a
// shell each, as (shell, first band) pairs.
void bcast_layout(mpole_plan_t *p) {
  p->bcast_items.clear();
  if (p->sep) return;
  for (int i = 0; i < p->nr; ++i) {
    const int n = (int)p->cls[p->shell_class[i]].bcast.size();
    for (int t = 0; t < n; t += kBcastBands) p->bcast_items.insert(p->bcast_items.end(), {i, t});
  }
}

// FP16 x2 row-split workgroups per shell: chunks of kSplitRowChunk pairs of
// the longest padded row of any class.
int split_chunks(const mpole_plan_t *p) {
  int n = 0;
  for (const auto &C : p->cls) n = std::max(n, C.npair_pad);
  return (n + kSplitRowChunk - 1) / kSplitRowChunk;
}

int phase_wgs_host(const mpole_plan_t *p, int h) {
  switch (h) {
    case PH_PACK: return p->mono_stride * p->nr;
    case PH_SPLITROWS: return p->precision == MPOLE_FP16X2 ? p->nr * split_chunks(p) : 0;
    case PH_MOMENT: return p->wg_mom;
    case PH_REDUCE: return (p->namp + 255) / 256 * p->nr;
    case PH_SCAN: return p->namp / p->scan_modes;
    case PH_COEF: return (p->nplanes || (p->fold && !p->sep)) ? p->nr : 0;
    case PH_EXPAND: return p->wg_exp;
    case PH_BCAST: return (int)(p->bcast_items.size() / 2);
  }
  return 0;
}

// Device views of plan p: the bind-time region of the workspace at ws, the
// per-solve region at sv (the workspace's own, or the static scratch array),
// the class views at device address classes_dev.
void make_views(const mpole_plan_t *p, char *ws, char *sv, ClassDev *classes_dev, PlanDev &D,
                std::vector<ClassDev> &cd, SepDev &S) {
  D = PlanDev{};
  D.pack_parts = p->mono_stride;
  D.split_chunks = p->precision == MPOLE_FP16X2 ? split_chunks(p) : 0;
  D.bcast_items = (const int2 *)(ws + p->off_bcast_items);
  D.wg_mom = p->wg_mom;
  D.tm_mom = p->tm_mom;
  D.tm_exp = p->tm_exp;
  D.wg_exp = p->wg_exp;
  D.nr = p->nr;
  D.ntheta = p->nt;
  D.nphi = p->np;
  D.lmax = p->L;
  D.nam = p->nam;
  D.namp = p->namp;
  D.ncell = p->ncell;
  D.nclasses = p->ncls;
  D.nplanes = p->nplanes;
  D.G = p->G;
  D.r_edges = (const double *)(ws + p->off_r);
  D.theta_edges = (const double *)(ws + p->off_th);
  D.phi_edges = (const double *)(ws + p->off_ph);
  D.shell_class = (const int32_t *)(ws + p->off_shell_class);
  D.shell_row = (const int32_t *)(ws + p->off_shell_row);
  D.classes = classes_dev;
  D.pavg = (double *)(ws + p->off_pavg);
  D.trig = (double *)(ws + p->off_trig);
  D.weight = (double *)(ws + p->off_weight);
  D.wrow = (double *)(ws + p->off_wrow);
  D.dphi = (double *)(ws + p->off_dphi);
  D.dom = (double *)(ws + p->off_dom);
  D.jr = (double *)(ws + p->off_jr);
  D.ji = (double *)(ws + p->off_ji);
  D.rr = (double *)(ws + p->off_rr);
  D.ri = (double *)(ws + p->off_ri);
  D.ang = (double *)(sv + p->off_ang);
  D.coef = (double *)(sv + p->off_coef);
  D.fold = p->fold ? 1 : 0;
  D.namp_m = p->namp_m;
  D.odd_m0 = p->odd_m0;
  D.namp_e = p->namp_e;
  D.odd_e0 = p->odd_e0;
  D.pos_m = p->fold ? (const int32_t *)(ws + p->off_pos_m) : nullptr;
  D.perm_m = p->fold ? (const int32_t *)(ws + p->off_perm_m) : nullptr;
  D.perm_e = p->fold ? (const int32_t *)(ws + p->off_perm_e) : nullptr;
  D.coef_e = (p->fold && p->nplanes == 0) ? (double *)(sv + p->off_coef_e) : D.coef;
  D.edge_r = (double *)(sv + p->off_edge_r);
  D.edge_i = (double *)(sv + p->off_edge_i);
  D.cplanes = (uint16_t *)(sv + p->off_cplanes);
  D.cscale = (double *)(sv + p->off_cscale);
  D.mono_part = p->nplanes ? (double *)(sv + p->off_mono) : nullptr;
  D.max_part = (double *)(sv + p->off_max);
  D.mono_stride = p->mono_stride;
  D.shift = (double *)(sv + p->off_shift);
  D.tsum_part = (double *)(ws + p->off_tsum_part);
  D.litems = (const int2 *)(ws + p->off_litems);
  D.lbase = (const int32_t *)(ws + p->off_lbase);
  D.lsum = p->sep ? nullptr : (double *)(sv + p->off_lsum);
  D.n_litems = (int32_t)(p->litems.size() / 2);
  D.lchunks = (const int4 *)(ws + p->off_lchunks);
  D.lpart = (double *)(sv + p->off_lpart);
  D.n_lchunks = (int32_t)(p->lchunks.size() / 4);
  cd.assign(p->ncls, ClassDev{});
  for (int c = 0; c < p->ncls; ++c) {
    const ClassHost &H = p->cls[c];
    ClassDev &C = cd[c];
    C.rows = (const int32_t *)(ws + H.off_rows);
    C.moff = (const int32_t *)(ws + H.off_moff);
    C.mem = (const int32_t *)(ws + H.off_mem);
    C.rect = H.rect.empty() ? nullptr : (const int4 *)(ws + H.off_rect);
    C.span0 = (const int32_t *)(ws + H.off_span0);
    C.pspan0 = (const int32_t *)(ws + H.off_pspan0);
    C.lidx = H.lidx.empty() ? nullptr : (const int32_t *)(ws + H.off_lidx);
    C.bands = H.bands.empty() ? nullptr : (const int4 *)(ws + H.off_bands);
    C.nbands = (int32_t)(H.bands.size() / 4);
    C.bcast = H.bcast.empty() ? nullptr : (const int32_t *)(ws + H.off_bcast);
    C.nbcast = (int32_t)H.bcast.size();
    D.max_bands = std::max(D.max_bands, C.nbands);
    C.table = (double *)(ws + H.off_table);
    C.pairs = (const int2 *)(ws + H.off_pairs);
    C.ptasks = H.ptasks.empty() ? nullptr : (const int4 *)(ws + H.off_ptasks);
    C.npack = H.npack;
    C.npair = H.npair;
    C.npair_pad = H.npair_pad;
    const bool f64fold = p->fold && p->nplanes == 0;
    C.tm = f64fold ? (double *)(ws + H.off_tm) : C.table;
    C.te = f64fold ? (double *)(ws + H.off_te) : C.table;
    C.tcol0 = (double *)(ws + H.off_tcol0);
    C.wsum = (double *)(ws + H.off_wsum);
    C.tsum = (double *)(ws + H.off_tsum);
    C.pack = (double *)(sv + H.off_pack);
    C.pack_o = p->fold ? (double *)(sv + H.off_pack_o) : nullptr;
    C.partial = (double *)(sv + H.off_partial);
    C.tplanes = (uint16_t *)(ws + H.off_tplanes);
    C.ttplanes = (uint16_t *)(ws + H.off_ttplanes);
    C.ppacks = (uint16_t *)(sv + H.off_ppacks);
    C.ppacks_o = p->fold ? (uint16_t *)(sv + H.off_ppacks_o) : nullptr;
    C.pscale = (double *)(sv + H.off_pscale);
    C.nrows = (int)H.rows.size();
    C.nblocks = H.nblocks;
    C.nblocks_pad = H.nblocks_pad;
    C.splits = H.splits;
    C.kchunk = H.kchunk;
    C.m_tiles_mom = H.m_tiles_mom;
    C.m_tiles_exp = H.m_tiles_exp;
    C.n_tiles_mom = H.n_tiles_mom;
    C.n_tiles_exp = H.n_tiles_exp;
    C.wg_mom_begin = H.wg_mom_begin;
    C.wg_exp_begin = H.wg_exp_begin;
  }
  S = SepDev{};
  if (p->sep) {
    S.tpad = p->tpad;
    S.tw = (double *)(ws + p->off_tw);
    S.pw = (double *)(ws + p->off_pw);
    S.pt = (double *)(ws + p->off_pt);
    S.shat = p->any_alt ? (double *)(sv + p->off_shat) : nullptr;
    S.rowalt = p->any_alt ? (const uint8_t *)(ws + p->off_rowalt) : nullptr;
    S.f = (double *)(sv + p->off_f);
    S.g = (double *)(sv + p->off_g);
    S.dom = D.dom;
    S.cls = (const SepClass *)(ws + p->off_scls);
    S.max_src = p->max_src;
    S.max_avg = p->max_avg;
    S.twf = p->sep_bf16 ? (const uint32_t *)(ws + p->off_twf) : nullptr;
    S.ttf = p->sep_bf16 ? (const uint32_t *)(ws + p->off_ttf) : nullptr;
    S.ks_a = p->ks_a;
    S.mt_a = p->mt_a;
    S.ks_s = p->ks_s;
    S.nt_s = p->nt_s;
    S.fuse_nk = p->sep_bf16 ? kSepFuseNk : 0;
  }
}

// Bind-time set-up of the allocation-free entry point: the device address
// of the current device's copy of the static scratch array, or null if it
// cannot be resolved.  The address is looked up once per device, with that
// device current, and kept; host code uses it, never the array's name (in
// host code the name is only a stand-in for the symbol).
char *scratch_address() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static char *addr[kMaxDevices] = {};
  static bool tried[kMaxDevices] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!tried[dev]) {
    tried[dev] = true;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess)
      addr[dev] = (char *)ptr;
    else
      (void)hipGetLastError();   // leave no sticky error for the launches that follow
  }
  return addr[dev];
}

// Device views of a plan in workspace ws, table construction and the
// single-plan batch view (device plan copy + prefix sums), all enqueued on s.
int bind_plan(mpole_plan_t *p, void *dev_ws, size_t bytes, void *stream) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  if (!dev_ws) return fail(MPOLE_ERR_WORKSPACE, "workspace is null");
  if (((uintptr_t)dev_ws & 255) != 0) return fail(MPOLE_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (bytes < p->ws_bytes)
    return fail(MPOLE_ERR_WORKSPACE, "workspace has %zu bytes, plan needs %zu", bytes, p->ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)dev_ws;
  make_views(p, ws, ws + p->solve_off, (ClassDev *)(ws + p->off_classes), p->dev, p->cdev, p->sdev);
  const PlanDev &D = p->dev;
  // the static-scratch views, when the per-solve region fits the array
  p->static_ok = false;
  if (p->solve_bytes <= kScratchBytes) {
    char *sc = scratch_address();
    if (sc != nullptr) {
      make_views(p, ws, sc, (ClassDev *)(ws + p->off_classes_s), p->dev_s, p->cdev_s, p->sdev_s);
      p->static_ok = hipGetDevice(&p->static_dev) == hipSuccess;
    }
  }
  hipError_t e = hipSuccess;
  // the bind-time region starts zeroed (padding rows and columns of every
  // table are 0); the per-solve region is filled with NaN bit patterns, so a
  // read of anything a solve has not written first shows up in its results
  if (e == hipSuccess) e = launch_fill_zero(ws, p->solve_off, s);
  if (e == hipSuccess) e = launch_fill_word(ws + p->solve_off, p->solve_bytes, 0xFFFFFFFFu, s);
  if (e == hipSuccess) e = upload(ws, p->off_r, p->r.data(), sizeof(double) * p->r.size(), s);
  if (e == hipSuccess) e = upload(ws, p->off_th, p->th.data(), sizeof(double) * p->th.size(), s);
  if (e == hipSuccess) e = upload(ws, p->off_ph, p->ph.data(), sizeof(double) * p->ph.size(), s);
  if (e == hipSuccess) e = upload(ws, p->off_shell_class, p->shell_class.data(), sizeof(int32_t) * p->nr, s);
  if (e == hipSuccess) e = upload(ws, p->off_shell_row, p->shell_row.data(), sizeof(int32_t) * p->nr, s);
  if (e == hipSuccess) e = upload(ws, p->off_classes, p->cdev.data(), sizeof(ClassDev) * p->ncls, s);
  for (int c = 0; c < p->ncls && e == hipSuccess; ++c) {
    const ClassHost &H = p->cls[c];
    e = upload(ws, H.off_rows, H.rows.data(), sizeof(int32_t) * H.rows.size(), s);
    if (e == hipSuccess) e = upload(ws, H.off_moff, H.moff.data(), sizeof(int32_t) * H.moff.size(), s);
    if (e == hipSuccess) e = upload(ws, H.off_mem, H.mem.data(), sizeof(int32_t) * H.mem.size(), s);
    if (e == hipSuccess) e = upload(ws, H.off_rect, H.rect.data(), sizeof(int32_t) * H.rect.size(), s);
    if (e == hipSuccess) e = upload(ws, H.off_span0, H.span0.data(), sizeof(int32_t) * H.span0.size(), s);
    if (e == hipSuccess) e = upload(ws, H.off_pspan0, H.pspan0.data(), sizeof(int32_t) * H.pspan0.size(), s);
    if (e == hipSuccess) e = upload(ws, H.off_lidx, H.lidx.data(), sizeof(int32_t) * H.lidx.size(), s);
    if (e == hipSuccess) e = upload(ws, H.off_bands, H.bands.data(), sizeof(int32_t) * H.bands.size(), s);
    if (e == hipSuccess) e = upload(ws, H.off_bcast, H.bcast.data(), sizeof(int32_t) * H.bcast.size(), s);
    if (e == hipSuccess) e = upload(ws, H.off_pairs, H.pairs.data(), sizeof(int32_t) * H.pairs.size(), s);
    if (e == hipSuccess) e = upload(ws, H.off_ptasks, H.ptasks.data(), sizeof(int32_t) * H.ptasks.size(), s);
  }
  if (e == hipSuccess) e = upload(ws, p->off_pos_m, p->pos_m.data(), sizeof(int32_t) * p->pos_m.size(), s);
  if (e == hipSuccess) e = upload(ws, p->off_perm_m, p->perm_m.data(), sizeof(int32_t) * p->perm_m.size(), s);
  if (e == hipSuccess) e = upload(ws, p->off_perm_e, p->perm_e.data(), sizeof(int32_t) * p->perm_e.size(), s);
  if (e == hipSuccess) e = upload(ws, p->off_litems, p->litems.data(), sizeof(int32_t) * p->litems.size(), s);
  if (e == hipSuccess) e = upload(ws, p->off_lbase, p->lbase.data(), sizeof(int32_t) * p->lbase.size(), s);
  if (e == hipSuccess) e = upload(ws, p->off_lchunks, p->lchunks.data(), sizeof(int32_t) * p->lchunks.size(), s);
  // single-plan batch view: the device plan and its phase prefix sums
  p->prefix.assign(PH_COUNT * 2, 0);
  for (int h = 0; h < PH_COUNT; ++h) p->prefix[2 * h + 1] = phase_wgs_host(p, h);
  if (e == hipSuccess) e = upload(ws, p->off_plandev, &p->dev, sizeof(PlanDev), s);
  if (e == hipSuccess) e = upload(ws, p->off_prefix, p->prefix.data(), sizeof(int32_t) * p->prefix.size(), s);
  if (e == hipSuccess) e = upload(ws, p->off_bcast_items, p->bcast_items.data(), sizeof(int32_t) * p->bcast_items.size(), s);
  if (e == hipSuccess && p->static_ok) {
    e = upload(ws, p->off_plandev_s, &p->dev_s, sizeof(PlanDev), s);
    if (e == hipSuccess) e = upload(ws, p->off_classes_s, p->cdev_s.data(), sizeof(ClassDev) * p->ncls, s);
  }
  if (p->sep) {
    p->scls.assign(p->ncls, SepClass{});
    for (int c = 0; c < p->ncls; ++c) {
      const ClassHost &H = p->cls[c];
      p->scls[c] = SepClass{(const int32_t *)(ws + H.off_sep_src), (int32_t)H.sep_src.size(),
                            (const int32_t *)(ws + H.off_sep_avg), (int32_t)H.sep_avg.size()};
      if (e == hipSuccess) e = upload(ws, H.off_sep_src, H.sep_src.data(), sizeof(int32_t) * H.sep_src.size(), s);
      if (e == hipSuccess) e = upload(ws, H.off_sep_avg, H.sep_avg.data(), sizeof(int32_t) * H.sep_avg.size(), s);
    }
    if (e == hipSuccess) e = upload(ws, p->off_rowalt, p->rowalt.data(), p->rowalt.size(), s);
    if (e == hipSuccess) e = upload(ws, p->off_scls, p->scls.data(), sizeof(SepClass) * p->scls.size(), s);
  }
  if (e == hipSuccess) e = launch_tables(D, p->cdev.data(), p->rule, !p->sep, s);
  if (e == hipSuccess && !p->sep) e = launch_pair_tables(D, p->cdev.data(), s);
  if (e == hipSuccess && p->sep) e = launch_sep_tables(D, p->sdev, s);
  if (e == hipSuccess && p->sep_bf16) e = launch_sep_split_tables(D, p->sdev, s);
  if (e == hipSuccess && p->nplanes) e = launch_split_tables(D, p->cdev.data(), p->precision, s);
  // the uploads above read host memory of this plan that later calls may
  // change (rebinding, tuning): wait for them before returning
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    p->bound = false;
    p->static_ok = false;
    return fail(MPOLE_ERR_DEVICE, "bind: %s", hipGetErrorString(e));
  }
  p->ws = ws;
  p->bound = true;
  return ok();
}

// A field with blocks of more than kLargeBlock cells: its device plan (host
// copy) and I/O, for the per-field launch_large calls around the batched
// packing and expansion kernels.
struct LargeJob {
  const PlanDev *P;
  const double *rho;
  double *phi;
};

// The kernel sequence of one solve for a batch view B of fields sharing
// `precision`; wgs[h] = total workgroups of phase h; phi == false skips the
// potential (moments only).
template <class Timer>
hipError_t run_solve(const BatchDev &B, int precision, const int *wgs, int scan_modes, bool phi,
                     const LargeJob *large, int nlarge, hipStream_t s, Timer &&timed) {
  const int k = precision;
  hipError_t e = launch_stamp_reset(B, s);
  if (e == hipSuccess) e = timed(MPOLE_PHASE_PACK, [&] {
    hipError_t r = hipSuccess;
    for (int q = 0; q < nlarge && r == hipSuccess; ++q) r = launch_large(*large[q].P, kLargeSum, large[q].rho, nullptr, s);
    if (r == hipSuccess) r = launch_pack(B, k, wgs[PH_PACK], s);
    if (r == hipSuccess) r = launch_split_rows(B, wgs[PH_SPLITROWS], s);
    return r;
  });
  if (e == hipSuccess) e = timed(MPOLE_PHASE_MOMENT, [&] { return launch_moment(B, k, wgs[PH_MOMENT], s); });
  if (e == hipSuccess) e = timed(MPOLE_PHASE_REDUCE, [&] { return launch_reduce(B, wgs[PH_REDUCE], s); });
  if (e == hipSuccess) e = timed(MPOLE_PHASE_SCAN, [&] { return launch_scan(B, wgs[PH_SCAN], scan_modes, s); });
  if (e == hipSuccess && phi && wgs[PH_COEF] > 0)
    e = timed(MPOLE_PHASE_SPLIT, [&] { return launch_split_coef(B, k, wgs[PH_COEF], s); });
  if (e == hipSuccess && phi) e = timed(MPOLE_PHASE_EXPAND, [&] {
    hipError_t r = launch_expand(B, k, wgs[PH_EXPAND], s);
    for (int q = 0; q < nlarge && r == hipSuccess; ++q) r = launch_large(*large[q].P, kLargeBcast, nullptr, large[q].phi, s);
    return r;
  });
  if (e == hipSuccess && phi && wgs[PH_BCAST] > 0)
    e = timed(MPOLE_PHASE_BCAST, [&] { return launch_bcast(B, wgs[PH_BCAST], s); });
  return e;
}

}  // namespace

extern "C" {

int mpole_plan_configure(mpole_plan p, int32_t moment_wgs) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  const mpole_tuning t = {moment_wgs, 0, 0};
  return mpole_plan_tune(p, &t);
}

int mpole_plan_tune(mpole_plan p, const mpole_tuning *t) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  if (!t) return fail(MPOLE_ERR_INVALID, "tuning is null");
  if (p->bound) return fail(MPOLE_ERR_INVALID, "tune before binding a workspace");
  int rc = check_tuning(p, t);
  if (rc) return rc;
  apply_tuning(p, t, t->moment_wgs > 0 ? t->moment_wgs : default_target(p));
  return ok();
}

int mpole_plan_get_tuning(mpole_plan p, mpole_tuning *t) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  if (!t) return fail(MPOLE_ERR_INVALID, "tuning is null");
  t->moment_wgs = p->moment_target;
  t->moment_tile_m = p->tm_mom;
  t->expand_tile_m = p->tm_exp;
  return ok();
}

int mpole_plan_moment_wgs(mpole_plan p) { return p ? p->wg_mom : 0; }

int mpole_gradient(mpole_plan p, const double *phi, double *d_r, double *d_theta, double *d_phi, void *stream) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  if (!p->bound) return fail(MPOLE_ERR_INVALID, "plan is not bound to a workspace");
  if (!phi) return fail(MPOLE_ERR_INVALID, "phi is null");
  if (!d_r && !d_theta && !d_phi) return ok();
  if (p->dev.nphi > MPOLE_GRADIENT_MAX_NPHI)
    return fail(MPOLE_ERR_UNSUPPORTED, "phi rows above %d cells", MPOLE_GRADIENT_MAX_NPHI);
  const hipError_t e = launch_gradient(p->dev, phi, d_r, d_theta, d_phi, p->phi_periodic, (hipStream_t)stream);
  if (e != hipSuccess) return fail(MPOLE_ERR_DEVICE, "gradient launch failed: %s", hipGetErrorString(e));
  return ok();
}

int mpole_gravity_sources(mpole_plan p, const double *phi, const double *rho, const double *v_r,
                          const double *v_theta, const double *v_phi, double *s_r, double *s_theta, double *s_phi,
                          double *s_energy, void *stream) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  if (!p->bound) return fail(MPOLE_ERR_INVALID, "plan is not bound to a workspace");
  if (!phi || !rho) return fail(MPOLE_ERR_INVALID, "phi and rho are required");
  if (!s_r && !s_theta && !s_phi && !s_energy) return ok();
  if (p->dev.nphi > MPOLE_GRADIENT_MAX_NPHI)
    return fail(MPOLE_ERR_UNSUPPORTED, "phi rows above %d cells", MPOLE_GRADIENT_MAX_NPHI);
  const double *v[3] = {v_r, v_theta, v_phi};
  double *out[4] = {s_r, s_theta, s_phi, s_energy};
  const hipError_t e = launch_gravity_sources(p->dev, phi, rho, v, out, p->phi_periodic, (hipStream_t)stream);
  if (e != hipSuccess) return fail(MPOLE_ERR_DEVICE, "gravity sources launch failed: %s", hipGetErrorString(e));
  return ok();
}

int mpole_coarsen(mpole_plan p, const double *in, double *out, void *stream) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  if (!p->bound) return fail(MPOLE_ERR_INVALID, "plan is not bound to a workspace");
  if (!in || !out) return fail(MPOLE_ERR_INVALID, "in or out is null");
  const hipError_t e = launch_coarsen(p->dev, p->cdev.data(), in, out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(MPOLE_ERR_DEVICE, "coarsen launch failed: %s", hipGetErrorString(e));
  return ok();
}

int mpole_plan_bind(mpole_plan p, void *dev_ws, size_t bytes, void *stream) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  return bind_plan(p, dev_ws, bytes, stream);
}

}  // extern "C"

namespace {

// The separable solve of one plan on stream s (phi == null: moments only).
// (scratch: the static-scratch views of mpole_solve_static)
template <class Timer>
hipError_t run_sep(mpole_plan_t *p, const double *rho, double *phi, double *ang, double *interior, double *exterior,
                   hipStream_t s, Timer &&T, bool scratch = false) {
  BatchDev B{};
  B.plans = (const PlanDev *)(p->ws + (scratch ? p->off_plandev_s : p->off_plandev));
  B.io = nullptr;
  B.io1 = SolveIO{rho, phi, ang, interior, exterior};
  B.prefix = (const int32_t *)(p->ws + p->off_prefix);
  B.nf = 1;
  B.stamps = nullptr;
  const PlanDev &D = scratch ? p->dev_s : p->dev;
  const SepDev &S = scratch ? p->sdev_s : p->sdev;
  hipError_t e = hipSuccess;
  if (p->any_alt) e = T(MPOLE_PHASE_PACK, [&] { return launch_sep_source(D, S, rho, s); });
  if (e == hipSuccess) e = T(MPOLE_PHASE_MOMENT, [&] {
    return p->sep_bf16 ? launch_sep_phi_anal_bf16(D, S, rho, s) : launch_sep_phi_anal(D, S, rho, s);
  });
  if (e == hipSuccess) e = T(MPOLE_PHASE_REDUCE, [&] { return launch_sep_theta_anal(D, S, ang, s); });
  if (e == hipSuccess) e = T(MPOLE_PHASE_SCAN, [&] { return launch_scan(B, p->prefix[2 * PH_SCAN + 1], p->scan_modes, s); });
  if (e == hipSuccess && phi) e = T(MPOLE_PHASE_SPLIT, [&] { return launch_sep_theta_syn(D, S, s); });
  if (e == hipSuccess && phi) e = T(MPOLE_PHASE_EXPAND, [&] {
    return p->sep_bf16 ? launch_sep_phi_syn_bf16(D, S, phi, s) : launch_sep_phi_syn(D, S, phi, s);
  });
  return e;
}

// One solve of plan p on stream s through its workspace views (scratch =
// false) or its static-scratch views; arguments already checked.
int solve_views(mpole_plan_t *p, const double *rho, double *phi, double *ang, double *interior, double *exterior,
                hipStream_t s, bool scratch) {
  BatchDev B{};
  B.plans = (const PlanDev *)(p->ws + (scratch ? p->off_plandev_s : p->off_plandev));
  B.io = nullptr;
  B.io1 = SolveIO{rho, phi, ang, interior, exterior};
  B.prefix = (const int32_t *)(p->ws + p->off_prefix);
  B.nf = 1;
  B.stamps = nullptr;
  int wgs[PH_COUNT];
  for (int h = 0; h < PH_COUNT; ++h) wgs[h] = p->prefix[2 * h + 1];
  // the static-scratch solve records no timing events (creating them would
  // allocate host objects)
  auto timer = [&](int phase, auto &&launch) { return scratch ? launch() : timed(p, phase, s, launch); };
  hipError_t e;
  if (p->sep) {
    e = run_sep(p, rho, phi, ang, interior, exterior, s, timer, scratch);
  } else {
    const LargeJob large{scratch ? &p->dev_s : &p->dev, rho, phi};
    e = run_solve(B, p->precision, wgs, p->scan_modes, phi != nullptr, &large, p->dev.n_litems > 0 ? 1 : 0, s,
                  timer);
  }
  if (e != hipSuccess) return fail(MPOLE_ERR_DEVICE, "solve: %s", hipGetErrorString(e));
  return ok();
}

}  // namespace

extern "C" {

int mpole_solve(mpole_plan p, const double *rho, double *phi, double *ang, double *interior, double *exterior,
                void *stream) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  if (!p->bound) return fail(MPOLE_ERR_WORKSPACE, "plan has no bound workspace");
  if (!rho) return fail(MPOLE_ERR_INVALID, "rho is null");
  return solve_views(p, rho, phi, ang, interior, exterior, (hipStream_t)stream, false);
}

int mpole_solve_static(mpole_plan p, const double *rho, double *phi, double *ang, double *interior,
                       double *exterior, void *stream) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  if (p->solve_bytes > kScratchBytes)
    return fail(MPOLE_ERR_UNSUPPORTED, "a solve of this plan needs %zu bytes of scratch; the static array holds %zu",
                p->solve_bytes, kScratchBytes);
  if (!p->bound) return fail(MPOLE_ERR_WORKSPACE, "plan has no bound workspace");
  if (!rho) return fail(MPOLE_ERR_INVALID, "rho is null");
  if (!p->static_ok) return fail(MPOLE_ERR_DEVICE, "the static scratch array was not resolved when the plan was bound");
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(MPOLE_ERR_DEVICE, "solve_static: %s", hipGetErrorString(e));
  if (dev != p->static_dev)
    return fail(MPOLE_ERR_INVALID, "current device %d is not the device %d the plan was bound on", dev, p->static_dev);
  return solve_views(p, rho, phi, ang, interior, exterior, (hipStream_t)stream, true);
}

int mpole_plan_copy_table(mpole_plan p, int32_t cls, double *host_out, int64_t *nblocks, void *stream) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  if (cls < 0 || cls >= p->ncls) return fail(MPOLE_ERR_INVALID, "class %d out of range", cls);
  const ClassHost &H = p->cls[cls];
  if (nblocks) *nblocks = H.nblocks;
  if (p->sep) return fail(MPOLE_ERR_UNSUPPORTED, "the separable path keeps no block x mode table");
  if (!host_out) return ok();
  if (!p->bound) return fail(MPOLE_ERR_WORKSPACE, "plan has no bound workspace");
  hipStream_t s = (hipStream_t)stream;
  // rows are namp wide on the device, nAM wide on the host
  hipError_t e = hipMemcpy2DAsync(host_out, sizeof(double) * p->nam, p->ws + H.off_table, sizeof(double) * p->namp,
                                  sizeof(double) * p->nam, H.nblocks, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(MPOLE_ERR_DEVICE, "copy_table: %s", hipGetErrorString(e));
  return ok();
}

int mpole_plan_set_timing(mpole_plan p, int enable) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  p->timing = enable != 0;
  p->ev_used = 0;
  return ok();
}

int mpole_plan_phase_ms(mpole_plan p, double *total_ms, int64_t *launches) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  if (!total_ms || !launches) return fail(MPOLE_ERR_INVALID, "output arrays are null");
  for (int k = 0; k < MPOLE_NPHASES; ++k) {
    total_ms[k] = 0.0;
    launches[k] = 0;
  }
  for (size_t k = 0; k < p->ev_used; ++k) {
    hipError_t e = hipEventSynchronize(p->ev[2 * k + 1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p->ev[2 * k], p->ev[2 * k + 1]);
    if (e != hipSuccess) return fail(MPOLE_ERR_DEVICE, "phase_ms: %s", hipGetErrorString(e));
    total_ms[p->ev_phase[k]] += ms;
    launches[p->ev_phase[k]] += 1;
  }
  p->ev_used = 0;
  return ok();
}

int mpole_plan_work(mpole_plan p, double *moment_flops, double *expand_flops, double *min_bytes) {
  if (!p) return fail(MPOLE_ERR_INVALID, "plan is null");
  double f = 0.0, tb = 0.0;
  if (p->sep) {
    // the phi transform of each direction, 2 flops per (shell, theta row, phi cell, trig mode)
    f = 2.0 * (double)p->nr * p->ncell * (2 * p->L + 1);
  } else {
    for (const auto &C : p->cls) {
      f += 2.0 * (double)C.rows.size() * C.nblocks * p->nam;
      if (!C.rows.empty()) tb += 8.0 * (double)C.nblocks * p->nam;
    }
  }
  if (moment_flops) *moment_flops = f;
  if (expand_flops) *expand_flops = f;
  if (min_bytes) *min_bytes = 16.0 * (double)p->nr * p->ncell + tb;
  return ok();
}

}  // extern "C"

namespace {
constexpr int kProbeWgs = 1024;                 // workgroups of the XCD probe
constexpr int kMaxXcc = 16;                     // XCD ids 0..15
constexpr int kPairFields = 2;                  // fields whose phases interleave in a queue
constexpr int kItemsPerPhase = 128;             // light phases: sub-items grouped to about this many items
constexpr int kMaxGroup = 64;                   // ... at most this many sub-items per item
constexpr uint32_t kWaitPolls = 1u << 22;       // default wait budget (seconds of polling)
constexpr double kMaxQueueImbalance = 1.25;     // longest queue over the mean, else launch per phase
}  // namespace

struct mpole_batch_t {
  std::vector<mpole_plan_t *> plans;
  std::vector<size_t> off;      // workspace offset of each field's plan
  size_t off_plans = 0, off_io = 0, off_prefix = 0, off_stamps = 0, ws_bytes = 0;
  // persistent launch: descriptor, segments, queue ranges, XCD -> queue,
  // sub-items and groups per phase, dispensers, completion counters, items,
  // error word, probe ids
  size_t off_pq = 0, off_segs = 0, off_qseg = 0, off_xccq = 0, off_sub = 0, off_grp = 0, off_next = 0, off_done = 0,
         off_tot = 0, off_err = 0, off_probe = 0;
  int precision = 0;
  std::vector<int32_t> prefix;  // [PH_COUNT][nf+1]
  std::vector<SolveIO> io;
  bool bound = false;
  char *ws = nullptr;
  double clock_khz = 0.0;
  int launch = MPOLE_LAUNCH_PERSISTENT;   // requested launch
  uint32_t wait_polls = kWaitPolls;
  bool pq_ok = false;                     // work queues built at bind
  bool pq_balanced = false;               // ... and within kMaxQueueImbalance
  bool last_persistent = false;           // the last solve ran the persistent launch
  int pq_grid = 0, pq_nq = 0;
  PersistDev pq{};                        // host copy of the descriptor (device pointers)
  std::string pq_note;                    // why the batch launches per phase, if it does
  ~mpole_batch_t() {
    for (auto *p : plans) delete p;
  }
};

namespace {

// Default per-field moment targets: one round of resident workgroups shared
// in proportion to each field's moment work.
void batch_layout(mpole_batch_t *b, const mpole_tuning *tunings) {
  const int nf = (int)b->plans.size();
  double total = 0.0;
  std::vector<double> work(nf);
  for (int f = 0; f < nf; ++f) {
    const mpole_plan_t *p = b->plans[f];
    double w = 0.0;
    for (const auto &C : p->cls) w += (double)C.rows.size() * C.npair_pad * p->namp_m;
    work[f] = w;
    total += w;
  }
  const int round = b->precision ? 768 : 1024;
  for (int f = 0; f < nf; ++f) {
    const mpole_tuning none = {0, 0, 0};
    const mpole_tuning &tf = tunings ? tunings[f] : none;
    const int t = tf.moment_wgs > 0 ? tf.moment_wgs : (int)std::lround(round * work[f] / std::max(total, 1.0));
    apply_tuning(b->plans[f], &tf, std::max(t, 1));
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  b->off.assign(nf, 0);
  for (int f = 0; f < nf; ++f) b->off[f] = take(b->plans[f]->ws_bytes);
  b->off_plans = take(sizeof(PlanDev) * nf);
  b->off_io = take(sizeof(SolveIO) * nf);
  b->off_prefix = take(sizeof(int32_t) * PH_COUNT * (nf + 1));
  b->off_stamps = take(sizeof(unsigned long long) * (nf + 1));
  b->off_pq = take(sizeof(PersistDev));
  b->off_segs = take(sizeof(int4) * PH_COUNT * nf);
  b->off_qseg = take(sizeof(int32_t) * (kMaxXcc + 1));
  b->off_xccq = take(sizeof(int32_t) * kMaxXcc);
  b->off_sub = take(sizeof(int32_t) * PH_COUNT * nf);
  b->off_grp = take(sizeof(int32_t) * PH_COUNT * nf);
  b->off_next = take(sizeof(uint32_t) * kMaxXcc);
  b->off_done = take(sizeof(uint32_t) * PH_COUNT * nf);
  b->off_tot = take(sizeof(int32_t) * PH_COUNT * nf);
  b->off_err = take(sizeof(uint32_t));
  b->off_probe = take(sizeof(int32_t) * kProbeWgs);
  b->ws_bytes = off;
  b->prefix.assign(PH_COUNT * (nf + 1), 0);
  for (int h = 0; h < PH_COUNT; ++h)
    for (int f = 0; f < nf; ++f)
      b->prefix[h * (nf + 1) + f + 1] = b->prefix[h * (nf + 1) + f] + phase_wgs_host(b->plans[f], h);
}

// Estimated time of one field's solve (seconds on the whole device, for the
// order in which lanes claim fields and for the balance test): streaming of
// the density, planes and potential, the two contractions at a sustained
// MFMA rate of the precision, and the radial part per (shell, mode).
double field_estimate(const mpole_plan_t *P) {
  double macs = 0.0;
  for (const auto &C : P->cls)
    macs += (double)round_up((int)C.rows.size(), 64) * C.npair_pad * (double)(P->namp_m + P->namp_e);
  const double mac_rate = P->precision == MPOLE_FP64 ? 1.6e13 : P->precision == MPOLE_FP16X2 ? 2e14 : 1e14;
  return 4e-12 * (double)P->nr * P->ncell + macs / mac_rate + 8.4e-11 * (double)P->nr * P->namp;
}

// Sub-items per item of phase h with `sub` sub-items: the light phases
// (packing, row split, split-K sum, coefficient step) are grouped to about
// kItemsPerPhase items, the contractions and the scan are one workgroup per
// item.
int phase_group(int h, int sub) {
  if (h == PH_MOMENT || h == PH_EXPAND || h == PH_SCAN || sub <= kItemsPerPhase) return 1;
  return std::min(kMaxGroup, (sub + kItemsPerPhase - 1) / kItemsPerPhase);
}

// Work queues of the persistent launch (on the bound workspace, enqueued on
// s and synchronised): eligibility, the XCD ids of the device, items per
// (field, phase), fields spread over one queue per XCD (longest estimate
// first onto the least loaded queue), shortest first within a queue, and
// the balance test.  Leaves pq_ok false, with the reason in pq_note, when the
// batch is to launch per phase.
hipError_t build_queues(mpole_batch_t *b, hipStream_t s) {
  b->pq_ok = false;
  b->pq_balanced = false;
  b->pq_note.clear();
  const int nf = (int)b->plans.size();
  const int smodes = persistent_scan_modes();
  if (b->precision == MPOLE_FP64_SEPARABLE || b->precision == MPOLE_BF16X3_SEPARABLE) {
    b->pq_note = "separable precisions launch per phase";
    return hipSuccess;
  }
  for (int f = 0; f < nf; ++f) {
    if (b->plans[f]->dev.n_litems > 0) {
      b->pq_note = "a field has blocks of more than " + std::to_string(kLargeBlock) + " cells";
      return hipSuccess;
    }
    if (b->plans[f]->namp % smodes != 0) {
      b->pq_note = "padded mode count not a multiple of the scan item";
      return hipSuccess;
    }
  }
  const int per_cu = persistent_blocks_per_cu(b->precision);
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (per_cu <= 0 || ncu <= 0) {
    b->pq_note = "no occupancy figure for the persistent kernel";
    return hipSuccess;
  }
  // XCD ids of a run of probe workgroups: they must repeat with the period of
  // the distinct ids (the round-robin dispatch of workgroups over XCDs),
  // which is what lets a queue be bound to the XCD that runs its workgroups
  std::vector<int32_t> ids(kProbeWgs, -1);
  int32_t *ids_d = (int32_t *)(b->ws + b->off_probe);
  e = launch_xcc_probe(ids_d, kProbeWgs, s);
  if (e == hipSuccess) e = hipMemcpyAsync(ids.data(), ids_d, sizeof(int32_t) * kProbeWgs, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  std::vector<int32_t> xq(kMaxXcc, -1);
  int period = 0;
  for (int w = 0; w < kProbeWgs; ++w) {
    if (ids[w] < 0 || ids[w] >= kMaxXcc) {
      b->pq_note = "XCD id out of range";
      return hipSuccess;
    }
    if (period == w && xq[ids[w]] < 0) {
      xq[ids[w]] = 0;
      ++period;
    }
  }
  for (int w = 0; w < kProbeWgs; ++w)
    if (ids[w] != ids[w % period]) {
      b->pq_note = "workgroups are not dispatched round-robin over XCDs";
      return hipSuccess;
    }
  int nq = 0;
  for (int x = 0; x < kMaxXcc; ++x)
    if (xq[x] == 0) xq[x] = nq++;
  // items per (field, phase) and each field's estimate
  std::vector<int32_t> tot(PH_COUNT * nf, 0), sub(PH_COUNT * nf, 0), grp(PH_COUNT * nf, 1);
  std::vector<double> est(nf, 0.0);
  double total = 0.0;
  for (int f = 0; f < nf; ++f) {
    const mpole_plan_t *P = b->plans[f];
    for (int h = 0; h < PH_COUNT; ++h) {
      const int n = h == PH_SCAN ? P->namp / smodes : phase_wgs_host(P, h);
      const int g = phase_group(h, n);
      sub[f * PH_COUNT + h] = n;
      grp[f * PH_COUNT + h] = g;
      tot[f * PH_COUNT + h] = (n + g - 1) / g;
    }
    est[f] = field_estimate(P);
    total += est[f];
  }
  std::vector<int> order(nf);
  for (int f = 0; f < nf; ++f) order[f] = f;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return est[a] > est[c]; });
  std::vector<double> load(nq, 0.0);
  std::vector<std::vector<int>> fq(nq);
  for (int f : order) {
    const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    fq[q].push_back(f);
    load[q] += est[f];
  }
  const double longest = *std::max_element(load.begin(), load.end());
  b->pq_balanced = longest <= kMaxQueueImbalance * total / nq;
  if (!b->pq_balanced) {
    char msg[128];
    std::snprintf(msg, sizeof msg, "fields do not spread over %d XCD queues (longest queue %.2f x the mean)", nq,
                  longest * nq / total);
    b->pq_note = msg;
  }
  // Within a queue, fields shortest first, taken in pairs whose phases are
  // interleaved (A pack, B pack, A moment, B moment, ...): while the last
  // round of one field's phase drains, the other field's items fill the
  // XCD, and a memory-bound phase of one runs beside a contraction of the
  // other.  Every item still follows the items it depends on.
  std::vector<int4> segs;
  std::vector<int32_t> qseg(kMaxXcc + 1, 0);
  for (int q = 0; q < nq; ++q) {
    std::reverse(fq[q].begin(), fq[q].end());   // shortest first
    qseg[q] = (int32_t)segs.size();
    int first = 0;
    for (size_t k = 0; k < fq[q].size(); k += kPairFields) {
      const size_t kend = std::min(fq[q].size(), k + kPairFields);
      for (int h = 0; h < PH_COUNT; ++h)
        for (size_t j = k; j < kend; ++j) {
          const int f = fq[q][j], n = tot[f * PH_COUNT + h];
          if (n == 0) continue;
          segs.push_back(int4{f, h, first, n});
          first += n;
        }
    }
  }
  qseg[nq] = (int32_t)segs.size();
  char *ws = b->ws;
  PersistDev Q{};
  Q.segs = (const int4 *)(ws + b->off_segs);
  Q.qseg = (const int32_t *)(ws + b->off_qseg);
  Q.xcc_q = (const int32_t *)(ws + b->off_xccq);
  Q.sub = (const int32_t *)(ws + b->off_sub);
  Q.grp = (const int32_t *)(ws + b->off_grp);
  Q.nq = nq;
  Q.next = (uint32_t *)(ws + b->off_next);
  Q.done = (uint32_t *)(ws + b->off_done);
  Q.tot = (const int32_t *)(ws + b->off_tot);
  Q.err = (uint32_t *)(ws + b->off_err);
  e = upload(ws, b->off_segs, segs.data(), sizeof(int4) * segs.size(), s);
  if (e == hipSuccess) e = upload(ws, b->off_qseg, qseg.data(), sizeof(int32_t) * qseg.size(), s);
  if (e == hipSuccess) e = upload(ws, b->off_xccq, xq.data(), sizeof(int32_t) * kMaxXcc, s);
  if (e == hipSuccess) e = upload(ws, b->off_sub, sub.data(), sizeof(int32_t) * sub.size(), s);
  if (e == hipSuccess) e = upload(ws, b->off_grp, grp.data(), sizeof(int32_t) * grp.size(), s);
  if (e == hipSuccess) e = upload(ws, b->off_tot, tot.data(), sizeof(int32_t) * tot.size(), s);
  if (e == hipSuccess) e = upload(ws, b->off_pq, &Q, sizeof(PersistDev), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host arrays above are temporaries
  if (e != hipSuccess) return e;
  b->pq = Q;
  b->pq_nq = nq;
  b->pq_grid = per_cu * ncu;
  b->pq_ok = true;
  return hipSuccess;
}

bool runs_persistent(const mpole_batch_t *b) {
  return b->pq_ok && (b->launch == MPOLE_LAUNCH_PERSISTENT_FORCED || (b->launch == MPOLE_LAUNCH_PERSISTENT && b->pq_balanced));
}

}  // namespace

extern "C" {

int mpole_batch_create(int32_t nfields, const mpole_mesh *meshes, mpole_batch *out) {
  if (!out) return fail(MPOLE_ERR_INVALID, "out is null");
  if (nfields < 1 || nfields > 4096) return fail(MPOLE_ERR_INVALID, "nfields %d outside [1, 4096]", nfields);
  if (!meshes) return fail(MPOLE_ERR_INVALID, "meshes is null");
  try {
    mpole_batch_t *b = new mpole_batch_t();
    for (int f = 0; f < nfields; ++f) {
      if (meshes[f].precision != meshes[0].precision) {
        delete b;
        return fail(MPOLE_ERR_INVALID, "field %d: all fields of a batch need the same precision", f);
      }
      mpole_plan_t *p = new mpole_plan_t();
      const int rc = build_plan(&meshes[f], p);
      if (rc != MPOLE_OK) {
        delete p;
        delete b;
        const std::string msg(g_error);
        return fail(rc, "field %d: %s", f, msg.c_str());
      }
      p->scan_modes = kScanModesNarrow;
      b->plans.push_back(p);
    }
    b->precision = meshes[0].precision;
    batch_layout(b, nullptr);
    *out = b;
    return ok();
  } catch (const std::bad_alloc &) {
    return fail(MPOLE_ERR_INVALID, "host allocation failed");
  } catch (...) {
    return fail(MPOLE_ERR_INVALID, "unexpected host exception");
  }
}

int mpole_batch_configure(mpole_batch b, const int32_t *moment_wgs) {
  if (!b) return fail(MPOLE_ERR_INVALID, "batch is null");
  if (!moment_wgs) return mpole_batch_tune(b, nullptr);
  std::vector<mpole_tuning> t(b->plans.size());
  for (size_t f = 0; f < t.size(); ++f) t[f] = {moment_wgs[f], 0, 0};
  return mpole_batch_tune(b, t.data());
}

int mpole_batch_tune(mpole_batch b, const mpole_tuning *tunings) {
  if (!b) return fail(MPOLE_ERR_INVALID, "batch is null");
  if (b->bound) return fail(MPOLE_ERR_INVALID, "tune before binding a workspace");
  if (tunings)
    for (size_t f = 0; f < b->plans.size(); ++f) {
      const int rc = check_tuning(b->plans[f], &tunings[f]);
      if (rc) {
        const std::string msg(g_error);
        return fail(rc, "field %zu: %s", f, msg.c_str());
      }
    }
  batch_layout(b, tunings);
  return ok();
}

int mpole_batch_get_tuning(mpole_batch b, mpole_tuning *tunings) {
  if (!b) return fail(MPOLE_ERR_INVALID, "batch is null");
  if (!tunings) return fail(MPOLE_ERR_INVALID, "tunings is null");
  for (size_t f = 0; f < b->plans.size(); ++f) {
    const int rc = mpole_plan_get_tuning(b->plans[f], &tunings[f]);
    if (rc) return rc;
  }
  return ok();
}

size_t mpole_batch_workspace_bytes(mpole_batch b) { return b ? b->ws_bytes : 0; }

int mpole_batch_bind(mpole_batch b, void *dev_ws, size_t bytes, const double *const *rho, double *const *phi,
                     void *stream) {
  if (!b) return fail(MPOLE_ERR_INVALID, "batch is null");
  if (!dev_ws) return fail(MPOLE_ERR_WORKSPACE, "workspace is null");
  if (((uintptr_t)dev_ws & 255) != 0) return fail(MPOLE_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (bytes < b->ws_bytes)
    return fail(MPOLE_ERR_WORKSPACE, "workspace has %zu bytes, batch needs %zu", bytes, b->ws_bytes);
  if (!rho || !phi) return fail(MPOLE_ERR_INVALID, "rho and phi pointer arrays are required");
  const int nf = (int)b->plans.size();
  for (int f = 0; f < nf; ++f)
    if (!rho[f] || !phi[f]) return fail(MPOLE_ERR_INVALID, "field %d: null rho or phi", f);
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)dev_ws;
  for (int f = 0; f < nf; ++f) {
    const int rc = bind_plan(b->plans[f], ws + b->off[f], b->plans[f]->ws_bytes, stream);
    if (rc != MPOLE_OK) {
      const std::string msg(g_error);
      return fail(rc, "field %d: %s", f, msg.c_str());
    }
  }
  std::vector<PlanDev> devs(nf);
  b->io.assign(nf, SolveIO{});
  for (int f = 0; f < nf; ++f) {
    devs[f] = b->plans[f]->dev;
    b->io[f].rho = rho[f];
    b->io[f].phi = phi[f];
  }
  hipError_t e = upload(ws, b->off_plans, devs.data(), sizeof(PlanDev) * nf, s);
  if (e == hipSuccess) e = upload(ws, b->off_io, b->io.data(), sizeof(SolveIO) * nf, s);
  if (e == hipSuccess) e = upload(ws, b->off_prefix, b->prefix.data(), sizeof(int32_t) * b->prefix.size(), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host arrays above are temporaries
  b->ws = ws;
  if (e == hipSuccess) e = build_queues(b, s);
  int dev = 0, khz = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) {
    b->pq_ok = false;
    return fail(MPOLE_ERR_DEVICE, "batch bind: %s", hipGetErrorString(e));
  }
  b->clock_khz = khz;
  b->bound = true;
  return ok();
}

int mpole_batch_solve(mpole_batch b, void *stream) {
  if (!b) return fail(MPOLE_ERR_INVALID, "batch is null");
  if (!b->bound) return fail(MPOLE_ERR_WORKSPACE, "batch has no bound workspace");
  const int nf = (int)b->plans.size();
  BatchDev B{};
  B.plans = (const PlanDev *)(b->ws + b->off_plans);
  B.io = (const SolveIO *)(b->ws + b->off_io);
  B.prefix = (const int32_t *)(b->ws + b->off_prefix);
  B.nf = nf;
  B.stamps = (unsigned long long *)(b->ws + b->off_stamps);
  int wgs[PH_COUNT];
  for (int h = 0; h < PH_COUNT; ++h) wgs[h] = b->prefix[h * (nf + 1) + nf];
  hipError_t e;
  if (b->precision == MPOLE_FP64_SEPARABLE || b->precision == MPOLE_BF16X3_SEPARABLE) {
    // separable fields: each field's launch sequence in turn (the fields are
    // independent; every launch fills the device on its own), with a
    // completion stamp after each field
    hipStream_t s = (hipStream_t)stream;
    e = launch_stamp_reset(B, s);
    if (e == hipSuccess) e = launch_stamp(B.stamps, nf, s);
    for (int f = 0; f < nf && e == hipSuccess; ++f) {
      e = run_sep(b->plans[f], b->io[f].rho, b->io[f].phi, nullptr, nullptr, nullptr, s,
                  [](int, auto &&launch) { return launch(); });
      if (e == hipSuccess) e = launch_stamp(B.stamps, f, s);
    }
  } else if (runs_persistent(b)) {
    e = launch_persistent(B, b->pq, (const PersistDev *)(b->ws + b->off_pq), b->wait_polls, b->precision, b->pq_grid,
                          (hipStream_t)stream);
  } else {
    std::vector<LargeJob> large;
    for (int f = 0; f < nf; ++f)
      if (b->plans[f]->dev.n_litems > 0) large.push_back(LargeJob{&b->plans[f]->dev, b->io[f].rho, b->io[f].phi});
    e = run_solve(B, b->precision, wgs, kScanModesNarrow, true, large.data(), (int)large.size(), (hipStream_t)stream,
                  [](int, auto &&launch) { return launch(); });
  }
  if (e != hipSuccess) return fail(MPOLE_ERR_DEVICE, "batch solve: %s", hipGetErrorString(e));
  b->last_persistent = runs_persistent(b);
  return ok();
}

int mpole_batch_set_launch(mpole_batch b, int32_t launch, uint32_t wait_polls) {
  if (!b) return fail(MPOLE_ERR_INVALID, "batch is null");
  if (launch != MPOLE_LAUNCH_PHASES && launch != MPOLE_LAUNCH_PERSISTENT && launch != MPOLE_LAUNCH_PERSISTENT_FORCED)
    return fail(MPOLE_ERR_INVALID, "unknown launch %d", launch);
  b->launch = launch;
  b->wait_polls = wait_polls ? wait_polls : kWaitPolls;
  return ok();
}

int mpole_batch_launch(mpole_batch b) {
  if (!b || !b->bound) return -1;
  return runs_persistent(b) ? MPOLE_LAUNCH_PERSISTENT : MPOLE_LAUNCH_PHASES;
}

const char *mpole_batch_launch_note(mpole_batch b) {
  if (!b || !b->bound) return "";
  return b->pq_note.c_str();
}

int mpole_batch_check(mpole_batch b, void *stream) {
  if (!b) return fail(MPOLE_ERR_INVALID, "batch is null");
  if (!b->bound) return fail(MPOLE_ERR_WORKSPACE, "batch has no bound workspace");
  if (!b->last_persistent) return ok();
  uint32_t err = 0;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(&err, b->pq.err, sizeof err, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(MPOLE_ERR_DEVICE, "batch check: %s", hipGetErrorString(e));
  if (err != 0)
    return fail(MPOLE_ERR_DEVICE,
                "batch solve: a dependency wait of the persistent launch gave up after %u polls; the potentials of "
                "that solve are undefined",
                b->wait_polls);
  return ok();
}

int mpole_batch_field_ms(mpole_batch b, double *ms) {
  if (!b) return fail(MPOLE_ERR_INVALID, "batch is null");
  if (!ms) return fail(MPOLE_ERR_INVALID, "ms is null");
  if (!b->bound) return fail(MPOLE_ERR_WORKSPACE, "batch has no bound workspace");
  const int nf = (int)b->plans.size();
  std::vector<unsigned long long> st(nf + 1);
  hipError_t e = hipMemcpy(st.data(), b->ws + b->off_stamps, sizeof(unsigned long long) * (nf + 1),
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(MPOLE_ERR_DEVICE, "field_ms: %s", hipGetErrorString(e));
  for (int f = 0; f < nf; ++f)
    ms[f] = (st[f] >= st[nf] && b->clock_khz > 0) ? (double)(st[f] - st[nf]) / b->clock_khz : -1.0;
  return ok();
}

int mpole_batch_destroy(mpole_batch b) {
  delete b;
  return ok();
}

int mpole_plan_destroy(mpole_plan p) {
  if (p)
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  delete p;
  return ok();
}

}  // extern "C"
