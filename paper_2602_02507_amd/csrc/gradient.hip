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
// Each wavefront owns a tile of GJ theta rows x 64 phi columns (a lane per
// column, the tile's rows in its registers) and walks a chunk of GR shells
// outward; a workgroup's four wavefronts take four theta-adjacent tiles.  A
// lane keeps its column's potential at the previous, current and next shell
// for the tile's rows and the rows just above and below it, so radial and
// theta neighbours come from registers; phi neighbours come from the
// adjacent lanes, and only the columns past the tile's edges (or across the
// periodic seam) are loaded.  Every load is issued one shell ahead of its
// use.  The reciprocal widths are computed once per row, column and shell.
// HBM-bound: about 8 B read (plus the halo rows and shells) and 24 B written
// per cell.  The gravitational sources of the balance equations (-rho grad
// Phi and -rho v . grad Phi, Sec. 3) come from the same pass, reading rho and
// the velocity beside the potential (40 B read and 32 B written per cell).
#include "device_util.h"

namespace mpole {
namespace {

constexpr int GTH = 256;   // threads: 4 wavefronts, one tile each
constexpr int GJ = 4;      // theta rows per tile (derivatives)
constexpr int GJS = 2;     // theta rows per tile (sources: more loads per cell)
constexpr int GR = 8;      // shells per workgroup

template <class T>
__device__ inline double centre(T e, int i) { return 0.5 * (e[i] + e[i + 1]); }

// Outputs of one launch: the three derivatives (SRC false), or the
// gravitational sources (SRC true): o[0..2] = -rho dPhi/dx^i and o[3] =
// -rho sum_i v^i dPhi/dx^i with v[i] the contravariant velocity (null: 0).
struct GradIO {
  double *o[4];
  const double *rho, *v[3];
};

template <bool SRC, int GJ>
__global__ __launch_bounds__(GTH) void k_gradient(PlanDev P, const double *phi_, GradIO io, int periodic) {
  double *const d_r = io.o[0], *const d_th = io.o[1], *const d_ph = io.o[2];
  const int ntk = (P.nphi + 63) / 64, ntj = (P.ntheta + GJ - 1) / GJ;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // theta-major tile order (adjacent rows in one workgroup and, through the
  // XCD-aware workgroup order, on one L2)
  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x) * 4 + w;
  const int tj = tile % ntj, tk = tile / ntj;
  const bool tin = tk < ntk;   // the last workgroup may hold tiles past the mesh
  const int k = tk * 64 + lane;
  const bool kin = tin && k < P.nphi;
  const int j0 = tj * GJ, nj = min(GJ, P.ntheta - j0);
  const long ncell = (long)P.ntheta * P.nphi;
  const auto re = gmem(P.r_edges), te = gmem(P.theta_edges), pe = gmem(P.phi_edges);

  // phi: neighbour columns and reciprocal width of this lane's column
  int klo = k, khi = k;
  double inv_ph = 0.0;
  if (kin && P.nphi > 1) {
    double xl, xh;
    if (periodic) {
      klo = k > 0 ? k - 1 : P.nphi - 1;
      khi = k < P.nphi - 1 ? k + 1 : 0;
      xl = centre(pe, klo) - (k == 0 ? 2.0 * kPi : 0.0);
      xh = centre(pe, khi) + (k == P.nphi - 1 ? 2.0 * kPi : 0.0);
    } else {
      klo = k > 0 ? k - 1 : k;
      khi = k < P.nphi - 1 ? k + 1 : k;
      xl = centre(pe, klo);
      xh = centre(pe, khi);
    }
    inv_ph = 1.0 / (xh - xl);
  }
  // where the phi neighbours come from: the cell itself (one-sided), the
  // adjacent lane, or a load (tile edge, periodic seam)
  const bool lo_self = klo == k, hi_self = khi == k;
  const bool lo_lane = !lo_self && klo == k - 1 && lane > 0, hi_lane = !hi_self && khi == k + 1 && lane < 63;
  const bool lo_load = kin && !lo_self && !lo_lane, hi_load = kin && !hi_self && !hi_lane;

  // theta: reciprocal widths of the tile's rows (one-sided at the poles)
  double inv_th[GJ];
#pragma unroll
  for (int u = 0; u < GJ; ++u) {
    const int j = j0 + u, jl = j > 0 ? j - 1 : j, jh = j < P.ntheta - 1 ? j + 1 : j;
    inv_th[u] = (u < nj && P.ntheta > 1) ? 1.0 / (centre(te, jh) - centre(te, jl)) : 0.0;
  }
  const bool has_top = j0 > 0, has_bot = j0 + nj < P.ntheta;

  // column values at one shell: v = rows -1 .. GJ (rows -1 and GJ: the halo
  // rows), lo / hi = the loaded phi neighbours of the tile's rows; the
  // previous shell keeps only the tile's rows
  double pv[GJ], cv[GJ + 2], nv[GJ + 2], clo[GJ], chi[GJ], nlo[GJ], nhi[GJ];
  // loads: a shell's base pointer (workgroup-uniform) plus 32-bit cell offsets
  int off[GJ + 2];
#pragma unroll
  for (int u = 0; u < GJ + 2; ++u) {
    const int j = j0 + u - 1;
    const bool row = u == 0 ? has_top : u == GJ + 1 ? has_bot : u - 1 < nj;
    off[u] = (kin && row) ? j * P.nphi + k : -1;
  }
  auto load = [&](double *v, double *lo, double *hi, int i) {
    const auto sp = gmem(phi_ + (size_t)i * ncell);
#pragma unroll
    for (int u = 0; u < GJ + 2; ++u) v[u] = off[u] >= 0 ? sp[(unsigned)off[u]] : 0.0;
#pragma unroll
    for (int u = 0; u < GJ; ++u) {
      lo[u] = (lo_load && u < nj) ? sp[(unsigned)(off[u + 1] - k + klo)] : 0.0;
      hi[u] = (hi_load && u < nj) ? sp[(unsigned)(off[u + 1] - k + khi)] : 0.0;
    }
  };

  const int i0 = blockIdx.y * GR, i1 = min(P.nr, i0 + GR);
  load(cv, clo, chi, i0);
  if (i0 > 0) {
    load(nv, nlo, nhi, i0 - 1);
#pragma unroll
    for (int u = 0; u < GJ; ++u) pv[u] = nv[u + 1];
  } else {
#pragma unroll
    for (int u = 0; u < GJ; ++u) pv[u] = cv[u + 1];
  }
  for (int i = i0; i < i1; ++i) {
    const bool up = i + 1 < P.nr;
    if (up) {
      load(nv, nlo, nhi, i + 1);
    } else {
#pragma unroll
      for (int u = 0; u < GJ + 2; ++u) nv[u] = cv[u];
    }
    double inv_r = 0.0;   // one-sided at the first and last shell, zero for one shell
    if (P.nr > 1) {
      const int lo = i > 0 ? i - 1 : i, hi = up ? i + 1 : i;
      inv_r = 1.0 / (centre(re, hi) - centre(re, lo));
    }
    const size_t base = (size_t)i * ncell;
    // sources: rho and the velocity of this shell, issued before the stores
    double srho[SRC ? GJ : 1], sv[SRC ? 3 : 1][SRC ? GJ : 1];
    if constexpr (SRC) {
#pragma unroll
      for (int u = 0; u < GJ; ++u) {
        const bool in = kin && u < nj;
        const size_t q = base + (unsigned)(in ? off[u + 1] : 0);
        srho[u] = in ? gmem(io.rho)[q] : 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) sv[c][u] = (in && io.v[c] != nullptr) ? gmem(io.v[c])[q] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < GJ; ++u) {
      const double c0 = cv[u + 1];
      // every lane takes part in the shuffles; only cells of the mesh store
      const double left = __shfl_up(c0, 1, 64), right = __shfl_down(c0, 1, 64);
      if (!kin || u >= nj) continue;
      const size_t q = base + (unsigned)off[u + 1];
      const double gr = (nv[u + 1] - pv[u]) * inv_r;
      const double gt = (((u + 1 < nj || has_bot) ? cv[u + 2] : c0) - ((u > 0 || has_top) ? cv[u] : c0)) * inv_th[u];
      const double gp = ((hi_self ? c0 : hi_lane ? right : chi[u]) - (lo_self ? c0 : lo_lane ? left : clo[u])) * inv_ph;
      if constexpr (!SRC) {
        if (d_r != nullptr) gmem(d_r)[q] = gr;
        if (d_th != nullptr) gmem(d_th)[q] = gt;
        if (d_ph != nullptr) gmem(d_ph)[q] = gp;
      } else {
        const double nrho = -srho[u];
        if (d_r != nullptr) gmem(d_r)[q] = nrho * gr;
        if (d_th != nullptr) gmem(d_th)[q] = nrho * gt;
        if (d_ph != nullptr) gmem(d_ph)[q] = nrho * gp;
        if (io.o[3] != nullptr)
          gmem(io.o[3])[q] = nrho * (sv[0][u] * gr + sv[1][u] * gt + sv[2][u] * gp);
      }
    }
#pragma unroll
    for (int u = 0; u < GJ; ++u) {
      pv[u] = cv[u + 1];
      clo[u] = nlo[u];
      chi[u] = nhi[u];
    }
#pragma unroll
    for (int u = 0; u < GJ + 2; ++u) cv[u] = nv[u];
  }
}

}  // namespace

hipError_t launch_gradient(const PlanDev &P, const double *phi, double *d_r, double *d_th, double *d_ph, int periodic,
                           hipStream_t s) {
  if (P.nr == 0 || P.ntheta == 0 || P.nphi == 0) return hipSuccess;
  const int tiles = ((P.ntheta + GJ - 1) / GJ) * ((P.nphi + 63) / 64);
  const unsigned groups = (unsigned)((tiles + 3) / 4), chunks = (unsigned)((P.nr + GR - 1) / GR);
  const GradIO io{{d_r, d_th, d_ph, nullptr}, nullptr, {nullptr, nullptr, nullptr}};
  hipLaunchKernelGGL((k_gradient<false, GJ>), dim3(groups, chunks), dim3(GTH), 0, s, P, phi, io, periodic);
  return hipGetLastError();
}

hipError_t launch_gravity_sources(const PlanDev &P, const double *phi, const double *rho, const double *const v[3],
                                  double *const out[4], int periodic, hipStream_t s) {
  if (P.nr == 0 || P.ntheta == 0 || P.nphi == 0) return hipSuccess;
  const int tiles = ((P.ntheta + GJS - 1) / GJS) * ((P.nphi + 63) / 64);
  const unsigned groups = (unsigned)((tiles + 3) / 4), chunks = (unsigned)((P.nr + GR - 1) / GR);
  const GradIO io{{out[0], out[1], out[2], out[3]}, rho, {v[0], v[1], v[2]}};
  hipLaunchKernelGGL((k_gradient<true, GJS>), dim3(groups, chunks), dim3(GTH), 0, s, P, phi, io, periodic);
  return hipGetLastError();
}

}  // namespace mpole
