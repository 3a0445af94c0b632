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
// lane holds three shells of its column (the rows of the tile and the rows
// just above and below it): the shell being differenced, the next one (the
// radial neighbour) and the one after, whose loads are issued while the
// current shell is differenced, so that one shell of loads is always in
// flight behind the stores.  The three shell buffers rotate through the
// fully unrolled shell loop (no register copies of loaded values).  Radial and
// theta neighbours come from registers, phi neighbours from the adjacent
// lanes (DPP lane shifts); only the two end lanes load a halo column (the
// column past the tile's edge, or across the periodic seam).  Every load is
// unconditional: rows, shells and columns past the mesh load a clamped copy
// (which is exactly the one-sided difference at the mesh's edges) or, for
// the columns past a closed phi circle, the column modulo nphi (so the lane
// after the last column holds column 0).  HBM-bound: about 8 B read (plus
// the halo rows and shells) and 24 B written per cell.  The gravitational
// sources of the balance equations (-rho grad Phi and -rho v . grad Phi,
// Sec. 3) come from the same pass, reading rho and the velocity beside the
// potential, two shells ahead as well (40 B read and 32 B written per cell).
#include "device_util.h"

namespace mpole {
namespace {

constexpr int GTH = 256;   // threads: 4 wavefronts, one tile each
constexpr int GJ = 4;      // theta rows per tile (derivatives)
constexpr int GJS = 2;     // theta rows per tile (sources: more loads per cell)
constexpr int GR = 8;      // shells per workgroup

template <class T>
__device__ inline double centre(T e, int i) { return 0.5 * (e[i] + e[i + 1]); }

// Whole-wavefront DPP shifts of a double: lane l receives lane l - 1
// (from_below) or lane l + 1 (from_above); the end lanes receive 0.
template <int CTRL>
__device__ inline double dpp_shift(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ inline double from_below(double x) { return dpp_shift<0x138>(x); }   // wave_shr:1
__device__ inline double from_above(double x) { return dpp_shift<0x130>(x); }   // wave_shl:1

// Raw buffer access to one phi row of an array: the descriptor holds the
// row's base address (wavefront-uniform, in scalar registers) and its size in
// bytes, a lane adds only its 32-bit byte offset, so that no lane keeps a
// 64-bit address in vector registers (and no address temporary of a store
// still in flight is overwritten, which would wait for that store).  The
// fourth descriptor word selects 32-bit raw data without swizzling.  Byte
// offsets within a row fit 31 bits: the entry points reject rows of 2^28
// cells or more.
typedef unsigned u2v __attribute__((ext_vector_type(2)));
__device__ inline __amdgpu_buffer_rsrc_t row_rsrc(const double *row, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)row, 0, bytes, 0x00020000);
}
__device__ inline double bload(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
// Stores carry the non-temporal hint: the derivatives and sources stream
// out once and nothing in this kernel reads them back (both kernels measured
// 5-20 % faster with it on the production and 942 x 256 x 512 meshes).
constexpr int kStoreNT = 2;   // cache-policy operand: nt
__device__ inline void bstore(__amdgpu_buffer_rsrc_t r, unsigned off, double x) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, x), r, (int)off, 0, kStoreNT);
}

// Outputs of one launch: the three derivatives (SRC false), or the
// gravitational sources (SRC true): o[0..2] = -rho dPhi/dx^i and o[3] =
// -rho sum_i v^i dPhi/dx^i with v[i] the contravariant velocity (null: 0).
struct GradIO {
  double *o[4];
  const double *rho, *v[3];
};

// One shell of a lane's column: rows -1 .. GJ of the tile (v), the tile's
// rows at the lane's halo column (h; meaningful on the end lanes only) and,
// for the sources, rho and the velocity at the tile's rows.
template <bool SRC, int GJ>
struct Shell {
  double v[GJ + 2], h[GJ];
  double rho[SRC ? GJ : 1], vel[SRC ? 3 : 1][SRC ? GJ : 1];
};

template <bool SRC, int GJ>
__global__ __launch_bounds__(GTH) void k_gradient(PlanDev P, const double *phi_, GradIO io, int periodic) {
  const int ntk = (P.nphi + 63) / 64, ntj = (P.ntheta + GJ - 1) / GJ;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  // theta-major tile order (adjacent rows in one workgroup and, through the
  // XCD-aware workgroup order, on one L2)
  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x) * 4 + w;
  const int tj = tile % ntj, tk = tile / ntj;
  const int k = tk * 64 + lane;
  const bool kin = tk < ntk && k < P.nphi;   // the last workgroup may hold tiles past the mesh
  const int j0 = tj * GJ, nj = min(GJ, P.ntheta - j0);
  const long ncell = (long)P.ntheta * P.nphi;
  const auto te = gmem(P.theta_edges), pe = gmem(P.phi_edges);

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
  // the column this lane loads, and where its phi neighbours come from: the
  // cell itself (one-sided), the adjacent lane (which holds column k - 1,
  // resp. k + 1 modulo nphi on a closed circle), or the halo load of an end
  // lane
  const int kc = periodic ? k % P.nphi : min(k, P.nphi - 1);
  const bool lo_self = klo == k, hi_self = khi == k;
  const bool lo_load = !lo_self && lane == 0, hi_load = !hi_self && lane == 63;
  const int kh = lo_load ? klo : hi_load ? khi : kc;

  // theta: reciprocal widths of the tile's rows (one-sided at the poles)
  double inv_th[GJ];
#pragma unroll
  for (int u = 0; u < GJ; ++u) {
    const int j = j0 + u, jl = j > 0 ? j - 1 : j, jh = j < P.ntheta - 1 ? j + 1 : j;
    inv_th[u] = (u < nj && P.ntheta > 1) ? 1.0 / (centre(te, jh) - centre(te, jl)) : 0.0;
  }

  // rows of the tile and its halo rows, clamped to the mesh (uniform), and
  // the lane's byte offsets within a row
  int jrow[GJ + 2];
#pragma unroll
  for (int u = 0; u < GJ + 2; ++u) jrow[u] = min(max(j0 + u - 1, 0), P.ntheta - 1);
  // Every access is unconditional, so that no wait has to count a path
  // without it: a missing array (a null output or velocity component) and
  // the rows of a ragged tile past the mesh get a descriptor of size zero,
  // and the lanes past the mesh store at an offset past any row; the
  // hardware's range check then drops such stores and returns zero for such
  // loads (a missing velocity component counts as zero).
  const unsigned om = 8u * (unsigned)kc, oh = 8u * (unsigned)kh, ost = kin ? om : 0x80000000u;
  const int rowb = 8 * P.nphi;
  auto row = [&](const double *p, int i, int u, bool live) __attribute__((always_inline)) {
    return live ? row_rsrc(p + (size_t)i * ncell + (size_t)jrow[u] * P.nphi, rowb) : row_rsrc(phi_, 0);
  };

  auto load = [&](Shell<SRC, GJ> &b, int i) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < GJ + 2; ++u) b.v[u] = bload(row(phi_, i, u, true), om);
#pragma unroll
    for (int u = 0; u < GJ; ++u) b.h[u] = bload(row(phi_, i, u + 1, true), oh);
    if constexpr (SRC) {
#pragma unroll
      for (int u = 0; u < GJ; ++u) {
        b.rho[u] = bload(row(io.rho, i, u + 1, true), om);
#pragma unroll
        for (int c = 0; c < 3; ++c) b.vel[c][u] = bload(row(io.v[c], i, u + 1, io.v[c] != nullptr), om);
      }
    }
  };

  const int i0 = blockIdx.y * GR, i1 = min(P.nr, i0 + GR);
  // the previous shell's tile rows (the first shell: itself, one-sided)
  double pv[GJ];
#pragma unroll
  for (int u = 0; u < GJ; ++u) pv[u] = bload(row(phi_, max(i0 - 1, 0), u + 1, true), om);
  // three shell buffers, rotated by the fully unrolled shell loop
  Shell<SRC, GJ> sb[3];
  load(sb[0], i0);
  load(sb[1], min(i0 + 1, P.nr - 1));   // the last shell: itself, one-sided

#pragma unroll
  for (int s = 0; s < GR; ++s) {
    // difference shell i (cur) against its neighbours (pv, nxt) while the
    // loads of shell i + 2 (far) are in flight
    const int i = i0 + s;
    Shell<SRC, GJ> &cur = sb[s % 3], &nxt = sb[(s + 1) % 3], &far = sb[(s + 2) % 3];
    // unconditional (a chunk's last shells past the mesh load a clamped
    // copy): a load behind a branch would make every later wait count the
    // path without it, and so wait for these loads too
    if (s + 1 < GR) load(far, min(i + 2, P.nr - 1));   // the last step's nxt is shell i0 + GR
    double inv_r = 0.0;   // one-sided at the first and last shell, zero for one shell
    if (P.nr > 1) {
      const int lo = i > 0 ? i - 1 : i, hi = i + 1 < P.nr ? i + 1 : i;
      const double xl = 0.5 * (ld_const(P.r_edges + lo) + ld_const(P.r_edges + lo + 1));
      const double xh = 0.5 * (ld_const(P.r_edges + hi) + ld_const(P.r_edges + hi + 1));
      inv_r = 1.0 / (xh - xl);
    }
#pragma unroll
    for (int u = 0; u < GJ; ++u) {
      const double c0 = cur.v[u + 1];
      // every lane takes part in the shifts; only cells of the mesh are stored
      const double left = from_below(c0), right = from_above(c0);
      const double gr = (nxt.v[u + 1] - pv[u]) * inv_r;
      const double gt = (cur.v[u + 2] - cur.v[u]) * inv_th[u];
      const double gp = ((hi_self ? c0 : hi_load ? cur.h[u] : right) - (lo_self ? c0 : lo_load ? cur.h[u] : left)) * inv_ph;
      pv[u] = c0;
      auto out = [&](int c) __attribute__((always_inline)) { return row(io.o[c], i, u + 1, io.o[c] != nullptr && u < nj); };
      if constexpr (!SRC) {
        bstore(out(0), ost, gr);
        bstore(out(1), ost, gt);
        bstore(out(2), ost, gp);
      } else {
        const double nrho = -cur.rho[u];
        bstore(out(0), ost, nrho * gr);
        bstore(out(1), ost, nrho * gt);
        bstore(out(2), ost, nrho * gp);
        bstore(out(3), ost, nrho * (cur.vel[0][u] * gr + cur.vel[1][u] * gt + cur.vel[2][u] * gp));
      }
    }
    if (i + 1 >= i1) break;
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
