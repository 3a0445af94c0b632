// Device code of the broadcast of merged blocks' potentials (shared by the
// per-phase kernel and the persistent batched launch).  In a class whose
// block map is made of theta bands (every block of rows [j0, j0 + nj) an
// nj x nk rectangle at a phi column divisible by nk), the expansion writes
// each merged block's value to its first cell only, and this step copies it
// to the block's other cells: a thread per cell, coalesced, instead of one
// lane writing a whole block (whose tiles would then carry up to 16 times the
// stores of a tile of single cells).  The first cells are never written
// here, so reading them in place is safe.
#pragma once
#include "device_util.h"

namespace mpole {
namespace {

// Item J.local = (shell i, first band t0): bands [t0, t0 + kBcastBands) of
// the shell's merged-block bands (every item has bands).
__device__ __forceinline__ void bcast_item(const BatchDev &B, const Job &J) {
  const PlanDev &P = J.P;
  const int2 it = ld_const(P.bcast_items + J.local);
  const int i = it.x, t0 = it.y;
  const ClassDev C = ld_const(P.classes + ld_const(P.shell_class + i));
  const int nb = min(kBcastBands, C.nbcast - t0);
  const auto phi = gmem(J.io.phi + (size_t)i * P.ncell);
  // up to kBcastCells cells per thread and band with all loads issued before
  // the stores, then what is left of taller bands a cell at a time
  constexpr int kBcastCells = 4;
  double v[kBcastBands][kBcastCells];
  int dst[kBcastBands][kBcastCells];
  int4 bd[kBcastBands];
#pragma unroll
  for (int t = 0; t < kBcastBands; ++t)
    bd[t] = t < nb ? ld_const(C.bands + ld_const(C.bcast + t0 + t)) : int4{0, 0, 1, 1};
#pragma unroll
  for (int t = 0; t < kBcastBands; ++t)
#pragma unroll
    for (int u = 0; u < kBcastCells; ++u) {
      const int q = item_tid() + u * 256;
      const int j = q / P.nphi, k = q - j * P.nphi, k0 = k - k % bd[t].z;
      const bool live = t < nb && j < bd[t].y && (j > 0 || k != k0);   // not the block's first cell
      dst[t][u] = live ? (bd[t].x + j) * P.nphi + k : -1;
      v[t][u] = live ? phi[bd[t].x * P.nphi + k0] : 0.0;
    }
#pragma unroll
  for (int t = 0; t < kBcastBands; ++t)
#pragma unroll
    for (int u = 0; u < kBcastCells; ++u)
      if (dst[t][u] >= 0) phi[dst[t][u]] = v[t][u];
  for (int t = 0; t < nb; ++t) {
    const int4 bt = ld_const(C.bands + ld_const(C.bcast + t0 + t));
    for (int q = item_tid() + kBcastCells * 256; q < bt.y * P.nphi; q += 256) {
      const int j = q / P.nphi, k = q - j * P.nphi, k0 = k - k % bt.z;
      phi[(bt.x + j) * P.nphi + k] = phi[bt.x * P.nphi + k0];
    }
  }
  stamp_done(B, J.f);
}

}  // namespace
}  // namespace mpole
