// Device code of the per-solve coefficient step of the dense paths (shared by
// the per-phase kernel and the persistent batched launch): one workgroup
// per shell splits its expansion coefficients with a power-of-two scale
// (split precisions) or copies them into the expansion mode columns (FP64
// folded plans).
#pragma once
#include "device_util.h"
#include "split_util.h"

namespace mpole {
namespace {

// One workgroup per shell: scale and split the expansion coefficients.
template <int KIND>
__device__ __forceinline__ void split_coef_item(const Job &J, double *red) {
  const PlanDev &P = J.P;
  const int i = J.local;
  const double *__restrict__ c = P.coef + (size_t)i * P.namp;
  double mx = 0.0;
  for (int n = item_tid() + 1; n < P.nam; n += 256) mx = fmax(mx, fabs(c[n]));
  const double scale = row_scale(block_max(mx, red));
  const double inv = 1.0 / scale;
  // expansion mode columns; the l = 0 term is added in FP64 by the expansion
  // epilogue
  for (int col = item_tid(); col < P.namp_e; col += 256) {
    const int n = P.perm_e ? P.perm_e[col] : col;
    split_store<KIND>((n > 0 && n < P.nam) ? c[n] * inv : 0.0, P.cplanes + slab_index<KIND>(i, col, P.nr), 16);
  }
  if (item_tid() == 0) P.cscale[i] = scale;
}

// Folded FP64: the coefficients of one shell in expansion mode columns.
__device__ __forceinline__ void perm_coef_item(const Job &J) {
  const PlanDev &P = J.P;
  const int i = J.local;
  const double *__restrict__ c = P.coef + (size_t)i * P.namp;
  for (int col = item_tid(); col < P.namp_e; col += 256) {
    const int n = P.perm_e[col];
    P.coef_e[(size_t)i * P.namp_e + col] = (n >= 0 && n < P.nam) ? c[n] : 0.0;
  }
}

}  // namespace
}  // namespace mpole
