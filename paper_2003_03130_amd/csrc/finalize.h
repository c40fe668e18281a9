// Sums of the finalize kernels, each in a fixed order (deterministic):
// per cell the tile energies and inverted counts, per material slot the
// parameter-gradient sums, per shared node its slot partials.
#pragma once
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"

namespace cm {

// Energy, inverted count and (with nonfin) non-finite count of cell c over
// its tiles, on every lane of the wave: lane l takes tiles l, l + 64, ...,
// then a fixed butterfly (the cells' long chains of loads run in parallel).
struct CellSums {
  double e;
  int ni, nf;
};
__device__ __forceinline__ CellSums cell_sums(const DeviceTables& T, int c, int lane,
                                              bool nonfin) {
  CellSums s{0.0, 0, 0};
  const int t0 = T.cell_tile_first[c], nt = T.cell_tile_count[c];
  for (int k = lane; k < nt; k += 64) {
    const int64_t t = t0 + (int64_t)k * T.tile_stride;
    s.e += T.tile_acc[t];
    s.ni += T.tile_ninv[t];
    if (nonfin) s.nf += T.tile_nonfin[t];
  }
  s.e = wave_sum(s.e);
  s.ni = wave_sum(s.ni);
  if (nonfin) s.nf = wave_sum(s.nf);
  return s;
}

// dL/d(mu, kappa, w) of material slot mt, on every lane of the wave:
//   dL/dmu = w g_I + (1 - w) g_K, dL/dkappa = g_J, dL/dw = mu (g_I - g_K)
// from its tiles' sums (tile_acc, three per tile) of dL/d(mu1, mu2, kappa)
// with mu1 = w mu, mu2 = (1 - w) mu; lane l takes tiles l, l + 64, ...,
// then a fixed butterfly.
__device__ __forceinline__ void slot_theta(const DeviceTables& T, const double* tile_acc,
                                           int mt, int lane, double t3[3]) {
  double gI = 0.0, gK = 0.0, gJ = 0.0;
  const int t0 = T.mat_tile_first[mt], nt = T.mat_tile_count[mt];
  for (int k = lane; k < nt; k += 64) {
    const int64_t t = t0 + (int64_t)k * T.tile_stride;
    gI += tile_acc[3 * t];
    gK += tile_acc[3 * t + 1];
    gJ += tile_acc[3 * t + 2];
  }
  gI = wave_sum(gI);
  gK = wave_sum(gK);
  gJ = wave_sum(gJ);
  const int nm = T.n_mat;
  const double mu = T.params[mt], w = T.params[2 * nm + mt];
  t3[0] = w * gI + (1.0 - w) * gK;
  t3[1] = gJ;
  t3[2] = mu * (gI - gK);
}

// Sum of shared node s's slot partials (part, three floats per slot) in
// tile order.
__device__ __forceinline__ float3 shared_sum(const DeviceTables& T, const float* part,
                                             int s) {
  float sx = 0.f, sy = 0.f, sz = 0.f;
  for (int q = T.shared_slot_ptr[s]; q < T.shared_slot_ptr[s + 1]; ++q) {
    const float* pp = part + 3 * (int64_t)T.shared_slots[q];
    sx += pp[0];
    sy += pp[1];
    sz += pp[2];
  }
  return make_float3(sx, sy, sz);
}

}  // namespace cm
