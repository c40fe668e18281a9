// Per-node arithmetic of the plate-compression step and of its adjoint,
// shared by the stand-alone plate kernels and by the force / adjoint passes
// that fuse the step into their epilogues (PlateFwd, PlateBwd), so that both
// routes compute the same floating-point operations.
//
// Reading of the compression setup (its force law and time integration are
// in the paper's unavailable supporting information): overdamped explicit
// steps with a quadratic penalty,
//   p_z = -k max(0, y_z - top)^2 + k max(0, bottom - y_z)^2,
//   y_next = y + m (f + p),   F = k sum max(0, y_z - top)^2,
// and the reverse step for a loss scale (F - F_target)^2 at this step,
//   lam = lam_next + m ((df/dy)^T lam_next + dp/dy lam_next) + g dF/dy,
// g = 2 scale (F - F_target), dp_z/dy_z = -2k (max(0, z - top) +
// max(0, bottom - z)), dF/dy_z = 2k max(0, z - top).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace cm {

__device__ inline void plate_node_step(float yx, float yy, float yz, float fx,
                                       float fy, float fz, float top, float bot,
                                       float k, float m, float* y_next,
                                       int64_t N, int64_t g) {
  const float dt = fmaxf(yz - top, 0.f), db = fmaxf(bot - yz, 0.f);
  const float pz = k * (db * db - dt * dt);
  y_next[g] = yx + m * fx;
  y_next[N + g] = yy + m * fy;
  y_next[2 * N + g] = yz + m * (fz + pz);
}

// g of the reverse step for cell c (0 without a loss term at this step).
__device__ inline float plate_loss_weight(const double* F_meas,
                                          const double* F_target, double scale,
                                          int c) {
  return F_target ? (float)(2.0 * scale * (F_meas[c] - F_target[c])) : 0.f;
}

// lx, ly, lz: lam_next; bx, by, bz: (df/dy)^T lam_next at the node.
__device__ inline void plate_node_adjoint(float yz, float lx, float ly, float lz,
                                          float bx, float by, float bz,
                                          float top, float bot, float k,
                                          float m, float g, float* lam,
                                          int64_t N, int64_t i) {
  const float dt = fmaxf(yz - top, 0.f), db = fmaxf(bot - yz, 0.f);
  lam[i] = lx + m * bx;
  lam[N + i] = ly + m * by;
  lam[2 * N + i] = lz + m * (bz - 2.f * k * (dt + db) * lz) + g * 2.f * k * dt;
}

// One node's term of the top-plate force, k max(0, z - top)^2 (float32
// product, accumulated in float64 by the callers).
__device__ inline double plate_top_term(float z, float top, float k) {
  const float dt = fmaxf(z - top, 0.f);
  return (double)(k * dt * dt);
}

}  // namespace cm
