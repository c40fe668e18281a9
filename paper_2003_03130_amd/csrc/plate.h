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

// Top-plate force of the nodes [n0, n1) of one cell, reduced in one fixed
// order whatever the workgroup size NT (a divisor of 1024 and a multiple of
// 64): virtual thread v < 1024 sums the nodes n0 + v, n0 + v + 1024, ...;
// the 64 virtual threads of each virtual wavefront are combined by a
// butterfly and the 16 wavefront totals in order.  red: 16 doubles of
// LDS.  Every thread of the workgroup must call it; all get the total.
template <int NT>
__device__ double plate_force_sum(const float* z, int64_t n0, int64_t n1,
                                  float top, float k, double* red) {
  static_assert(1024 % NT == 0 && NT % 64 == 0, "workgroup size");
  constexpr int J = 1024 / NT;
  double acc[J];
#pragma unroll
  for (int j = 0; j < J; ++j) acc[j] = 0.0;
  // the J virtual threads of a thread advance together (independent loads)
  for (int64_t b = n0 + threadIdx.x; b < n1; b += 1024) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int64_t i = b + j * NT;
      if (i < n1) {
        const float dt = fmaxf(z[i] - top, 0.f);
        acc[j] += (double)(k * dt * dt);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    double v = acc[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[(threadIdx.x + j * NT) >> 6] = v;
  }
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < 16; ++w) r += red[w];
  __syncthreads();  // red may be reused after the return
  return r;
}

}  // namespace cm
