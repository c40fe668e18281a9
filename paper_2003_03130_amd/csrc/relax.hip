// Plate compression steps for gfx950 (forward and adjoint), stand-alone
// passes over the nodes of every cell.  The per-node arithmetic and the
// reading of the compression setup are in plate.h; the force and adjoint
// passes can also apply the same steps in their epilogues.  One workgroup
// per cell: the cell's nodes are contiguous in the internal order; each
// thread walks a fixed strided subset and the per-cell force is reduced in
// a fixed order, so the result is deterministic.
#include <hip/hip_runtime.h>

#include "aux_kernels.h"
#include "plate.h"

namespace cm {
namespace {

constexpr int kRelaxThreads = 1024;

struct StepArgs {
  const int64_t* node_off;
  int64_t N;
  const float* y;
  const float* f;
  const double* plate;  // per cell: top, bottom
  double k, m;
  float* y_next;
  double* force;
};

// Workgroup sum in a fixed order: a butterfly inside each wavefront, then
// the wavefront totals in wavefront order (deterministic).
__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < kRelaxThreads / 64; ++w) r += red[w];
  return r;
}

__global__ __launch_bounds__(kRelaxThreads) void plate_step_kernel(StepArgs a) {
  __shared__ double red[kRelaxThreads / 64];
  const int c = blockIdx.x;
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1];
  const float top = (float)a.plate[2 * c], bot = (float)a.plate[2 * c + 1];
  const float k = (float)a.k, m = (float)a.m;
  const int64_t N = a.N;
  double acc = 0.0;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kRelaxThreads) {
    const float z = a.y[2 * N + i];
    plate_node_step(a.y[i], a.y[N + i], z, a.f[i], a.f[N + i], a.f[2 * N + i], top,
                    bot, k, m, a.y_next, N, i);
    acc += plate_top_term(z, top, k);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0 && a.force) a.force[c] = s;
}

struct AdjArgs {
  const int64_t* node_off;
  int64_t N;
  const float* y;
  const float* lam_next;
  const float* ybar_el;
  const double* plate;
  double k, m;
  const double* F_meas;    // nullable (with F_target)
  const double* F_target;  // nullable: no loss term at this step
  double scale;
  const double* thetabar_el;  // nullable (with thetabar_acc)
  double* thetabar_acc;
  int n_regions;              // material slots per cell (3 gradient entries each)
  float* lam;
};

// The reverse step of plate_step_kernel (plate.h).
__global__ __launch_bounds__(kRelaxThreads) void plate_adjoint_kernel(AdjArgs a) {
  const int c = blockIdx.x;
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1];
  const float top = (float)a.plate[2 * c], bot = (float)a.plate[2 * c + 1];
  const float k = (float)a.k, m = (float)a.m;
  const float g = plate_loss_weight(a.F_meas, a.F_target, a.scale, c);
  const int64_t N = a.N;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kRelaxThreads)
    plate_node_adjoint(a.y[2 * N + i], a.lam_next[i], a.lam_next[N + i],
                       a.lam_next[2 * N + i], a.ybar_el[i], a.ybar_el[N + i],
                       a.ybar_el[2 * N + i], top, bot, k, m, g, a.lam, N, i);
  const int nq = 3 * a.n_regions;
  if ((int)threadIdx.x < nq && a.thetabar_acc) {
    const int64_t q = (int64_t)nq * c + threadIdx.x;
    a.thetabar_acc[q] += a.m * a.thetabar_el[q];
  }
}

}  // namespace

hipError_t launch_plate_step(const int64_t* node_off, int64_t N, int32_t n_cells,
                             const float* y, const float* f, const double* plate,
                             double k, double m, float* y_next, double* force,
                             hipStream_t st) {
  StepArgs a{node_off, N, y, f, plate, k, m, y_next, force};
  hipLaunchKernelGGL(plate_step_kernel, dim3(n_cells), dim3(kRelaxThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_plate_adjoint(const int64_t* node_off, int64_t N,
                                int32_t n_cells, const float* y,
                                const float* lam_next, const float* ybar_el,
                                const double* plate, double k, double m,
                                const double* F_meas, const double* F_target,
                                double scale, const double* thetabar_el,
                                double* thetabar_acc, int n_regions, float* lam,
                                hipStream_t st) {
  AdjArgs a{node_off, N, y, lam_next, ybar_el, plate, k, m, F_meas, F_target,
            scale, thetabar_el, thetabar_acc, n_regions, lam};
  hipLaunchKernelGGL(plate_adjoint_kernel, dim3(n_cells), dim3(kRelaxThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace cm
