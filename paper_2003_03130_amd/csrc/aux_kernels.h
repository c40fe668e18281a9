// Launch interface of the per-cell auxiliary kernels (host side): plate
// compression steps and their adjoint, quasi-static compression, shape
// diagnostics.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace cm {

// Shape diagnostics (Taylor deformation, cell strain): kShapeFields float64
// per cell = volume, centre of mass (3), semi-axes a1 <= a2 <= a3, D, d_max,
// strain.  mom: 10 float64 per tile; d2max: one uint64 per cell;
// pair_blocks: (cell, row block, column block, 0) over the 256-node blocks
// of every cell with row <= column.
constexpr int kShapeFields = 10;
size_t shape_lds(int nloc);
hipError_t launch_shape(const DeviceTables& T, const int64_t* node_off,
                        const int4* pair_blocks, int64_t n_pair_blocks,
                        const float* y, const double* d_ref, double* mom,
                        unsigned long long* d2max, double* out,
                        hipStream_t st);

// Quasi-static plate compression (one workgroup per cell): Newton residual,
// one conjugate-gradient iteration, bounded Newton update, plate predictor.
// Per-cell state: kQsState float64 = |r|^2, |r_0|^2, active, |f + p|^2,
// applied step scale, |penalty|^2, largest node move of the last step, spare.
constexpr int kQsState = 8;
hipError_t launch_qs_residual(const int64_t* node_off, int64_t N, int32_t n_cells,
                              const float* y, const float* f, const double* plate,
                              double k, double abs_tol, double rel_tol,
                              double step_tol, int restart, float* r, float* p,
                              float* x, double* st, double* force, hipStream_t s);
hipError_t launch_qs_cg(const int64_t* node_off, int64_t N, int32_t n_cells,
                        const float* y, const double* plate, double k,
                        double rel_tol, const float* ybar, float* x, float* r,
                        float* p, float* Ap, double* st, hipStream_t s);
hipError_t launch_qs_update(const int64_t* node_off, int64_t N, int32_t n_cells,
                            const float* x, double cap, float* y, double* st,
                            hipStream_t s);
hipError_t launch_qs_predict(const int64_t* node_off, int64_t N, int32_t n_cells,
                             const double* plate_old, const double* plate_new,
                             float* y, hipStream_t s);

// Plate compression step and its adjoint (one workgroup per cell).
hipError_t launch_plate_step(const int64_t* node_off, int64_t N, int32_t n_cells,
                             const float* y, const float* f, const double* plate,
                             double k, double m, float* y_next, double* force,
                             hipStream_t st);
hipError_t launch_plate_adjoint(const int64_t* node_off, int64_t N,
                                int32_t n_cells, const float* y,
                                const float* lam_next, const float* ybar_el,
                                const double* plate, double k, double m,
                                const double* F_meas, const double* F_target,
                                double scale, const double* thetabar_el,
                                double* thetabar_acc, int n_regions, float* lam,
                                hipStream_t st);

}  // namespace cm
