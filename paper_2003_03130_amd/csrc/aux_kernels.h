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
// strain.  mom: 10 float64 per tile; d2max: one uint64 per cell; node
// blocks: (cell, block) for every candidate block of 256 nodes (a cell's
// nodes ordered candidates first), with a bounding box (6 float64) each;
// cand_blocks: (cell, row block, column block, first node block of the cell)
// over the candidate blocks of every cell with row <= column; chunk_neg: per
// chunk, the lanes of negative reference orientation.
constexpr int kShapeFields = 10;
size_t shape_lds(int nloc);
hipError_t launch_shape(const DeviceTables& T, const int64_t* node_off,
                        const int4* cand_blocks, int64_t n_cand_blocks,
                        const int2* node_blocks, int64_t n_node_blocks,
                        const int32_t* order, const float* y, const double* d_ref,
                        const uint64_t* chunk_neg, double* mom, int32_t* tile_inv,
                        int32_t* cell_inv,
                        double* bbox, unsigned long long* d2max, double* out,
                        hipStream_t st);

// Quasi-static plate compression (one workgroup per cell): Newton residual,
// one conjugate-gradient iteration, bounded Newton update, plate predictor.
// Per-cell state: kQsState float64 = 0 CG r . z (|r|^2 without
// preconditioner), 1 CG |r_0|^2, 2 CG active,
// 3 Newton |r_N|^2, 4 accepted step scale, 5 |penalty|^2, 6 largest node move
// of the last step, 7 float32 floor of the residual, 8 Pi(y), 9 line-search
// scale, 10 slope r_N . x, 11 not in equilibrium, 12 line search pending,
// 13 max |x|, 14 CG forcing term eta of the Newton step, 15 |r_N|^2 of the
// last residual (for the next forcing term).
constexpr int kQsState = 16;
hipError_t launch_qs_residual(const int64_t* node_off, int64_t N, int32_t n_cells,
                              const float* y, const float* f, const double* energy,
                              const double* plate, double k, double abs_tol,
                              double rel_tol, double step_tol, double floor_factor,
                              double eta_max, int restart, float* r, float* p,
                              float* x, float* rn, double* st, double* force,
                              const float* kel, float* minv, hipStream_t s,
                              const Indenter& ind = Indenter{});
hipError_t launch_qs_ls_start(const int64_t* node_off, int64_t N, int32_t n_cells,
                              float* x, const float* rn, double cap,
                              const float* y, float* yt, double* st, hipStream_t s);
hipError_t launch_qs_ls_accept(const int64_t* node_off, int64_t N, int32_t n_cells,
                               const float* x, const double* plate, double k,
                               const double* energy_t, double armijo,
                               double min_move, float* y, float* yt, double* st,
                               const int32_t* ninv_t, int32_t* ninv, hipStream_t s,
                               const Indenter& ind = Indenter{});
hipError_t launch_qs_noise(const int64_t* node_off, int64_t N, int32_t n_cells,
                           const float* y, float* e, hipStream_t s);
hipError_t launch_qs_floor(const int64_t* node_off, int64_t N, int32_t n_cells,
                           const float* y, const double* plate, double k,
                           const float* e, const float* ybar, double* st,
                           hipStream_t s, const Indenter& ind = Indenter{});
// Start of the adjoint CG solve Hess(Pi) lam = weight_c dF_top/dy (under the
// sphere, of the projected system).
hipError_t launch_qs_adjoint_rhs(const int64_t* node_off, int64_t N, int32_t n_cells,
                                 const float* y, const double* plate, double k,
                                 const double* weight, float* r, float* p, float* x,
                                 double* st, const float* minv, hipStream_t s,
                                 const Indenter& ind = Indenter{});
// With slots set, ybar holds the owned nodes only (a backward tile pass
// without its finalize) and the shared nodes' values are summed from the
// slot partials of those tables (bitwise the finalize's sums).
hipError_t launch_qs_cg(const int64_t* node_off, int64_t N, int32_t n_cells,
                        const float* y, const double* plate, double k,
                        double rel_tol, const float* ybar, float* x, float* r,
                        float* p, float* Ap, double* st, const float* minv,
                        hipStream_t s, const DeviceTables* slots = nullptr,
                        const Indenter& ind = Indenter{});
// Small-strain stiffness blocks (the Newton preconditioner), 6 n_nodes
// floats SoA: xx yy zz xy xz yz; uses the forward scratch.
hipError_t launch_qs_stiffness(const DeviceTables& T, const Range& r, float* kel,
                               hipStream_t s);
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
