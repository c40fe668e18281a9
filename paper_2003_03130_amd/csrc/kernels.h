// Launch interface of the device kernels (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.h"

namespace cm {

// Device-resident tables of a prepared batch (see layout.h).
struct DeviceTables {
  const TileDesc* tiles = nullptr;
  const TetChunk* chunks = nullptr;
  const int32_t* slot_node = nullptr;
  const int32_t* shared_node = nullptr;
  const int32_t* shared_slot_ptr = nullptr;
  const int32_t* shared_slots = nullptr;
  const int32_t* shared_cell = nullptr;  // cell of every shared node
  const int32_t* cell_shared_off = nullptr;  // shared nodes of cell c: [off[c], off[c + 1])
  const int32_t* cell_shared_first = nullptr;  // node id of shared_node[off[c]]
  // slot_node with bit 31 set on the first slot of every shared node (the
  // one slot whose tile adds the node's top-plate force to its sum)
  const int32_t* slot_node_first = nullptr;
  // shared nodes of no tetrahedron, per cell: orphan_node[orphan_off[c] ..
  // orphan_off[c + 1])
  const int32_t* orphan_off = nullptr;
  const int32_t* orphan_node = nullptr;
  // tiles of cell c: cell_tile_first[c] + k * tile_stride, k < cell_tile_count[c]
  const int32_t* cell_tile_first = nullptr;
  const int32_t* cell_tile_count = nullptr;
  int32_t tile_stride = 1;
  // material slot of every tile (cell * n_regions + region); tiles of slot
  // m: mat_tile_first[m] + k * tile_stride, k < mat_tile_count[m]
  const int32_t* tile_mat = nullptr;
  const int32_t* mat_tile_first = nullptr;
  const int32_t* mat_tile_count = nullptr;
  int32_t n_regions = 1;
  int32_t n_mat = 0;               // n_cells * n_regions
  const double* params = nullptr;  // SoA: mu[n_mat], kappa[n_mat], w[n_mat]
  float* part = nullptr;           // slot partials, (x, y, z) per slot
  double* tile_acc = nullptr;      // per tile: energy (fwd) or 3 sums (bwd)
  double* tile_plate = nullptr;    // per tile: top-plate force (fwd)
  int32_t* tile_ninv = nullptr;    // per tile
  int32_t* tile_nonfin = nullptr;  // per tile: tets with a non-finite energy
                                   // or force (written by checked passes)
  int64_t n_nodes = 0, n_slots = 0, n_tiles = 0;
  int32_t n_cells = 0;
  int32_t nloc = 0;                // LDS node capacity per wave (multiple of 4)
};

// Work range of one launch: tiles, shared nodes and cells.
struct Range {
  int32_t tile_begin, tile_end;
  int32_t shared_begin, shared_end;
  int32_t cell_begin, cell_end;
};

// Restricts a backward pass to the cells c with flags[c * stride] != 0 (all
// cells when flags is null).
struct CellMask {
  const double* flags = nullptr;
  int64_t stride = 1;
};

// Arguments of a force pass with the plate step fused in: the pass writes
// y_next instead of the forces, and the top-plate force per cell.
struct PlateFwd {
  const double* plate = nullptr;     // per cell: top, bottom (null: no step)
  float k = 0.f, m = 0.f;
  float* y_next = nullptr;
  double* force = nullptr;           // per cell, nullable
};

// Arguments of an adjoint pass (fbar = lam_next, no energy cotangent) with
// the reverse plate step fused in: the pass writes lam instead of ybar and
// adds m thetabar to thetabar_acc instead of storing thetabar.
struct PlateBwd {
  const double* plate = nullptr;     // null: no step
  float k = 0.f, m = 0.f;
  double m64 = 0.0;
  const double* F_meas = nullptr;    // with F_target
  const double* F_target = nullptr;  // nullable: no loss term
  double scale = 0.0;
  double* thetabar_acc = nullptr;    // nullable
  float* lam = nullptr;
};

// Top contact of the quasi-static solver: R = 0 the flat top plate at the
// plate height; R > 0 a sphere of radius R with its lowest point at the plate
// height and its axis at (axis[2c], axis[2c + 1]) for cell c (the colloidal
// probe).  Under the sphere the cells' centroids are held laterally; geo
// receives per cell the centroid x, y and sum (dx^2 + dy^2) about it of the
// positions at the last Newton residual, for the CG's projections.
struct Indenter {
  double R = 0.0;
  const double* axis = nullptr;
  double* geo = nullptr;
};

struct LaunchCfg {
  int waves = 1;   // tiles (wavefronts) per workgroup: 1, 2, 4 or 8
  int blocks = 0;  // persistent workgroups; 0 = one workgroup per W tiles
};

// LDS bytes per wave of the forward / backward kernel for nloc tile nodes.
size_t forward_lds_per_wave(int nloc);
size_t backward_lds_per_wave(int nloc);
size_t forward_backward_lds_per_wave(int nloc);

// The two kernels of each pass, separately (for per-kernel timing).
// With pl.plate set, the forward pass applies one plate-compression step
// (see plate.h): it writes pl.y_next (and pl.force) instead of f, and the
// finalize kernel needs y.
// With check set, the tile pass counts per tile the tetrahedra whose energy
// or force contribution is not finite (T.tile_nonfin) and the finalize sums
// them per cell into nonfin.
hipError_t launch_forward_main(const DeviceTables& T, const Range& r,
                               const LaunchCfg& cfg, const float* y, float* f,
                               hipStream_t st, const PlateFwd& pl = PlateFwd{},
                               bool check = false);
hipError_t launch_forward_finalize(const DeviceTables& T, const Range& r,
                                   float* f, double* energy, int32_t* ninv,
                                   hipStream_t st, const float* y = nullptr,
                                   const PlateFwd& pl = PlateFwd{},
                                   int32_t* nonfin = nullptr);
// grad = false: the Hessian-vector product alone (ebar ignored, the per-tile
// parameter-gradient sums not written; the finalize must not form thetabar).
hipError_t launch_backward_main(const DeviceTables& T, const Range& r,
                                const LaunchCfg& cfg, const float* y,
                                const float* fbar, const double* ebar,
                                float* ybar, hipStream_t st,
                                const CellMask& mask = CellMask{},
                                const PlateBwd& pl = PlateBwd{}, bool grad = true);
// With pl.plate set, the backward pass (fbar = lam_next, no ebar) applies
// the reverse plate step: it writes pl.lam instead of ybar and adds m
// thetabar to pl.thetabar_acc; the finalize kernel needs y and lam_next.
hipError_t launch_backward_finalize(const DeviceTables& T, const Range& r,
                                    float* ybar, double* thetabar,
                                    hipStream_t st,
                                    const CellMask& mask = CellMask{},
                                    const float* y = nullptr,
                                    const float* lam_next = nullptr,
                                    const PlateBwd& pl = PlateBwd{});

hipError_t launch_forward(const DeviceTables& T, const Range& r,
                          const LaunchCfg& cfg, const float* y, float* f,
                          double* energy, int32_t* ninv, hipStream_t st,
                          const PlateFwd& pl = PlateFwd{},
                          int32_t* nonfin = nullptr);

hipError_t launch_backward(const DeviceTables& T, const Range& r,
                           const LaunchCfg& cfg, const float* y,
                           const float* fbar, const double* ebar, float* ybar,
                           double* thetabar, hipStream_t st,
                           const CellMask& mask = CellMask{},
                           const PlateBwd& pl = PlateBwd{});

// Forward and backward in one tile pass (fused.hip): the outputs of
// launch_forward (f, energy, ninv) and of launch_backward (ybar, thetabar)
// for cotangents fbar, ebar given up front, bitwise equal to the two
// separate passes.  T holds the forward's scratch, Tb the backward's (both
// with the same tiling).  The main kernel alone, for per-kernel timing:
hipError_t launch_forward_backward_main(const DeviceTables& T, const DeviceTables& Tb,
                                        const Range& r, const LaunchCfg& cfg,
                                        const float* y, float* f, const float* fbar,
                                        const double* ebar, float* ybar, hipStream_t st,
                                        bool grad = true);
hipError_t launch_forward_backward_finalize(const DeviceTables& T, const DeviceTables& Tb,
                                            const Range& r, float* f, double* energy,
                                            int32_t* ninv, float* ybar, double* thetabar,
                                            hipStream_t st);
hipError_t launch_forward_backward(const DeviceTables& T, const DeviceTables& Tb,
                                   const Range& r, const LaunchCfg& cfg, const float* y,
                                   float* f, double* energy, int32_t* ninv,
                                   const float* fbar, const double* ebar, float* ybar,
                                   double* thetabar, hipStream_t st);

}  // namespace cm
