// Host-side preparation of tetrahedral cells for the device kernels.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "layout.h"

namespace cm {

struct PrepOptions {
  int order = 3;                // 0 input, 1 RCM, 2 Morton, 3 bisection
  int tile_tets = 768;         // multiple of 64, <= kMaxTileTets
  double degenerate_tol = 1e-12;
};

// Everything the device needs, in host memory, for all cells.
struct Prepared {
  int64_t n_cells = 0, n_nodes = 0, n_tets = 0;
  std::vector<TileDesc> tiles;
  std::vector<TetChunk> chunks;
  std::vector<uint64_t> chunk_neg;       // per chunk: bit l set when lane l's
                                         // reference orientation is negative
  std::vector<int32_t> slot_node;        // internal node id of every slot
  std::vector<int32_t> shared_node;      // internal node id of every shared node
  std::vector<int32_t> shared_slot_ptr;  // CSR (n_shared + 1) into shared_slots
  std::vector<int32_t> shared_slots;     // slot ids, grouped by shared node, in tile order
  std::vector<int32_t> cell_tile_off;    // n_cells + 1 (contiguous tiles per cell)
  std::vector<int32_t> cell_tile_first;  // n_cells: first tile of the cell
  std::vector<int32_t> cell_tile_count;  // n_cells: tiles of the cell
  int32_t tile_stride = 1;               // distance between a cell's tiles
  // Materials: slot c * n_regions + r holds the parameters of region r of
  // cell c; every tile lies in one region.  Tiles of a slot:
  // mat_tile_first[slot] + k * tile_stride, k < mat_tile_count[slot].
  int32_t n_regions = 1;
  std::vector<int32_t> tile_mat;          // n_tiles
  std::vector<int32_t> mat_tile_first;    // n_cells * n_regions
  std::vector<int32_t> mat_tile_count;
  std::vector<int32_t> cell_shared_off;  // n_cells + 1
  std::vector<int64_t> node_off;         // n_cells + 1 (same as input)
  std::vector<int64_t> new_to_old;       // n_nodes
  std::vector<int32_t> space_order;      // n_nodes: per cell, internal ids,
                                         // the cell's candidates for the
                                         // largest node distance first, each
                                         // part in Morton order of the
                                         // reference node
  std::vector<int32_t> cell_candidates;  // n_cells: leading candidates
  int32_t max_tile_nodes = 0;
  double volume = 0.0, min_v0 = 0.0, max_cond = 0.0;
};

// Returns 0 on success, or a CM_* status with `err` set.
// prepare_template: n_cells cells that share one reference mesh (n_nodes,
// n_tets, ref_xyz, tets).  The tet chunks are stored once; tile descriptors,
// slot and shared-node tables are replicated per cell with offsets, ordered
// template tile major and cell minor (tile k of every cell, then tile k + 1),
// so cell_tile_off is empty and the tiles of cell c are c + k * n_cells.
// tet_region (nullable, per tetrahedron in input order, each < n_regions)
// splits every cell into material regions.
int prepare_template(int32_t n_cells, int64_t n_nodes, int64_t n_tets,
                     const double* ref_xyz, const int32_t* tets,
                     const uint8_t* tet_region, int32_t n_regions,
                     const PrepOptions& opt, Prepared* out, std::string* err);

int prepare_batch(int32_t n_cells, const int64_t* node_off,
                  const int64_t* tet_off, const double* ref_xyz,
                  const int32_t* tets, const uint8_t* tet_region,
                  int32_t n_regions, const PrepOptions& opt, Prepared* out,
                  std::string* err);

}  // namespace cm
