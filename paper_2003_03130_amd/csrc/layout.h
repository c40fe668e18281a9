// Device data layout of a prepared batch of tetrahedral cells.
//
// Tetrahedra are grouped into tiles of at most `tile_tets` tetrahedra, one
// wavefront (64 lanes) per tile.  A tile's distinct vertices ("tile nodes")
// are staged in LDS; the tile's tetrahedra refer to them by 16-bit local
// index.  Nodes touched by exactly one tile are "owned" and numbered so that
// each tile's owned nodes form one contiguous internal range: the tile loads
// their positions and stores their forces with plain coalesced accesses.
// Nodes touched by several tiles are "shared": every (tile, shared node) pair
// is a "slot"; the tile writes its partial force to the slot, and a second
// pass sums the slots of each shared node in tile order.  No floating-point
// global atomics are used and the result is deterministic.
#pragma once
#include <cstdint>

namespace cm {

constexpr int kChunk = 64;          // tetrahedra per chunk = lanes per wave
constexpr int kMaxTileTets = 4096;  // keeps local indices below 2^16

// 32 bytes, read with scalar loads.
struct TileDesc {
  int32_t chunk_begin;  // index of the tile's first chunk
  int32_t n_tets;       // tetrahedra in the tile (<= tile_tets)
  int32_t own_begin;    // internal id of the tile's first owned node
  int32_t n_own;        // owned nodes: local indices [0, n_own)
  int32_t shr_begin;    // first slot of the tile
  int32_t n_shr;        // shared nodes: local indices [n_own, n_own + n_shr)
  int32_t cell;         // cell the tile belongs to
  int32_t pad;
};

// 64 tetrahedra, structure of arrays inside the chunk (3072 bytes): every
// lane of a wave reads its tetrahedron with fully coalesced loads.
struct TetChunk {
  uint32_t idx[kChunk][2];  // 4 x uint16 local vertex indices (v0|v1<<16, v2|v3<<16)
  float B[9][kChunk];       // B = J^-1, row-major B[k][j], k = edge, j = axis
  float V0[kChunk];         // reference volume |det J| / 6
};
static_assert(sizeof(TetChunk) == 3072, "chunk layout");
static_assert(sizeof(TileDesc) == 32, "tile layout");

}  // namespace cm
