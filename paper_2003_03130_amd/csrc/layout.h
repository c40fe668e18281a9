// Device data layout of a prepared batch of tetrahedral cells.
//
// Tetrahedra are grouped into tiles of at most `tile_tets` tetrahedra, one
// wavefront (64 lanes) per tile, processed 64 at a time ("chunks").  A tile's distinct vertices ("tile nodes")
// are staged in LDS; the tile's tetrahedra refer to them by 16-bit local
// index.  Nodes touched by exactly one tile are "owned" and numbered so that
// each tile's owned nodes form one contiguous internal range: the tile loads
// their positions and stores their forces with plain coalesced accesses.
// Nodes touched by several tiles are "shared": every (tile, shared node) pair
// is a "slot"; the tile writes its partial force to the slot, and a second
// pass sums the slots of each shared node in tile order.  No atomics are used
// anywhere and the result is deterministic.
#pragma once
#include <cstdint>

namespace cm {

constexpr int kChunk = 64;          // tetrahedra per chunk = lanes per wave
constexpr int kMaxTileTets = 4096;  // keeps local indices below 2^16
constexpr int kMaxRegions = 64;     // material regions per cell

// 32 bytes, read with scalar loads.
struct TileDesc {
  int32_t chunk_begin;  // index of the tile's first chunk
  int32_t n_tets;       // tetrahedra in the tile (<= tile_tets)
  int32_t own_begin;    // internal id of the tile's first owned node
  int32_t n_own;        // owned nodes: local indices [0, n_own)
  int32_t shr_begin;    // first slot of the tile
  int32_t n_shr;        // shared nodes: local indices [n_own, n_own + n_shr)
  int32_t cell;         // cell the tile belongs to
  int32_t n_chunks;     // chunks of the tile (lanes without a tetrahedron
                        // carry kEmptyLane in idx[lane][0])
};

// Marks a chunk lane that holds no tetrahedron.
constexpr uint32_t kEmptyLane = 0xffffffffu;

// 64 tetrahedra per chunk (3072 bytes).  Within a chunk the tetrahedra and
// the order of their vertices are chosen
// so that, for each vertex slot 0..3, the 64 lanes name 64 different tile
// nodes: the lanes of one wave can then add their contributions to the
// tile's LDS accumulators slot by slot with plain read-modify-writes and no
// two lanes of an instruction touch the same node.
// The 64 tetrahedra of a chunk are stored as three rows of 64 16-byte
// records, so that each row is one 16-byte load per lane over 1,024
// contiguous bytes:
//   a[l] = (v0 | v1 << 16, v2 | v3 << 16, bits of V0, bits of B[0])
//   b[l] = (B[1], B[2], B[3], B[4]),   c[l] = (B[5], B[6], B[7], B[8])
// with the 4 x uint16 local vertex indices, the reference volume
// V0 = |det J| / 6 and B = J^-1 row-major (B[3k + j], k = edge, j = axis).
// An empty lane has a[l][0] = a[l][1] = kEmptyLane and zeros elsewhere.
struct TetChunk {
  uint32_t a[kChunk][4];
  float b[kChunk][4];
  float c[kChunk][4];
};
static_assert(sizeof(TetChunk) == 3072, "chunk layout");
static_assert(sizeof(TileDesc) == 32, "tile layout");

}  // namespace cm
