// Device helpers shared by the forward and backward kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace cm {

// LDS written by one lane is read by other lanes of the same wavefront only
// after this point: LDS instructions of a wavefront execute in order, so a
// compiler-level fence plus a wave barrier is enough.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// One lane's tetrahedron of a chunk: packed local indices, B and V0.
struct TetRegs {
  uint2 q;
  float B[9];
  float V0;
};

// Chunks are read once per pass: three 16-byte loads per lane, each row of
// the chunk 1,024 contiguous bytes (16-byte loads stream at about 1.5 times
// the rate of 4-byte ones), non-temporal so that the chunk stream does not
// displace the node data that neighbouring tiles reuse from the caches.
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load_tet(const TetChunk* ch, int lane,
                                         TetRegs& r) {
  const u32x4_t va = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(ch->a[lane]));
  const f32x4_t vb = __builtin_nontemporal_load(reinterpret_cast<const f32x4_t*>(ch->b[lane]));
  const f32x4_t vc = __builtin_nontemporal_load(reinterpret_cast<const f32x4_t*>(ch->c[lane]));
  r.q.x = va.x;
  r.q.y = va.y;
  r.V0 = __uint_as_float(va.z);
  r.B[0] = __uint_as_float(va.w);
  r.B[1] = vb.x; r.B[2] = vb.y; r.B[3] = vb.z; r.B[4] = vb.w;
  r.B[5] = vc.x; r.B[6] = vc.y; r.B[7] = vc.z; r.B[8] = vc.w;
}

// Adds the contributions h[0..2] of vertex slots 0..2 and -(h0 + h1 + h2) of
// slot 3 to the accumulators acc(i_s) (acc maps a tile-local node index to
// its three accumulator floats).  The layout guarantees that the active
// lanes of the wave name distinct nodes within each slot, so each slot is
// one LDS read and one LDS write per lane with no races; slots are processed
// in order (LDS instructions of a wavefront execute in order).
template <class Acc>
__device__ __forceinline__ void lds_accumulate(Acc acc, int i0, int i1, int i2,
                                               int i3, const float h[3][3]) {
  float* a = acc(i0);
  a[0] += h[0][0]; a[1] += h[0][1]; a[2] += h[0][2];
  a = acc(i1);
  a[0] += h[1][0]; a[1] += h[1][1]; a[2] += h[1][2];
  a = acc(i2);
  a[0] += h[2][0]; a[1] += h[2][1]; a[2] += h[2][2];
  a = acc(i3);
  a[0] -= h[0][0] + h[1][0] + h[2][0];
  a[1] -= h[0][1] + h[1][1] + h[2][1];
  a[2] -= h[0][2] + h[1][2] + h[2][2];
}

// Runs body(regs) over the n chunks ch[0..n) with the next chunk's loads in
// flight while the current one is evaluated; two register sets alternate, so
// no register copies are needed between chunks.  Every call site of body is
// reached with one fixed set of outstanding loads (one chunk in flight, or
// none at the last chunk), so the compiler waits only for the chunk that
// body reads.
// As for_each_chunk, with the first chunk's registers ra loaded by the
// caller (before the tile's nodes are staged, so that its loads are in
// flight meanwhile).
template <class Body>
__device__ __forceinline__ void for_each_chunk_from(const TetChunk* ch, int n,
                                                    int lane, TetRegs ra, Body body) {
  if (n <= 0) return;
  TetRegs rb;
  for (int k = 0;; k += 2) {
    if (k + 1 >= n) {
      body(ra);
      return;
    }
    load_tet(ch + k + 1, lane, rb);
    body(ra);
    if (k + 2 >= n) {
      body(rb);
      return;
    }
    load_tet(ch + k + 2, lane, ra);
    body(rb);
  }
}

template <class Body>
__device__ __forceinline__ void for_each_chunk(const TetChunk* ch, int n,
                                               int lane, Body body) {
  if (n <= 0) return;
  TetRegs ra;
  load_tet(ch, lane, ra);
  for_each_chunk_from(ch, n, lane, ra, body);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous run of logical block ids so neighbouring tiles (which share
// nodes) run under the same L2.
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int x = b & 7, j = b >> 3, q = G >> 3, r = G & 7;
  return x * q + (x < r ? x : r) + j;
}

// Tiles [t0, t1) of logical block lb out of G.
__device__ __forceinline__ void block_tiles(const Range& r, int& t0, int& t1) {
  const int G = gridDim.x;
  const int lb = xcd_block(blockIdx.x, G);
  const int64_t ntl = r.tile_end - r.tile_begin;
  t0 = r.tile_begin + (int)((int64_t)lb * ntl / G);
  t1 = r.tile_begin + (int)((int64_t)(lb + 1) * ntl / G);
}

inline int grid_for(const Range& r, const LaunchCfg& cfg) {
  const int64_t ntl = r.tile_end - r.tile_begin;
  const int64_t groups = (ntl + cfg.waves - 1) / cfg.waves;
  int64_t g = cfg.blocks > 0 ? std::min<int64_t>(cfg.blocks, groups) : groups;
  return (int)std::max<int64_t>(g, 1);
}

}  // namespace cm
