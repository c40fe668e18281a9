// Forward (forces + energy) kernels for gfx950.
//
// One wavefront per tile.  A tile's nodes are staged in LDS (positions as
// float4, force accumulators as three float arrays); each lane evaluates one
// tetrahedron per 64-tetrahedron chunk and adds its 12 force components to
// the LDS accumulators with ds_add_f32.  Because a tile belongs to exactly
// one wavefront, the order of those additions is fixed by the lane order of
// each instruction and the chunk order, so results are bitwise repeatable.
// Owned nodes are then written straight to the output; shared nodes write a
// per-slot partial that the finalize kernel sums in tile order.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "mr_tet.h"

namespace cm {
namespace {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void lds_add(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
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

struct FwdArgs {
  DeviceTables T;
  Range r;
  const float* y;
  float* f;
};

template <int W>
__global__ __launch_bounds__(64 * W) void forward_kernel(FwdArgs a) {
  extern __shared__ float4 lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nloc = a.T.nloc;
  float4* ys = lds + (size_t)wave * (7 * nloc / 4);
  float* fx = reinterpret_cast<float*>(ys + nloc);
  float* fy = fx + nloc;
  float* fz = fy + nloc;
  const int64_t N = a.T.n_nodes, S = a.T.n_slots;

  const int G = gridDim.x;
  const int lb = xcd_block(blockIdx.x, G);
  const int64_t ntl = a.r.tile_end - a.r.tile_begin;
  const int t0 = a.r.tile_begin + (int)((int64_t)lb * ntl / G);
  const int t1 = a.r.tile_begin + (int)((int64_t)(lb + 1) * ntl / G);

  for (int t = t0 + wave; t < t1; t += W) {
    const TileDesc d = a.T.tiles[t];
    const int nc = a.T.n_cells;
    const double mu = a.T.params[d.cell];
    const double kappa = a.T.params[nc + d.cell];
    const double w = a.T.params[2 * nc + d.cell];
    const Material mat{w * mu, (1.0 - w) * mu, kappa};

    for (int i = lane; i < d.n_own; i += 64) {
      const int64_t g = d.own_begin + i;
      ys[i] = make_float4(a.y[g], a.y[N + g], a.y[2 * N + g], 0.f);
      fx[i] = 0.f; fy[i] = 0.f; fz[i] = 0.f;
    }
    for (int j = lane; j < d.n_shr; j += 64) {
      const int64_t g = a.T.slot_node[d.shr_begin + j];
      const int l = d.n_own + j;
      ys[l] = make_float4(a.y[g], a.y[N + g], a.y[2 * N + g], 0.f);
      fx[l] = 0.f; fy[l] = 0.f; fz[l] = 0.f;
    }
    wave_sync();

    double eacc = 0.0;
    int ninv = 0;
    const TetChunk* ch = a.T.chunks + d.chunk_begin;
    for (int base = 0; base < d.n_tets; base += 64, ++ch) {
      const uint2 q = *reinterpret_cast<const uint2*>(ch->idx[lane]);
      float B[9];
#pragma unroll
      for (int m = 0; m < 9; ++m) B[m] = ch->B[m][lane];
      const float V0 = ch->V0[lane];
      if (base + lane < d.n_tets) {
        const int i0 = q.x & 0xffff, i1 = q.x >> 16;
        const int i2 = q.y & 0xffff, i3 = q.y >> 16;
        const float4 p0 = ys[i0], p1 = ys[i1], p2 = ys[i2], p3 = ys[i3];
        const float e[3][3] = {{p0.x - p3.x, p0.y - p3.y, p0.z - p3.z},
                               {p1.x - p3.x, p1.y - p3.y, p1.z - p3.z},
                               {p2.x - p3.x, p2.y - p3.y, p2.z - p3.z}};
        float h[3][3];
        double vU;
        bool inv;
        tet_forward(e, B, V0, mat, h, vU, inv);
        lds_add(fx + i0, h[0][0]); lds_add(fy + i0, h[0][1]); lds_add(fz + i0, h[0][2]);
        lds_add(fx + i1, h[1][0]); lds_add(fy + i1, h[1][1]); lds_add(fz + i1, h[1][2]);
        lds_add(fx + i2, h[2][0]); lds_add(fy + i2, h[2][1]); lds_add(fz + i2, h[2][2]);
        lds_add(fx + i3, -(h[0][0] + h[1][0] + h[2][0]));
        lds_add(fy + i3, -(h[0][1] + h[1][1] + h[2][1]));
        lds_add(fz + i3, -(h[0][2] + h[1][2] + h[2][2]));
        eacc += vU;
        ninv += inv ? 1 : 0;
      }
    }
    wave_sync();

    for (int i = lane; i < d.n_own; i += 64) {
      const int64_t g = d.own_begin + i;
      a.f[g] = fx[i]; a.f[N + g] = fy[i]; a.f[2 * N + g] = fz[i];
    }
    for (int j = lane; j < d.n_shr; j += 64) {
      const int64_t s = d.shr_begin + j;
      const int l = d.n_own + j;
      a.T.part[s] = fx[l]; a.T.part[S + s] = fy[l]; a.T.part[2 * S + s] = fz[l];
    }
    eacc = wave_sum(eacc);
    ninv = wave_sum(ninv);
    if (lane == 0) {
      a.T.tile_acc[t] = eacc;
      a.T.tile_ninv[t] = ninv;
    }
    wave_sync();
  }
}

struct FinArgs {
  DeviceTables T;
  Range r;
  float* f;
  double* energy;
  int32_t* ninv;
};

// Sums the slot partials of every shared node in tile order, and the tile
// energies / inverted counts of every cell.
__global__ __launch_bounds__(256) void forward_finalize_kernel(FinArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = a.T.n_nodes, S = a.T.n_slots;
  if (gid < a.r.shared_end - a.r.shared_begin) {
    const int s = a.r.shared_begin + (int)gid;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    for (int q = a.T.shared_slot_ptr[s]; q < a.T.shared_slot_ptr[s + 1]; ++q) {
      const int64_t sl = a.T.shared_slots[q];
      sx += a.T.part[sl];
      sy += a.T.part[S + sl];
      sz += a.T.part[2 * S + sl];
    }
    const int64_t g = a.T.shared_node[s];
    a.f[g] = sx; a.f[N + g] = sy; a.f[2 * N + g] = sz;
  }
  if (gid < a.r.cell_end - a.r.cell_begin) {
    const int c = a.r.cell_begin + (int)gid;
    double e = 0.0;
    int ni = 0;
    for (int t = a.T.cell_tile_off[c]; t < a.T.cell_tile_off[c + 1]; ++t) {
      e += a.T.tile_acc[t];
      ni += a.T.tile_ninv[t];
    }
    if (a.energy) a.energy[c] = e;
    if (a.ninv) a.ninv[c] = ni;
  }
}

int grid_for(const Range& r, const LaunchCfg& cfg) {
  const int64_t ntl = r.tile_end - r.tile_begin;
  const int64_t groups = (ntl + cfg.waves - 1) / cfg.waves;
  int64_t g = cfg.blocks > 0 ? std::min<int64_t>(cfg.blocks, groups) : groups;
  return (int)std::max<int64_t>(g, 1);
}

template <int W>
hipError_t fwd_w(const FwdArgs& a, int grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(forward_kernel<W>, dim3(grid), dim3(64 * W), lds, st, a);
  return hipGetLastError();
}

}  // namespace

size_t forward_lds_per_wave(int nloc) { return (size_t)28 * nloc; }

hipError_t launch_forward(const DeviceTables& T, const Range& r,
                          const LaunchCfg& cfg, const float* y, float* f,
                          double* energy, int32_t* ninv, hipStream_t st) {
  if (r.tile_end > r.tile_begin) {
    FwdArgs a{T, r, y, f};
    const int grid = grid_for(r, cfg);
    const size_t lds = forward_lds_per_wave(T.nloc) * cfg.waves;
    hipError_t e;
    switch (cfg.waves) {
      case 1: e = fwd_w<1>(a, grid, lds, st); break;
      case 2: e = fwd_w<2>(a, grid, lds, st); break;
      case 4: e = fwd_w<4>(a, grid, lds, st); break;
      case 8: e = fwd_w<8>(a, grid, lds, st); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  const int64_t work = std::max<int64_t>(r.shared_end - r.shared_begin,
                                         r.cell_end - r.cell_begin);
  if (work > 0) {
    FinArgs b{T, r, f, energy, ninv};
    hipLaunchKernelGGL(forward_finalize_kernel, dim3((unsigned)((work + 255) / 256)),
                       dim3(256), 0, st, b);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace cm
