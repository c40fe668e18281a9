// Forward (forces + energy) kernels for gfx950.
//
// One wavefront per tile.  A tile's nodes are staged in LDS (positions and
// force accumulators, one float4 each); each lane evaluates one tetrahedron
// per 64-tetrahedron chunk.  The chunks are packed so that, for each vertex
// slot, the 64 lanes name 64 different nodes, so the wave adds its
// contributions slot by slot with plain LDS read-modify-writes (no atomics).
// The order of all additions is fixed by the layout: results are bitwise
// repeatable.  Owned nodes are then written straight to the output; shared
// nodes write a per-slot partial that the finalize kernel sums in tile order.
// With a plate step fused in (plate.h), the same passes write the positions
// after one compression step instead of the forces.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "finalize.h"
#include "kernels.h"
#include "mr_tet.h"
#include "plate.h"

namespace cm {
namespace {

struct FwdArgs {
  DeviceTables T;
  Range r;
  const float* y;
  float* f;
  PlateFwd pl;  // used when PL
  int check;    // count tets with a non-finite energy or force
};

template <int W, bool PL>
__global__ __launch_bounds__(64 * W) void forward_kernel(FwdArgs a) {
  extern __shared__ float4 lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nloc = a.T.nloc;
  // positions as a float4 array (16-byte records spread random-index reads
  // over all banks), force accumulators as packed float3 (12 bytes): 28
  // bytes per tile node; the wave's stride of 7 nloc / 4 float4 is exact
  // because nloc is a multiple of 4
  float4* ys = lds + (size_t)wave * (7 * nloc / 4);
  float* fs = reinterpret_cast<float*>(ys + nloc);
  const int64_t N = a.T.n_nodes;

  int t0, t1;
  block_tiles(a.r, t0, t1);
  for (int t = t0 + wave; t < t1; t += W) {
    const TileDesc d = a.T.tiles[t];
    const int mt = a.T.tile_mat[t], nm = a.T.n_mat;
    const double mu = a.T.params[mt];
    const double kappa = a.T.params[nm + mt];
    const double w = a.T.params[2 * nm + mt];
    const Material mat{w * mu, (1.0 - w) * mu, kappa};
    // plate step: the plates are read here, long before the epilogue needs
    // them; the 4th LDS component flags the nodes whose top-plate force this
    // tile adds (its owned nodes and the shared nodes of their first slot)
    float top = 0.f, bot = 0.f;
    if constexpr (PL) {
      top = (float)a.pl.plate[2 * d.cell];
      bot = (float)a.pl.plate[2 * d.cell + 1];
    }

    // the first chunk's loads go out before the node gather
    TetRegs first{};
    if (d.n_chunks > 0) load_tet(a.T.chunks + d.chunk_begin, lane, first);
    for (int l = lane; l < d.n_own + d.n_shr; l += 64) {
      int64_t g;
      float flag = 0.f;
      if constexpr (PL) {
        // one int32 load per shared node as in the plain pass, from the copy
        // of slot_node that carries the first-slot flag in bit 31
        const int32_t v = l < d.n_own ? INT32_MIN | (d.own_begin + l)
                                      : a.T.slot_node_first[d.shr_begin + l - d.n_own];
        g = v & 0x7fffffff;
        flag = v < 0 ? 1.f : 0.f;
      } else {
        g = l < d.n_own ? (int64_t)d.own_begin + l
                        : (int64_t)a.T.slot_node[d.shr_begin + l - d.n_own];
      }
      ys[l] = make_float4(a.y[g], a.y[N + g], a.y[2 * N + g], flag);
      fs[3 * l] = 0.f; fs[3 * l + 1] = 0.f; fs[3 * l + 2] = 0.f;
    }
    wave_sync();

    double eacc = 0.0;
    int ninv = 0, nonfin = 0;
    for_each_chunk_from(a.T.chunks + d.chunk_begin, d.n_chunks, lane, first,
                   [&](const TetRegs& cur) {
      const uint2 q = cur.q;
      if (q.x != kEmptyLane) {
        const int i0 = q.x & 0xffff, i1 = q.x >> 16;
        const int i2 = q.y & 0xffff, i3 = q.y >> 16;
        const float4 p0 = ys[i0], p1 = ys[i1], p2 = ys[i2], p3 = ys[i3];
        float h[3][3];
        double vU;
        bool inv;
        tet_forward(p0, p1, p2, p3, cur.B, cur.V0, mat, h, vU, inv);
        lds_accumulate([&](int i) { return &fs[3 * i]; }, i0, i1, i2, i3, h);
        eacc += vU;
        ninv += inv ? 1 : 0;
        if (a.check) {
          // a NaN or infinity in any component makes the sum non-finite
          float hs = 0.f;
#pragma unroll
          for (int k = 0; k < 3; ++k) hs += h[k][0] + h[k][1] + h[k][2];
          nonfin += (isfinite(vU) && isfinite(hs)) ? 0 : 1;
        }
      }
    });
    wave_sync();

    if constexpr (PL) {
      // the step of the owned nodes, and the tile's share of the top-plate
      // force (the flagged nodes)
      double fp = 0.0;
      for (int i = lane; i < d.n_own; i += 64) {
        const float4 p = ys[i];
        const float3 v = make_float3(fs[3 * i], fs[3 * i + 1], fs[3 * i + 2]);
        plate_node_step(p.x, p.y, p.z, v.x, v.y, v.z, top, bot, a.pl.k, a.pl.m,
                        a.pl.y_next, N, (int64_t)d.own_begin + i);
        fp += plate_top_term(p.z, top, a.pl.k);
      }
      for (int j = lane; j < d.n_shr; j += 64) {
        const float4 p = ys[d.n_own + j];
        if (p.w != 0.f) fp += plate_top_term(p.z, top, a.pl.k);
      }
      fp = wave_sum(fp);
      if (lane == 0) a.T.tile_plate[t] = fp;
    } else {
      for (int i = lane; i < d.n_own; i += 64) {
        const int64_t g = d.own_begin + i;
        const float3 v = make_float3(fs[3 * i], fs[3 * i + 1], fs[3 * i + 2]);
        a.f[g] = v.x; a.f[N + g] = v.y; a.f[2 * N + g] = v.z;
      }
    }
    for (int j = lane; j < d.n_shr; j += 64) {
      const int64_t s = d.shr_begin + j;
      const int l3 = 3 * (d.n_own + j);
      const float3 v = make_float3(fs[l3], fs[l3 + 1], fs[l3 + 2]);
      float* pp = a.T.part + 3 * s;
      pp[0] = v.x; pp[1] = v.y; pp[2] = v.z;
    }
    eacc = wave_sum(eacc);
    ninv = wave_sum(ninv);
    if (a.check) nonfin = wave_sum(nonfin);
    if (lane == 0) {
      a.T.tile_acc[t] = eacc;
      a.T.tile_ninv[t] = ninv;
      if (a.check) a.T.tile_nonfin[t] = nonfin;
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
  const float* y;  // with a plate step
  PlateFwd pl;
  int32_t* nonfin;  // per cell, nullable (needs a checked tile pass)
};

// The first cell_blocks workgroups sum the tile energies / inverted counts
// of every cell, one wavefront per cell (lane l takes tiles l, l + 64, ...,
// then a fixed butterfly: deterministic, and the cells' long chains of
// loads run in parallel); the others sum the slot partials of every shared
// node in tile order (with a plate step, the shared nodes are stepped
// instead of stored).
__global__ __launch_bounds__(256) void forward_finalize_kernel(FinArgs a,
                                                               int cell_blocks) {
  if ((int)blockIdx.x < cell_blocks) {
    const int wv = ((int)blockIdx.x * 256 + (int)threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wv >= a.r.cell_end - a.r.cell_begin) return;  // uniform per wave
    const int c = a.r.cell_begin + wv;
    const CellSums cs = cell_sums(a.T, c, lane, a.nonfin != nullptr);
    if (lane == 0) {
      if (a.energy) a.energy[c] = cs.e;
      if (a.ninv) a.ninv[c] = cs.ni;
      if (a.nonfin) a.nonfin[c] = cs.nf;
    }
    if (a.pl.force) {
      const int t0 = a.T.cell_tile_first[c], nt = a.T.cell_tile_count[c];
      // top-plate force: the tile shares, then the nodes of no tetrahedron
      double fp = 0.0;
      for (int k = lane; k < nt; k += 64)
        fp += a.T.tile_plate[t0 + (int64_t)k * a.T.tile_stride];
      const float top = (float)a.pl.plate[2 * c];
      for (int o = a.T.orphan_off[c] + lane; o < a.T.orphan_off[c + 1]; o += 64)
        fp += plate_top_term(a.y[2 * a.T.n_nodes + a.T.orphan_node[o]], top, a.pl.k);
      fp = wave_sum(fp);
      if (lane == 0) a.pl.force[c] = fp;
    }
    return;
  }
  const int64_t N = a.T.n_nodes;
  const int64_t gid = (int64_t)(blockIdx.x - cell_blocks) * blockDim.x + threadIdx.x;
  if (gid < a.r.shared_end - a.r.shared_begin) {
    const int s = a.r.shared_begin + (int)gid;
    const int64_t g = a.T.shared_node[s];
    // plate step: the node's position and plates are loaded before the
    // partial sums, so that the two chains of loads overlap
    float px = 0.f, py = 0.f, pz = 0.f, top = 0.f, bot = 0.f;
    if (a.pl.plate) {
      const int c = a.T.shared_cell[s];
      px = a.y[g];
      py = a.y[N + g];
      pz = a.y[2 * N + g];
      top = (float)a.pl.plate[2 * c];
      bot = (float)a.pl.plate[2 * c + 1];
    }
    const float3 sm = shared_sum(a.T, a.T.part, s);
    if (a.pl.plate) {
      plate_node_step(px, py, pz, sm.x, sm.y, sm.z, top, bot, a.pl.k, a.pl.m, a.pl.y_next,
                      N, g);
    } else {
      a.f[g] = sm.x; a.f[N + g] = sm.y; a.f[2 * N + g] = sm.z;
    }
  }
}

template <int W>
hipError_t fwd_w(const FwdArgs& a, int grid, size_t lds, hipStream_t st) {
  if (a.pl.plate)
    hipLaunchKernelGGL((forward_kernel<W, true>), dim3(grid), dim3(64 * W), lds, st, a);
  else
    hipLaunchKernelGGL((forward_kernel<W, false>), dim3(grid), dim3(64 * W), lds, st, a);
  return hipGetLastError();
}

}  // namespace

size_t forward_lds_per_wave(int nloc) { return (size_t)28 * nloc; }

hipError_t launch_forward_main(const DeviceTables& T, const Range& r,
                               const LaunchCfg& cfg, const float* y, float* f,
                               hipStream_t st, const PlateFwd& pl, bool check) {
  if (r.tile_end <= r.tile_begin) return hipSuccess;
  if (check && !T.tile_nonfin) return hipErrorInvalidValue;
  // the per-wave LDS stride (7 nloc / 4 float4) needs nloc % 4 == 0
  if (T.nloc <= 0 || T.nloc % 4 != 0) return hipErrorInvalidValue;
  FwdArgs a{T, r, y, f, pl, check ? 1 : 0};
  const int grid = grid_for(r, cfg);
  const size_t lds = forward_lds_per_wave(T.nloc) * cfg.waves;
  switch (cfg.waves) {
    case 1: return fwd_w<1>(a, grid, lds, st);
    case 2: return fwd_w<2>(a, grid, lds, st);
    case 4: return fwd_w<4>(a, grid, lds, st);
    case 8: return fwd_w<8>(a, grid, lds, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_forward_finalize(const DeviceTables& T, const Range& r,
                                   float* f, double* energy, int32_t* ninv,
                                   hipStream_t st, const float* y,
                                   const PlateFwd& pl, int32_t* nonfin) {
  const int64_t n_shr = r.shared_end - r.shared_begin;
  const int64_t n_cells = r.cell_end - r.cell_begin;
  if (n_shr <= 0 && n_cells <= 0) return hipSuccess;
  const int cell_blocks = (int)((n_cells + 3) / 4);  // four waves per block
  const int64_t blocks = cell_blocks + (n_shr + 255) / 256;
  FinArgs b{T, r, f, energy, ninv, y, pl, nonfin};
  hipLaunchKernelGGL(forward_finalize_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     st, b, cell_blocks);
  return hipGetLastError();
}

hipError_t launch_forward(const DeviceTables& T, const Range& r,
                          const LaunchCfg& cfg, const float* y, float* f,
                          double* energy, int32_t* ninv, hipStream_t st,
                          const PlateFwd& pl, int32_t* nonfin) {
  hipError_t e = launch_forward_main(T, r, cfg, y, f, st, pl, nonfin != nullptr);
  if (e != hipSuccess) return e;
  return launch_forward_finalize(T, r, f, energy, ninv, st, y, pl, nonfin);
}

}  // namespace cm
