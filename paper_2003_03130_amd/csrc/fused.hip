// Forward and backward in one tile pass, for a loss L(f, E) whose cotangents
// fbar = dL/df and ebar = dL/dE are known before the forces are (a loss
// linear in f and E, such as sum_i v_i . f_i, or a caller that holds them
// already).  The separate passes read every chunk and stage every tile node
// twice and form F, the invariants and cof F of every tetrahedron twice;
// here each lane evaluates its tetrahedron once -- the forward half, then the
// adjoint half from the same F, invariants and cof F -- and adds the forces
// and the ybar contributions to two LDS accumulators of the same tile nodes.
// Per-tet arithmetic, tile order and every summation order are those of the
// forward kernel and of the backward kernel, so f, E, the inverted counts,
// ybar and thetabar equal those of the two separate passes bit for bit.  Scratch: the forward's slot partials and tile records
// (T) and the backward's (part_b, tile_acc_b), finalized by one kernel that
// forms both passes' sums.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "finalize.h"
#include "kernels.h"
#include "mr_tet.h"

namespace cm {
namespace {

struct FusedArgs {
  DeviceTables T;       // forward scratch: part, tile_acc (energy), tile_ninv
  float* part_b;        // backward slot partials
  double* tile_acc_b;   // backward per-tile parameter-gradient sums
  Range r;
  const float* y;
  const float* fbar;    // nullable
  const double* ebar;   // nullable
  float* f;
  float* ybar;
};

template <int W, bool GRAD>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(3)))
void forward_backward_kernel(FusedArgs a) {
  extern __shared__ float4 lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nloc = a.T.nloc;
  // per wave (48 bytes per tile node): (y.x, y.y, y.z, fbar.x) as float4,
  // (fbar.y, fbar.z) as float2, force and ybar accumulators as packed
  // float3; the wave's stride of 3 nloc float4 is exact
  float4* ys = lds + (size_t)wave * (3 * nloc);
  float2* vs = reinterpret_cast<float2*>(ys + nloc);
  float* fs = reinterpret_cast<float*>(vs + nloc);
  float* gs = fs + 3 * nloc;
  const int64_t N = a.T.n_nodes;
  const bool has_fbar = a.fbar != nullptr;

  int t0, t1;
  block_tiles(a.r, t0, t1);
  for (int t = t0 + wave; t < t1; t += W) {
    const TileDesc d = a.T.tiles[t];
    const int mt = a.T.tile_mat[t], nm = a.T.n_mat;
    const double mu = a.T.params[mt];
    const double kappa = a.T.params[nm + mt];
    const double w = a.T.params[2 * nm + mt];
    const Material mat{w * mu, (1.0 - w) * mu, kappa};
    const double eb = (GRAD && a.ebar) ? a.ebar[d.cell] : 0.0;

    // the first chunk's loads go out before the node gather
    TetRegs first{};
    if (d.n_chunks > 0) load_tet(a.T.chunks + d.chunk_begin, lane, first);
    for (int l = lane; l < d.n_own + d.n_shr; l += 64) {
      const int64_t g = l < d.n_own ? (int64_t)d.own_begin + l
                                    : (int64_t)a.T.slot_node[d.shr_begin + l - d.n_own];
      const float vx = has_fbar ? a.fbar[g] : 0.f;
      ys[l] = make_float4(a.y[g], a.y[N + g], a.y[2 * N + g], vx);
      vs[l] = has_fbar ? make_float2(a.fbar[N + g], a.fbar[2 * N + g])
                       : make_float2(0.f, 0.f);
      fs[3 * l] = 0.f; fs[3 * l + 1] = 0.f; fs[3 * l + 2] = 0.f;
      gs[3 * l] = 0.f; gs[3 * l + 1] = 0.f; gs[3 * l + 2] = 0.f;
    }
    wave_sync();

    double eacc = 0.0;
    int ninv = 0;
    double acc[3] = {0.0, 0.0, 0.0}, acce[3] = {0.0, 0.0, 0.0};
    for_each_chunk_from(a.T.chunks + d.chunk_begin, d.n_chunks, lane, first,
                        [&](const TetRegs& cur) {
      const uint2 q = cur.q;
      if (q.x != kEmptyLane) {
        const int i0 = q.x & 0xffff, i1 = q.x >> 16;
        const int i2 = q.y & 0xffff, i3 = q.y >> 16;
        const float4 p0 = ys[i0], p1 = ys[i1], p2 = ys[i2], p3 = ys[i3];
        // forward half: F, the invariants, the forces and the energy,
        // as tet_forward
        double Fd[3][3], vU;
        float F[3][3], Cf[6], hf[3][3];
        deformation_gradient(p0, p1, p2, p3, cur.B, Fd, F);
        Scalars sc;
        invariants(Fd, Cf, sc);
        stress_forces(F, Cf, sc, cur.B, cur.V0, mat, hf, vU);
        lds_accumulate([&](int i) { return &fs[3 * i]; }, i0, i1, i2, i3, hf);
        eacc += vU;
        ninv += sc.J > 0.0 ? 0 : 1;
        // the forward half's temporaries are dead before the adjoint half
        // is formed: the kernel fits the 168 VGPRs of three waves per SIMD
        // (185 without the barrier: two waves)
        __builtin_amdgcn_sched_barrier(0);
        // adjoint half from the same F, invariants and cof F, as tet_backward
        const float2 w0 = vs[i0], w1 = vs[i1], w2 = vs[i2], w3 = vs[i3];
        const float4 v0 = make_float4(p0.w, w0.x, w0.y, 0.f);
        const float4 v1 = make_float4(p1.w, w1.x, w1.y, 0.f);
        const float4 v2 = make_float4(p2.w, w2.x, w2.y, 0.f);
        const float4 v3 = make_float4(p3.w, w3.x, w3.y, 0.f);
        float dF[3][3], K[3][3], h[3][3];
        double gp[3], ge[3];
        cofactor(F, K);
        direction_gradient(v0, v1, v2, v3, cur.B, dF);
        adjoint_terms<GRAD>(F, dF, Cf, K, sc, cur.B, cur.V0, mat, eb, h, gp, ge);
        lds_accumulate([&](int i) { return &gs[3 * i]; }, i0, i1, i2, i3, h);
        if constexpr (GRAD) {
          const double vol = (double)cur.V0;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            acc[c] = fma(vol, gp[c], acc[c]);
            acce[c] = fma(vol, ge[c], acce[c]);
          }
        }
      }
    });
    wave_sync();

    for (int i = lane; i < d.n_own; i += 64) {
      const int64_t g = d.own_begin + i;
      a.f[g] = fs[3 * i]; a.f[N + g] = fs[3 * i + 1]; a.f[2 * N + g] = fs[3 * i + 2];
      a.ybar[g] = gs[3 * i]; a.ybar[N + g] = gs[3 * i + 1]; a.ybar[2 * N + g] = gs[3 * i + 2];
    }
    for (int j = lane; j < d.n_shr; j += 64) {
      const int64_t s = d.shr_begin + j;
      const int l = d.n_own + j;
      float* pf = a.T.part + 3 * s;
      pf[0] = fs[3 * l]; pf[1] = fs[3 * l + 1]; pf[2] = fs[3 * l + 2];
      float* pb = a.part_b + 3 * s;
      pb[0] = gs[3 * l]; pb[1] = gs[3 * l + 1]; pb[2] = gs[3 * l + 2];
    }
    eacc = wave_sum(eacc);
    ninv = wave_sum(ninv);
    if constexpr (GRAD) {
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] = wave_sum(fma(0.5 * eb, acce[c], -acc[c]));
    }
    if (lane == 0) {
      a.T.tile_acc[t] = eacc;
      a.T.tile_ninv[t] = ninv;
      if constexpr (GRAD) {
        a.tile_acc_b[3 * (int64_t)t] = acc[0];
        a.tile_acc_b[3 * (int64_t)t + 1] = acc[1];
        a.tile_acc_b[3 * (int64_t)t + 2] = acc[2];
      }
    }
    wave_sync();
  }
}

struct FusedFinArgs {
  DeviceTables T;             // forward tables: part holds the force partials
  const float* part_b;        // ybar partials
  const double* tile_acc_b;   // per-tile parameter-gradient sums
  Range r;
  float* f;
  double* energy;             // nullable
  int32_t* ninv;              // nullable
  float* ybar;
  double* thetabar;           // nullable (then slot_blocks = 0)
};

// One launch for both passes' finalize work: the first cell_blocks
// workgroups form each cell's energy and inverted count (one wavefront per
// cell), the next slot_blocks each material slot's parameter gradient (one
// wavefront per slot); the others sum the force and the ybar partials of
// every shared node in tile order from one read of its slot list.  Every
// sum is the one the forward and the backward finalize kernels form.
__global__ __launch_bounds__(256) void forward_backward_finalize_kernel(
    FusedFinArgs a, int cell_blocks, int slot_blocks) {
  const int b = blockIdx.x;
  if (b < cell_blocks + slot_blocks) {
    const int lane = threadIdx.x & 63;
    if (b < cell_blocks) {
      const int wv = (b * 256 + (int)threadIdx.x) >> 6;
      if (wv >= a.r.cell_end - a.r.cell_begin) return;  // uniform per wave
      const int c = a.r.cell_begin + wv;
      const CellSums cs = cell_sums(a.T, c, lane, false);
      if (lane == 0) {
        if (a.energy) a.energy[c] = cs.e;
        if (a.ninv) a.ninv[c] = cs.ni;
      }
    } else {
      const int R = a.T.n_regions;
      const int wv = ((b - cell_blocks) * 256 + (int)threadIdx.x) >> 6;
      if (wv >= (a.r.cell_end - a.r.cell_begin) * R) return;  // uniform per wave
      const int mt = a.r.cell_begin * R + wv;  // material slot
      double t3[3];
      slot_theta(a.T, a.tile_acc_b, mt, lane, t3);
      if (lane == 0) {
        a.thetabar[3 * (int64_t)mt] = t3[0];
        a.thetabar[3 * (int64_t)mt + 1] = t3[1];
        a.thetabar[3 * (int64_t)mt + 2] = t3[2];
      }
    }
    return;
  }
  const int64_t gid =
      (int64_t)(b - cell_blocks - slot_blocks) * blockDim.x + threadIdx.x;
  if (gid >= a.r.shared_end - a.r.shared_begin) return;
  const int s = a.r.shared_begin + (int)gid;
  const int64_t g = a.T.shared_node[s];
  const int64_t N = a.T.n_nodes;
  float fx = 0.f, fy = 0.f, fz = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
  for (int q = a.T.shared_slot_ptr[s]; q < a.T.shared_slot_ptr[s + 1]; ++q) {
    const int64_t sl = a.T.shared_slots[q];
    const float* pf = a.T.part + 3 * sl;
    const float* pb = a.part_b + 3 * sl;
    fx += pf[0];
    fy += pf[1];
    fz += pf[2];
    bx += pb[0];
    by += pb[1];
    bz += pb[2];
  }
  a.f[g] = fx; a.f[N + g] = fy; a.f[2 * N + g] = fz;
  a.ybar[g] = bx; a.ybar[N + g] = by; a.ybar[2 * N + g] = bz;
}

template <int W>
hipError_t fb_w(const FusedArgs& a, int grid, size_t lds, hipStream_t st, bool grad) {
  if (grad)
    hipLaunchKernelGGL((forward_backward_kernel<W, true>), dim3(grid), dim3(64 * W), lds,
                       st, a);
  else
    hipLaunchKernelGGL((forward_backward_kernel<W, false>), dim3(grid), dim3(64 * W), lds,
                       st, a);
  return hipGetLastError();
}

}  // namespace

size_t forward_backward_lds_per_wave(int nloc) { return (size_t)48 * nloc; }

hipError_t launch_forward_backward_main(const DeviceTables& T, const DeviceTables& Tb,
                                        const Range& r, const LaunchCfg& cfg,
                                        const float* y, float* f, const float* fbar,
                                        const double* ebar, float* ybar, hipStream_t st,
                                        bool grad) {
  if (r.tile_end <= r.tile_begin) return hipSuccess;
  // every layout rounds nloc up to a multiple of 4 (the separate passes'
  // LDS strides need it; this pass's 48-byte stride keeps its float4
  // records aligned for any nloc)
  if (T.nloc <= 0 || T.nloc % 4 != 0) return hipErrorInvalidValue;
  FusedArgs a{T, Tb.part, Tb.tile_acc, r, y, fbar, ebar, f, ybar};
  const int grid = grid_for(r, cfg);
  const size_t lds = forward_backward_lds_per_wave(T.nloc) * cfg.waves;
  switch (cfg.waves) {
    case 1: return fb_w<1>(a, grid, lds, st, grad);
    case 2: return fb_w<2>(a, grid, lds, st, grad);
    case 4: return fb_w<4>(a, grid, lds, st, grad);
    case 8: return fb_w<8>(a, grid, lds, st, grad);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_forward_backward(const DeviceTables& T, const DeviceTables& Tb,
                                   const Range& r, const LaunchCfg& cfg, const float* y,
                                   float* f, double* energy, int32_t* ninv,
                                   const float* fbar, const double* ebar, float* ybar,
                                   double* thetabar, hipStream_t st) {
  // as in the backward pass: without an energy cotangent or a parameter
  // gradient the adjoint half is the Hessian-vector product alone
  const bool grad = ebar != nullptr || thetabar != nullptr;
  hipError_t e =
      launch_forward_backward_main(T, Tb, r, cfg, y, f, fbar, ebar, ybar, st, grad);
  if (e != hipSuccess) return e;
  return launch_forward_backward_finalize(T, Tb, r, f, energy, ninv, ybar, thetabar, st);
}

hipError_t launch_forward_backward_finalize(const DeviceTables& T, const DeviceTables& Tb,
                                            const Range& r, float* f, double* energy,
                                            int32_t* ninv, float* ybar, double* thetabar,
                                            hipStream_t st) {
  const int64_t n_shr = r.shared_end - r.shared_begin;
  const int64_t n_cells = r.cell_end - r.cell_begin;
  const int64_t n_slots = thetabar ? n_cells * T.n_regions : 0;
  if (n_shr <= 0 && n_cells <= 0) return hipSuccess;
  const int cell_blocks = (int)((n_cells + 3) / 4);  // four waves per block
  const int slot_blocks = (int)((n_slots + 3) / 4);
  const int64_t blocks = cell_blocks + slot_blocks + (n_shr + 255) / 256;
  FusedFinArgs b{T, Tb.part, Tb.tile_acc, r, f, energy, ninv, ybar, thetabar};
  hipLaunchKernelGGL(forward_backward_finalize_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     st, b, cell_blocks, slot_blocks);
  return hipGetLastError();
}

}  // namespace cm
