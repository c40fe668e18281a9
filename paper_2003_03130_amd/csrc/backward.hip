// Backward (adjoint) kernels for gfx950: for a loss L(f, E) with cotangents
// fbar = dL/df (per node) and ebar = dL/dE (per cell),
//   ybar     = (df/dy)^T fbar - ebar f  (a Hessian-vector product of E),
//   thetabar = dL/d(mu, kappa, w) per material slot (cell and region).
// Same tiling as the forward kernel: one wavefront per tile; position, fbar
// and ybar accumulator of each tile node form one LDS record; ybar is
// accumulated in LDS slot by slot without atomics (see layout.h), owned
// nodes are stored directly and shared nodes go through the slot partials
// and the finalize kernel, in a fixed order (deterministic).  With the
// reverse plate step fused in (plate.h), the same passes write the adjoint
// state of the previous step instead of ybar.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "finalize.h"
#include "kernels.h"
#include "mr_tet.h"
#include "plate.h"

namespace cm {
namespace {

struct BwdArgs {
  DeviceTables T;
  Range r;
  const float* y;
  const float* fbar;    // nullable
  const double* ebar;   // nullable
  float* ybar;
  CellMask mask;
  PlateBwd pl;  // used when PL
};

// GRAD = false: the Hessian-vector product alone (no energy cotangent, no
// parameter gradient; tile_acc is not written).
template <int W, bool PL, bool GRAD>
__global__ __launch_bounds__(64 * W) void backward_kernel(BwdArgs a) {
  extern __shared__ float4 lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nloc = a.T.nloc;
  // per wave (40 bytes per tile node): (y.x, y.y, y.z, fbar.x) as float4,
  // ybar accumulators as float4, (fbar.y, fbar.z) as float2; the wave's
  // stride of 10 nloc / 4 float4 covers the float2 array exactly because
  // nloc is a multiple of 4 (checked at launch)
  float4* ys = lds + (size_t)wave * (10 * nloc / 4);
  float4* gs = ys + nloc;
  float2* vs = reinterpret_cast<float2*>(gs + nloc);
  const int64_t N = a.T.n_nodes;
  const bool has_fbar = a.fbar != nullptr;

  int t0, t1;
  block_tiles(a.r, t0, t1);
  for (int t = t0 + wave; t < t1; t += W) {
    const TileDesc d = a.T.tiles[t];
    if (a.mask.flags && a.mask.flags[(int64_t)d.cell * a.mask.stride] == 0.0)
      continue;  // cell not selected (uniform over the wave)
    const int mt = a.T.tile_mat[t], nm = a.T.n_mat;
    const double mu = a.T.params[mt];
    const double kappa = a.T.params[nm + mt];
    const double w = a.T.params[2 * nm + mt];
    const Material mat{w * mu, (1.0 - w) * mu, kappa};
    const double eb = (GRAD && a.ebar) ? a.ebar[d.cell] : 0.0;
    // plate step: per-cell values read here, long before the epilogue
    float top = 0.f, bot = 0.f, gw = 0.f;
    if constexpr (PL) {
      top = (float)a.pl.plate[2 * d.cell];
      bot = (float)a.pl.plate[2 * d.cell + 1];
      gw = plate_loss_weight(a.pl.F_meas, a.pl.F_target, a.pl.scale, d.cell);
    }

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
      gs[l] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    wave_sync();

    // per lane: sum V0 gp and sum V0 ge (the tile's parameter gradient is
    // -sum V0 gp + ebar/2 sum V0 ge)
    double acc[3] = {0.0, 0.0, 0.0}, acce[3] = {0.0, 0.0, 0.0};
    for_each_chunk_from(a.T.chunks + d.chunk_begin, d.n_chunks, lane, first,
                   [&](const TetRegs& cur) {
      const uint2 q = cur.q;
      if (q.x != kEmptyLane) {
        const int i0 = q.x & 0xffff, i1 = q.x >> 16;
        const int i2 = q.y & 0xffff, i3 = q.y >> 16;
        const float4 p0 = ys[i0], p1 = ys[i1], p2 = ys[i2], p3 = ys[i3];
        const float2 w0 = vs[i0], w1 = vs[i1], w2 = vs[i2], w3 = vs[i3];
        const float4 v0 = make_float4(p0.w, w0.x, w0.y, 0.f);
        const float4 v1 = make_float4(p1.w, w1.x, w1.y, 0.f);
        const float4 v2 = make_float4(p2.w, w2.x, w2.y, 0.f);
        const float4 v3 = make_float4(p3.w, w3.x, w3.y, 0.f);
        float h[3][3];
        double gp[3], ge[3];
        tet_backward<GRAD>(p0, p1, p2, p3, v0, v1, v2, v3, cur.B, cur.V0, mat, eb,
                           h, gp, ge);
        lds_accumulate([&](int i) { return &gs[i].x; }, i0, i1, i2, i3, h);
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

    if constexpr (PL) {
      for (int i = lane; i < d.n_own; i += 64) {
        const float4 p = ys[i], v = gs[i];
        const float2 l = vs[i];
        plate_node_adjoint(p.z, p.w, l.x, l.y, v.x, v.y, v.z, top, bot, a.pl.k,
                           a.pl.m, gw, a.pl.lam, N, (int64_t)d.own_begin + i);
      }
    } else {
      for (int i = lane; i < d.n_own; i += 64) {
        const int64_t g = d.own_begin + i;
        const float4 v = gs[i];
        a.ybar[g] = v.x; a.ybar[N + g] = v.y; a.ybar[2 * N + g] = v.z;
      }
    }
    for (int j = lane; j < d.n_shr; j += 64) {
      const int64_t s = d.shr_begin + j;
      const float4 v = gs[d.n_own + j];
      float* pp = a.T.part + 3 * s;
      pp[0] = v.x; pp[1] = v.y; pp[2] = v.z;
    }
    if constexpr (GRAD) {
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] = wave_sum(fma(0.5 * eb, acce[c], -acc[c]));
      if (lane == 0) {
        a.T.tile_acc[3 * (int64_t)t] = acc[0];
        a.T.tile_acc[3 * (int64_t)t + 1] = acc[1];
        a.T.tile_acc[3 * (int64_t)t + 2] = acc[2];
      }
    }
    wave_sync();
  }
}

struct BwdFinArgs {
  DeviceTables T;
  Range r;
  float* ybar;
  double* thetabar;  // nullable
  CellMask mask;
  const float* y;        // with a plate step
  const float* lam_next;
  PlateBwd pl;
};

// The first slot_blocks workgroups form, one wavefront per material slot,
//   dL/dmu = w g_I + (1 - w) g_K, dL/dkappa = g_J, dL/dw = mu (g_I - g_K)
// from the per-tile sums of dL/d(mu1, mu2, kappa) (mu1 = w mu, mu2 = (1-w) mu;
// lane l takes tiles l, l + 64, ..., then a fixed butterfly); the others sum
// the slot partials of every shared node in tile order.  With a plate
// step, m thetabar is added to pl.thetabar_acc instead of storing thetabar,
// and the shared nodes take the reverse step instead of storing ybar.
__global__ __launch_bounds__(256) void backward_finalize_kernel(BwdFinArgs a,
                                                                int slot_blocks) {
  const CellMask& m = a.mask;
  const int R = a.T.n_regions;
  if ((int)blockIdx.x < slot_blocks) {
    const int wv = ((int)blockIdx.x * 256 + (int)threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    double* const tb = a.pl.plate ? a.pl.thetabar_acc : a.thetabar;
    if (!tb || wv >= (a.r.cell_end - a.r.cell_begin) * R) return;
    const int mt = a.r.cell_begin * R + wv;  // material slot
    if (m.flags && m.flags[(int64_t)(mt / R) * m.stride] == 0.0) return;
    double t3[3];
    slot_theta(a.T, a.T.tile_acc, mt, lane, t3);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (a.pl.plate)
          tb[3 * (int64_t)mt + q] += a.pl.m64 * t3[q];
        else
          tb[3 * (int64_t)mt + q] = t3[q];
      }
    }
    return;
  }
  const int64_t gid = (int64_t)(blockIdx.x - slot_blocks) * blockDim.x + threadIdx.x;
  const int64_t N = a.T.n_nodes;
  if (gid < a.r.shared_end - a.r.shared_begin) {
    const int s = a.r.shared_begin + (int)gid;
    const int64_t g = a.T.shared_node[s];
    if (!m.flags || m.flags[(int64_t)a.T.shared_cell[s] * m.stride] != 0.0) {
      // plate step: the node's values are loaded before the partial sums,
      // so that the two chains of loads overlap
      float pz = 0.f, lx = 0.f, ly = 0.f, lz = 0.f, top = 0.f, bot = 0.f, gw = 0.f;
      if (a.pl.plate) {
        const int c = a.T.shared_cell[s];
        pz = a.y[2 * N + g];
        lx = a.lam_next[g];
        ly = a.lam_next[N + g];
        lz = a.lam_next[2 * N + g];
        top = (float)a.pl.plate[2 * c];
        bot = (float)a.pl.plate[2 * c + 1];
        gw = plate_loss_weight(a.pl.F_meas, a.pl.F_target, a.pl.scale, c);
      }
      const float3 sm = shared_sum(a.T, a.T.part, s);
      if (a.pl.plate) {
        plate_node_adjoint(pz, lx, ly, lz, sm.x, sm.y, sm.z, top, bot, a.pl.k, a.pl.m, gw,
                           a.pl.lam, N, g);
      } else {
        a.ybar[g] = sm.x; a.ybar[N + g] = sm.y; a.ybar[2 * N + g] = sm.z;
      }
    }
  }
}

template <int W, bool GRAD>
hipError_t bwd_wg(const BwdArgs& a, int grid, size_t lds, hipStream_t st) {
  if (a.pl.plate)
    hipLaunchKernelGGL((backward_kernel<W, true, GRAD>), dim3(grid), dim3(64 * W), lds, st,
                       a);
  else
    hipLaunchKernelGGL((backward_kernel<W, false, GRAD>), dim3(grid), dim3(64 * W), lds,
                       st, a);
  return hipGetLastError();
}

template <int W>
hipError_t bwd_w(const BwdArgs& a, int grid, size_t lds, hipStream_t st, bool grad) {
  return grad ? bwd_wg<W, true>(a, grid, lds, st) : bwd_wg<W, false>(a, grid, lds, st);
}

}  // namespace

size_t backward_lds_per_wave(int nloc) { return (size_t)40 * nloc; }

hipError_t launch_backward_main(const DeviceTables& T, const Range& r,
                                const LaunchCfg& cfg, const float* y,
                                const float* fbar, const double* ebar,
                                float* ybar, hipStream_t st, const CellMask& mask,
                                const PlateBwd& pl, bool grad) {
  if (r.tile_end <= r.tile_begin) return hipSuccess;
  // the per-wave LDS stride (10 nloc / 4 float4) needs nloc % 4 == 0, else
  // a wave's last float2 would overlap the next wave's records
  if (T.nloc <= 0 || T.nloc % 4 != 0) return hipErrorInvalidValue;
  BwdArgs a{T, r, y, fbar, ebar, ybar, mask, pl};
  const int grid = grid_for(r, cfg);
  const size_t lds = backward_lds_per_wave(T.nloc) * cfg.waves;
  switch (cfg.waves) {
    case 1: return bwd_w<1>(a, grid, lds, st, grad);
    case 2: return bwd_w<2>(a, grid, lds, st, grad);
    case 4: return bwd_w<4>(a, grid, lds, st, grad);
    case 8: return bwd_w<8>(a, grid, lds, st, grad);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_backward_finalize(const DeviceTables& T, const Range& r,
                                    float* ybar, double* thetabar,
                                    hipStream_t st, const CellMask& mask,
                                    const float* y, const float* lam_next,
                                    const PlateBwd& pl) {
  const int64_t n_shr = r.shared_end - r.shared_begin;
  const bool has_tb = pl.plate ? pl.thetabar_acc != nullptr : thetabar != nullptr;
  const int64_t n_slots = has_tb ? (int64_t)(r.cell_end - r.cell_begin) * T.n_regions : 0;
  if (n_shr <= 0 && n_slots <= 0) return hipSuccess;
  const int slot_blocks = (int)((n_slots + 3) / 4);  // four waves per block
  const int64_t blocks = slot_blocks + (n_shr + 255) / 256;
  BwdFinArgs b{T, r, ybar, thetabar, mask, y, lam_next, pl};
  hipLaunchKernelGGL(backward_finalize_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     st, b, slot_blocks);
  return hipGetLastError();
}

hipError_t launch_backward(const DeviceTables& T, const Range& r,
                           const LaunchCfg& cfg, const float* y,
                           const float* fbar, const double* ebar, float* ybar,
                           double* thetabar, hipStream_t st, const CellMask& mask,
                           const PlateBwd& pl) {
  // the parameter gradient and the energy cotangent need the full adjoint;
  // without them the pass is the Hessian-vector product alone
  const bool grad = ebar != nullptr || (pl.plate ? pl.thetabar_acc != nullptr
                                                 : thetabar != nullptr);
  hipError_t e = launch_backward_main(T, r, cfg, y, fbar, ebar, ybar, st, mask, pl, grad);
  if (e != hipSuccess) return e;
  return launch_backward_finalize(T, r, ybar, thetabar, st, mask, y, fbar, pl);
}

}  // namespace cm
