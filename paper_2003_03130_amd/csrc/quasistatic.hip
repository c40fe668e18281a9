// Quasi-static plate compression for gfx950: Newton steps on the total
// potential Pi(y) = E(y) + sum_nodes phi(y_z), with the plate penalty
// phi(z) = (k/3) [max(0, z - top)^3 + max(0, bottom - z)^3] (its force is the
// penalty of the plate-compression steps), each Newton system
// Hess(Pi) dx = f + p solved by conjugate gradients per cell, preconditioned
// by the inverse 3x3 node blocks of the small-strain stiffness plus the
// penalty Hessian (block Jacobi).  Hessian-vector products of E come from the
// backward kernels (ybar = (df/dy)^T v = -Hess(E) v); the penalty Hessian is
// diagonal, 2k (max(0, z - top) + max(0, bottom - z)) on the z entries.
//
// One workgroup per cell (cells are independent systems); per-cell scalars
// live in a float64 state of kQsState entries per cell, so a whole Newton
// step runs without host synchronisation.  Reductions are block sums in a
// fixed order (deterministic).
#include <hip/hip_runtime.h>

#include "aux_kernels.h"
#include "device_util.h"
#include "kernels.h"

namespace cm {
namespace {

constexpr int kThreads = 1024;
// The residual kernel keeps more values live (the FP64 block inversion):
// 512-thread workgroups leave it 256 VGPRs instead of 128 (no spills).
constexpr int kResThreads = 512;

// Workgroup sum in a fixed order: a butterfly inside each wavefront (every
// lane ends with the same bits), then every thread adds the wavefront totals
// in wavefront order.  red: at least NT / 64 doubles of LDS.
template <int NT = kThreads>
__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) r += red[w];
  __syncthreads();  // red is reused by the next reduction
  return r;
}

// K workgroup sums at once, each in the order of block_sum (bitwise its
// result): the wavefront totals of sum k are added up by thread k alone, so
// no thread holds all K NT / 64 totals at once.  red: at least K (NT / 64 +
// 1) doubles.
template <int K, int NT = kThreads>
__device__ void block_sums(double (&v)[K], double* red) {
  constexpr int NW = NT / 64;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * NW + (threadIdx.x >> 6)] = v[k];
  }
  __syncthreads();
  if ((int)threadIdx.x < K) {
    const int k = threadIdx.x;
    double r = red[k * NW];
    for (int w = 1; w < NW; ++w) r += red[k * NW + w];
    red[K * NW + k] = r;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = red[K * NW + k];
  __syncthreads();  // red is reused by the next reduction
}

__device__ double block_max(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < kThreads / 64; ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

// Sphere indenter (Indenter with R > 0): node (x, y, z) against the sphere
// of cell c whose lowest point is at height top.  g = max(0, R - d) is the
// penetration, d the distance to the centre, n the unit vector from the
// centre to the node (zero without contact).  The penalty potential is
// (k/3) g^3 as for the plates: force k g^2 n on the node, k g^2 (c_z - z) / d
// upward on the sphere, Hessian 2 k g n n^T - k (g^2 / d) (I - n n^T).
struct SphereHit {
  double g, d, n[3];
};

__device__ __forceinline__ SphereHit sphere_hit(const Indenter& ind, int c, double top,
                                                double x, double y, double z) {
  SphereHit h;
  const double rx = x - ind.axis[2 * c], ry = y - ind.axis[2 * c + 1];
  const double rz = z - (top + ind.R);
  h.d = sqrt(rx * rx + ry * ry + rz * rz);
  h.g = h.d > 0.0 ? fmax(ind.R - h.d, 0.0) : 0.0;
  const double inv = h.g > 0.0 ? 1.0 / h.d : 0.0;
  h.n[0] = rx * inv;
  h.n[1] = ry * inv;
  h.n[2] = rz * inv;
  return h;
}

// Hessian of the sphere's penalty potential times v.
__device__ __forceinline__ void sphere_hess(const SphereHit& h, double k, double vx,
                                            double vy, double vz, double out[3]) {
  if (!(h.g > 0.0)) {
    out[0] = out[1] = out[2] = 0.0;
    return;
  }
  const double nv = h.n[0] * vx + h.n[1] * vy + h.n[2] * vz;
  const double a = 2.0 * k * h.g * nv, b = k * h.g * h.g / h.d;
  out[0] = a * h.n[0] - b * (vx - nv * h.n[0]);
  out[1] = a * h.n[1] - b * (vy - nv * h.n[1]);
  out[2] = a * h.n[2] - b * (vz - nv * h.n[2]);
}

// Projection onto the complement of the modes the sphere setup removes
// (translations in x and y, which the held centroid takes, and the rotation
// about the vertical axis through the centroid (cx, cy), a symmetry): from
// the cell sums sx = sum v_x, sy = sum v_y, sr = sum (dx v_y - dy v_x), with
// inv_n = 1 / nodes and ww = sum (dx^2 + dy^2).
struct ModeFit {
  double tx, ty, om;
};

__device__ __forceinline__ ModeFit mode_fit(double sx, double sy, double sr,
                                           double inv_n, double ww) {
  return ModeFit{sx * inv_n, sy * inv_n, ww > 0.0 ? sr / ww : 0.0};
}

// Inverse of the symmetric 3x3 block (xx yy zz xy xz yz) in float64; the
// identity where the block is not positive definite (unused nodes).
__device__ void sym3_inverse(const double m[6], float o[6]) {
  const double c00 = m[1] * m[2] - m[5] * m[5], c11 = m[0] * m[2] - m[4] * m[4];
  const double c22 = m[0] * m[1] - m[3] * m[3], c01 = m[4] * m[5] - m[3] * m[2];
  const double c02 = m[3] * m[5] - m[4] * m[1], c12 = m[3] * m[4] - m[0] * m[5];
  const double det = m[0] * c00 + m[3] * c01 + m[4] * c02;
  if (!(det > 0.0 && m[0] > 0.0 && c22 > 0.0) || !isfinite(det)) {
    o[0] = o[1] = o[2] = 1.f;
    o[3] = o[4] = o[5] = 0.f;
    return;
  }
  const double r = 1.0 / det;
  o[0] = (float)(c00 * r); o[1] = (float)(c11 * r); o[2] = (float)(c22 * r);
  o[3] = (float)(c01 * r); o[4] = (float)(c02 * r); o[5] = (float)(c12 * r);
}

// z = M r for one symmetric 3x3 block m = (xx yy zz xy xz yz).
__device__ __forceinline__ void sym3_mul(const float* m, float rx, float ry, float rz,
                                         float& zx, float& zy, float& zz) {
  zx = m[0] * rx + m[3] * ry + m[4] * rz;
  zy = m[3] * rx + m[1] * ry + m[5] * rz;
  zz = m[4] * rx + m[5] * ry + m[2] * rz;
}

// z = Minv r for node i (Minv SoA: xx yy zz xy xz yz, 6 n_nodes floats).
__device__ __forceinline__ void apply_minv(const float* mi, int64_t N, int64_t i,
                                           float rx, float ry, float rz, float& zx,
                                           float& zy, float& zz) {
  const float xx = mi[i], yy = mi[N + i], z2 = mi[2 * N + i];
  const float xy = mi[3 * N + i], xz = mi[4 * N + i], yz = mi[5 * N + i];
  zx = xx * rx + xy * ry + xz * rz;
  zy = xy * rx + yy * ry + yz * rz;
  zz = xz * rx + yz * ry + z2 * rz;
}

struct ResArgs {
  const int64_t* node_off;
  int64_t N;
  const float* y;
  const float* f;
  const double* energy;  // per cell E(y), nullable (no potential recorded)
  const double* plate;   // per cell: top, bottom
  double k, abs_tol, rel_tol, step_tol, floor_factor;
  double eta_max;  // largest CG forcing term (0: fixed CG tolerance)
  int restart;  // 1: first call at this plate position (forget the last step)
  float *r, *p, *x;
  float* rn;      // copy of the Newton residual (nullable)
  double* st;     // kQsState per cell
  double* force;  // per cell: top, bottom plate force (nullable)
  const float* kel;  // small-strain stiffness blocks (6 n_nodes), nullable
  float* minv;       // out with kel: inverse preconditioner blocks (6 n_nodes)
  Indenter ind;
};

// r = f + p (the negative gradient of Pi) with its components along the
// exact symmetries of the plate problem removed: translations along x and y
// and the rotation about the z axis through the centroid (the plates are
// invariant under them, so Hess(Pi) annihilates them and the forces have no
// net component along them up to rounding).  CG start x = 0, p = r.  A cell
// is active (not yet in equilibrium) when |r|_2 > max(abs_tol,
// rel_tol |pen|_2, floor_factor rho), pen the plate penalty forces and rho
// the cell's float32 floor (qs_floor_kernel), and its last Newton step moved
// some node by more than step_tol.
//
// Inexact Newton: with eta_max > 0 the CG of this Newton step stops at a
// relative residual eta (Eisenstat and Walker's second choice of forcing
// term, gamma = 0.9, exponent 2): eta = 0.9 (|r_N| / |r_N,prev|)^2, kept at
// least 0.9 eta_prev^2 when that exceeds 0.1, at most eta_max (eta_max at a
// new plate position), and at least half the ratio of the equilibrium
// tolerance to |r_N| (no more accuracy than the test needs).
__global__ __launch_bounds__(kResThreads) void qs_residual_kernel(ResArgs a) {
  __shared__ double red[64];
  const int c = blockIdx.x;
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1], N = a.N;
  const double top = a.plate[2 * c], bot = a.plate[2 * c + 1];
  const double inv_n = 1.0 / (double)(n1 - n0);
  const bool sph = a.ind.R > 0.0;  // uniform over the workgroup
  auto rz_of = [&](int64_t i, double& dt, double& db, double& pz) {
    const double z = a.y[2 * N + i];
    dt = fmax(z - top, 0.0);
    db = fmax(bot - z, 0.0);
    pz = a.k * (db * db - dt * dt);
    return (double)a.f[2 * N + i] + pz;
  };
  // lateral force of the sphere on node i (zero for the plates)
  auto lat = [&](int64_t i, double& px, double& py) {
    px = py = 0.0;
    if (sph) {
      const SphereHit h = sphere_hit(a.ind, c, top, a.y[i], a.y[N + i], a.y[2 * N + i]);
      px = a.k * h.g * h.g * h.n[0];
      py = a.k * h.g * h.g * h.n[1];
    }
  };
  // centroid (x, y) and mean residual (x, y)
  double sx = 0.0, sy = 0.0, mx = 0.0, my = 0.0;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kResThreads) {
    sx += a.y[i];
    sy += a.y[N + i];
    if (sph) {
      double px, py;
      lat(i, px, py);
      mx += (double)a.f[i] + px;
      my += (double)a.f[N + i] + py;
    } else {
      mx += a.f[i];
      my += a.f[N + i];
    }
  }
  const double cx = block_sum<kResThreads>(sx, red) * inv_n;
  const double cy = block_sum<kResThreads>(sy, red) * inv_n;
  mx = block_sum<kResThreads>(mx, red) * inv_n;
  my = block_sum<kResThreads>(my, red) * inv_n;
  // torque about the z axis through the centroid and |w|^2, w = e_z x (y - c)
  double tq = 0.0, ww = 0.0;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kResThreads) {
    const double dx = a.y[i] - cx, dy = a.y[N + i] - cy;
    if (sph) {
      double px, py;
      lat(i, px, py);
      tq += dx * ((double)a.f[N + i] + py) - dy * ((double)a.f[i] + px);
    } else {
      tq += dx * a.f[N + i] - dy * a.f[i];
    }
    ww += dx * dx + dy * dy;
  }
  tq = block_sum<kResThreads>(tq, red);
  ww = block_sum<kResThreads>(ww, red);
  const double om = ww > 0.0 ? tq / ww : 0.0;
  double rr = 0.0, rzs = 0.0, ft = 0.0, fb = 0.0, pp = 0.0, phi = 0.0;
  double zs[3] = {0.0, 0.0, 0.0};  // sphere: mode sums of z = M^-1 r
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kResThreads) {
    double dt, db, pz;
    double rzd = rz_of(i, dt, db, pz);
    double fx = a.f[i], fy = a.f[N + i];
    double blk_c[6] = {0.0, 0.0, 2.0 * a.k * (dt + db), 0.0, 0.0, 0.0};
    if (sph) {
      // the sphere in place of the top plate: dt = 0, its force on all axes
      const SphereHit h = sphere_hit(a.ind, c, top, a.y[i], a.y[N + i], a.y[2 * N + i]);
      const double kg2 = a.k * h.g * h.g, kg = 2.0 * a.k * h.g;
      dt = 0.0;
      pz = a.k * db * db + kg2 * h.n[2];
      rzd = (double)a.f[2 * N + i] + pz;
      fx += kg2 * h.n[0];
      fy += kg2 * h.n[1];
      phi += h.g * h.g * h.g;
      ft += kg2 * -h.n[2];
      pp += kg2 * h.n[0] * kg2 * h.n[0] + kg2 * h.n[1] * kg2 * h.n[1];
      // the preconditioner takes the positive part 2 k g n n^T of its Hessian
      blk_c[0] = kg * h.n[0] * h.n[0];
      blk_c[1] = kg * h.n[1] * h.n[1];
      blk_c[2] = 2.0 * a.k * db + kg * h.n[2] * h.n[2];
      blk_c[3] = kg * h.n[0] * h.n[1];
      blk_c[4] = kg * h.n[0] * h.n[2];
      blk_c[5] = kg * h.n[1] * h.n[2];
    }
    phi += dt * dt * dt + db * db * db;
    const double dx = a.y[i] - cx, dy = a.y[N + i] - cy;
    const float rx = (float)(fx - mx + om * dy);
    const float ry = (float)(fy - my - om * dx);
    const float rz = (float)rzd;
    pp += pz * pz;
    // preconditioned start direction p = z = M^-1 r, M = stiffness block +
    // penalty Hessian (2 k (max(0, z - top) + max(0, bottom - z)) on zz)
    float zx = rx, zy = ry, zz = rz;
    if (a.kel) {
      double blk[6] = {a.kel[i], a.kel[N + i], a.kel[2 * N + i] + blk_c[2],
                       a.kel[3 * N + i], a.kel[4 * N + i], a.kel[5 * N + i]};
      if (sph) {
        blk[0] += blk_c[0];
        blk[1] += blk_c[1];
        blk[3] += blk_c[3];
        blk[4] += blk_c[4];
        blk[5] += blk_c[5];
      }
      float o[6];
      sym3_inverse(blk, o);
#pragma unroll
      for (int q = 0; q < 6; ++q) a.minv[q * N + i] = o[q];
      apply_minv(a.minv, N, i, rx, ry, rz, zx, zy, zz);
    }
    a.r[i] = rx; a.r[N + i] = ry; a.r[2 * N + i] = rz;
    a.p[i] = zx; a.p[N + i] = zy; a.p[2 * N + i] = zz;
    rzs += (double)rx * zx + (double)ry * zy + (double)rz * zz;
    if (sph) {
      zs[0] += zx;
      zs[1] += zy;
      zs[2] += dx * zy - dy * zx;
    }
    a.x[i] = 0.f; a.x[N + i] = 0.f; a.x[2 * N + i] = 0.f;
    if (a.rn) { a.rn[i] = rx; a.rn[N + i] = ry; a.rn[2 * N + i] = rz; }
    rr += (double)rx * rx + (double)ry * ry + (double)rz * rz;
    ft += a.k * dt * dt;
    fb += a.k * db * db;
  }
  if (sph) {
    // p = z projected like r (the CG then stays in the complement of the
    // modes); r . z is unchanged by it since r lies in that complement
    block_sums<3, kResThreads>(zs, red);
    const ModeFit m = mode_fit(zs[0], zs[1], zs[2], inv_n, ww);
    for (int64_t i = n0 + threadIdx.x; i < n1; i += kResThreads) {
      const double dx = a.y[i] - cx, dy = a.y[N + i] - cy;
      a.p[i] = (float)((double)a.p[i] - m.tx + m.om * dy);
      a.p[N + i] = (float)((double)a.p[N + i] - m.ty - m.om * dx);
    }
    if (threadIdx.x == 0) {
      a.ind.geo[3 * c] = cx;
      a.ind.geo[3 * c + 1] = cy;
      a.ind.geo[3 * c + 2] = ww;
    }
  }
  rr = block_sum<kResThreads>(rr, red);
  rzs = block_sum<kResThreads>(rzs, red);
  ft = block_sum<kResThreads>(ft, red);
  fb = block_sum<kResThreads>(fb, red);
  pp = block_sum<kResThreads>(pp, red);
  phi = block_sum<kResThreads>(phi, red) * (a.k / 3.0);
  if (threadIdx.x == 0) {
    double* s = a.st + kQsState * c;
    const double fl = a.floor_factor * s[7];
    const double tol2 = fmax(fmax(a.abs_tol * a.abs_tol, a.rel_tol * a.rel_tol * pp), fl * fl);
    if (a.restart) s[6] = __builtin_inf();
    s[0] = rzs;                     // CG r . z (|r|^2 without preconditioner)
    s[1] = rr;                      // |r_0|^2
    const double act = (rr > tol2 && s[6] > a.step_tol) ? 1.0 : 0.0;
    double eta = 0.0;
    if (a.eta_max > 0.0) {
      const double prev = s[15], eta_prev = s[14];
      if (a.restart || !(prev > 0.0)) {
        eta = a.eta_max;
      } else {
        eta = 0.9 * rr / prev;
        const double sg = 0.9 * eta_prev * eta_prev;
        if (sg > 0.1) eta = fmax(eta, sg);
      }
      if (rr > 0.0) eta = fmax(eta, 0.5 * sqrt(tol2 / rr));
      eta = fmin(eta, a.eta_max);
    }
    s[14] = eta;                    // CG forcing term of this Newton step
    s[15] = rr;                     // |r_N|^2 for the next forcing term
    s[2] = act;                     // CG active
    s[11] = act;                    // not yet in equilibrium
    s[3] = rr;                      // Newton residual |f + p|^2 (projected)
    s[5] = pp;                      // |penalty forces|^2
    if (a.energy) s[8] = a.energy[c] + phi;  // Pi(y)
    if (a.force) { a.force[2 * c] = ft; a.force[2 * c + 1] = fb; }
  }
}

// Preconditioner of the Newton systems: the diagonal 3x3 blocks of the
// small-strain (linear-elastic) stiffness, shear modulus mu and bulk modulus
// kappa being the small-strain limit of the energy.  Per tetrahedron and
// vertex a with gradient row b_a (row a of B, b_4 = -(b_1 + b_2 + b_3)) the
// block is V0 (mu |b_a|^2 I + (kappa + mu/3) b_a b_a^T); one wavefront per
// tile adds them per node in LDS (the chunk colouring keeps the lanes of a
// vertex slot on distinct nodes), pass 0 the (xx, yy, zz) entries, pass 1
// (xy, xz, yz); owned nodes are stored, shared nodes go through the slot
// partials and the forward finalize pass.
struct StiffArgs {
  DeviceTables T;
  int pass;
  float* out;  // 3 n_nodes floats (SoA) of this pass
};

__global__ __launch_bounds__(64) void qs_stiffness_kernel(StiffArgs a) {
  extern __shared__ float4 acc[];
  const int lane = threadIdx.x;
  const int t = blockIdx.x;
  const TileDesc d = a.T.tiles[t];
  const int mt = a.T.tile_mat[t], nm = a.T.n_mat;
  const float mu = (float)a.T.params[mt];
  const float cb = (float)a.T.params[nm + mt] + mu * (1.f / 3.f);
  const int64_t N = a.T.n_nodes;
  for (int l = lane; l < d.n_own + d.n_shr; l += 64) acc[l] = make_float4(0.f, 0.f, 0.f, 0.f);
  wave_sync();
  const TetChunk* ch = a.T.chunks + d.chunk_begin;
  for (int k = 0; k < d.n_chunks; ++k) {
    TetRegs tr;
    load_tet(ch + k, lane, tr);
    const uint2 q = tr.q;
    if (q.x != kEmptyLane) {
      const int idx[4] = {(int)(q.x & 0xffff), (int)(q.x >> 16), (int)(q.y & 0xffff),
                          (int)(q.y >> 16)};
      float b[4][3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int j = 0; j < 3; ++j) b[r][j] = tr.B[3 * r + j];
#pragma unroll
      for (int j = 0; j < 3; ++j) b[3][j] = -(b[0][j] + b[1][j] + b[2][j]);
      const float v0 = tr.V0;
      // vertex slots in order: the lanes of one slot name distinct nodes
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float* g = b[s];
        float e0, e1, e2;
        if (a.pass == 0) {
          const float nb = mu * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
          e0 = v0 * (nb + cb * g[0] * g[0]);
          e1 = v0 * (nb + cb * g[1] * g[1]);
          e2 = v0 * (nb + cb * g[2] * g[2]);
        } else {
          e0 = v0 * cb * g[0] * g[1];
          e1 = v0 * cb * g[0] * g[2];
          e2 = v0 * cb * g[1] * g[2];
        }
        float4 v = acc[idx[s]];
        v.x += e0; v.y += e1; v.z += e2;
        acc[idx[s]] = v;
      }
    }
  }
  wave_sync();
  for (int i = lane; i < d.n_own; i += 64) {
    const int64_t g = d.own_begin + i;
    const float4 v = acc[i];
    a.out[g] = v.x; a.out[N + g] = v.y; a.out[2 * N + g] = v.z;
  }
  for (int j = lane; j < d.n_shr; j += 64) {
    const float4 v = acc[d.n_own + j];
    float* pp = a.T.part + 3 * ((int64_t)d.shr_begin + j);
    pp[0] = v.x; pp[1] = v.y; pp[2] = v.z;
  }
}

struct CgArgs {
  const int64_t* node_off;
  int64_t N;
  const float* y;
  const double* plate;
  double k, rel_tol;
  const float* ybar;  // (df/dy)^T p
  float *x, *r, *p, *Ap;
  double* st;
  const float* minv;  // preconditioner blocks (6 n_nodes), nullable
  // With part set, ybar holds the owned nodes only (a backward tile pass
  // without its finalize) and the shared nodes' values are the sums of
  // their slot partials, formed here in the finalize's order.
  const float* part;
  const int32_t* shared_slot_ptr;
  const int32_t* shared_slots;
  const int32_t* cell_shared_off;
  const int32_t* cell_shared_first;  // first shared node of every cell
  Indenter ind;
};

// The shared nodes of a cell are the contiguous ids [sh0, sh0 + ns) (owned
// nodes first, see layout.h); s0 is the cell's first shared-node entry.
struct ShrRange {
  int64_t sh0, sh1;
  int s0;
};

__device__ __forceinline__ ShrRange shared_range(const CgArgs& a, int c, int64_t n1) {
  ShrRange r{n1, n1, 0};
  if (a.part) {
    r.s0 = a.cell_shared_off[c];
    const int ns = a.cell_shared_off[c + 1] - r.s0;
    if (ns > 0) {
      r.sh0 = a.cell_shared_first[c];
      r.sh1 = r.sh0 + ns;
    }
  }
  return r;
}

// ybar of node i: stored, or for a shared node the sum of its slot partials
// in slot order (the order of backward_finalize_kernel: bitwise its result).
__device__ __forceinline__ void ybar_of(const CgArgs& a, const ShrRange& sr, int64_t i,
                                        float& bx, float& by, float& bz) {
  if (i >= sr.sh0 && i < sr.sh1) {
    const int s = sr.s0 + (int)(i - sr.sh0);
    float sx = 0.f, sy = 0.f, sz = 0.f;
    for (int q = a.shared_slot_ptr[s]; q < a.shared_slot_ptr[s + 1]; ++q) {
      const float* pp = a.part + 3 * (int64_t)a.shared_slots[q];
      sx += pp[0];
      sy += pp[1];
      sz += pp[2];
    }
    bx = sx; by = sy; bz = sz;
  } else {
    bx = a.ybar[i]; by = a.ybar[a.N + i]; bz = a.ybar[2 * a.N + i];
  }
}

// Nodes per thread up to which a cell's CG iteration keeps every operand in
// registers (cells of at most kRegNodes * kThreads nodes; cells of at most
// kThreads * 2 nodes take a 2-node variant that needs fewer registers).
constexpr int kRegNodes = 4;

__device__ __forceinline__ void cg_finish(const CgArgs& a, double* s, double rn,
                                          double rzn) {
  if (threadIdx.x == 0) {
    s[0] = rzn;
    const double tol = fmax(a.rel_tol, s[14]);
    if (rn <= tol * tol * s[1]) s[2] = 0.0;
  }
}


// The iteration of qs_cg_kernel for a cell of at most R * kThreads nodes: p,
// r, x, Hess(Pi) p and the preconditioner block of every node are loaded
// once and kept in registers through the three phases (Ap is not stored).
// The loads come in three waves, each issued whole before any of its
// results is used: the node values with the slot ranges of the shared
// nodes, then the ids of their first FS slots (most shared nodes have 2 or
// 3; the others finish in a loop), then those slots' partials, summed in
// slot order as the finalize does.  Same operations in the same order as
// the streaming version (which fused multiply-adds the compiler forms may
// differ between the two, a last-bit difference).
template <int R, bool SPH>
__device__ void cg_step_regs(const CgArgs& a, double* s, int c, int64_t n0, int64_t n1,
                             double top, double bot, double* red, const ShrRange& sr) {
  constexpr int kRegNodes = R;
  constexpr int kFastSlots = R <= 2 ? 4 : 2;
  const int64_t N = a.N;
  float p[kRegNodes][3], r[kRegNodes][3], ap[kRegNodes][3], x[kRegNodes][3];
  float m[kRegNodes][6], b[kRegNodes][3];
  double h[kRegNodes];        // plates: penalty Hessian on zz
  float yv[kRegNodes][3];     // sphere: positions
  int q0[kRegNodes], nq[kRegNodes];
#pragma unroll
  for (int u = 0; u < kRegNodes; ++u) {
    const int64_t i = n0 + threadIdx.x + (int64_t)u * kThreads;
    nq[u] = 0;
    q0[u] = 0;
    if (i < n1) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        p[u][d] = a.p[d * N + i];
        r[u][d] = a.r[d * N + i];
        x[u][d] = a.x[d * N + i];
      }
      if (a.minv) {
#pragma unroll
        for (int q = 0; q < 6; ++q) m[u][q] = a.minv[q * N + i];
      }
      if constexpr (SPH) {
#pragma unroll
        for (int d = 0; d < 3; ++d) yv[u][d] = a.y[d * N + i];
      } else {
        const double z = a.y[2 * N + i];
        h[u] = 2.0 * a.k * (fmax(z - top, 0.0) + fmax(bot - z, 0.0));
      }
      if (i >= sr.sh0 && i < sr.sh1) {
        const int sn = sr.s0 + (int)(i - sr.sh0);
        q0[u] = a.shared_slot_ptr[sn];
        nq[u] = a.shared_slot_ptr[sn + 1] - q0[u];
        b[u][0] = b[u][1] = b[u][2] = 0.f;
      } else {
        b[u][0] = a.ybar[i];
        b[u][1] = a.ybar[N + i];
        b[u][2] = a.ybar[2 * N + i];
      }
    }
  }
  int sl[kRegNodes][kFastSlots];
#pragma unroll
  for (int u = 0; u < kRegNodes; ++u)
#pragma unroll
    for (int j = 0; j < kFastSlots; ++j)
      sl[u][j] = j < nq[u] ? a.shared_slots[q0[u] + j] : 0;
#pragma unroll
  for (int u = 0; u < kRegNodes; ++u) {
#pragma unroll
    for (int j = 0; j < kFastSlots; ++j) {
      if (j < nq[u]) {
        const float* pp = a.part + 3 * (int64_t)sl[u][j];
        b[u][0] += pp[0];
        b[u][1] += pp[1];
        b[u][2] += pp[2];
      }
    }
    for (int j = kFastSlots; j < nq[u]; ++j) {
      const float* pp = a.part + 3 * (int64_t)a.shared_slots[q0[u] + j];
      b[u][0] += pp[0];
      b[u][1] += pp[1];
      b[u][2] += pp[2];
    }
  }
  // sphere: centroid and sum (dx^2 + dy^2) of the Newton step's positions
  double gcx = 0.0, gcy = 0.0, gww = 0.0;
  if constexpr (SPH) {
    gcx = a.ind.geo[3 * c];
    gcy = a.ind.geo[3 * c + 1];
    gww = a.ind.geo[3 * c + 2];
  }
  const double inv_n = 1.0 / (double)(n1 - n0);
  double pap = 0.0, sa[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < kRegNodes; ++u) {
    const int64_t i = n0 + threadIdx.x + (int64_t)u * kThreads;
    if (i < n1) {
      if constexpr (SPH) {
        const SphereHit hh = sphere_hit(a.ind, c, top, yv[u][0], yv[u][1], yv[u][2]);
        double hp[3];
        sphere_hess(hh, a.k, p[u][0], p[u][1], p[u][2], hp);
        hp[2] += 2.0 * a.k * fmax(bot - (double)yv[u][2], 0.0) * (double)p[u][2];
#pragma unroll
        for (int d = 0; d < 3; ++d) ap[u][d] = (float)(-(double)b[u][d] + hp[d]);
        const double dx = yv[u][0] - gcx, dy = yv[u][1] - gcy;
        sa[0] += ap[u][0];
        sa[1] += ap[u][1];
        sa[2] += dx * ap[u][1] - dy * ap[u][0];
      } else {
        ap[u][0] = -b[u][0];
        ap[u][1] = -b[u][1];
        ap[u][2] = (float)(-(double)b[u][2] + h[u] * (double)p[u][2]);
      }
      pap += (double)p[u][0] * ap[u][0] + (double)p[u][1] * ap[u][1] +
             (double)p[u][2] * ap[u][2];
    }
  }
  ModeFit ma{0.0, 0.0, 0.0};
  if constexpr (SPH) {
    double v[4] = {pap, sa[0], sa[1], sa[2]};
    block_sums(v, red);
    pap = v[0];
    ma = mode_fit(v[1], v[2], v[3], inv_n, gww);
  } else {
    pap = block_sum(pap, red);
  }
  const double rs = s[0];
  if (!(pap > 0.0)) {
    if (threadIdx.x == 0) s[2] = 0.0;
    return;
  }
  const float alpha = (float)(rs / pap);
  double rn = 0.0, rzn = 0.0, sz[3] = {0.0, 0.0, 0.0};
  float zv[kRegNodes][3];
#pragma unroll
  for (int u = 0; u < kRegNodes; ++u) {
    const int64_t i = n0 + threadIdx.x + (int64_t)u * kThreads;
    if (i < n1) {
      if constexpr (SPH) {
        // Ap projected: the held centroid and the symmetry take its mode part
        const double dx = yv[u][0] - gcx, dy = yv[u][1] - gcy;
        ap[u][0] = (float)((double)ap[u][0] - ma.tx + ma.om * dy);
        ap[u][1] = (float)((double)ap[u][1] - ma.ty - ma.om * dx);
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int64_t q = d * N + i;
        a.x[q] = x[u][d] + alpha * p[u][d];
        r[u][d] = r[u][d] - alpha * ap[u][d];
        a.r[q] = r[u][d];
        rn += (double)r[u][d] * r[u][d];
      }
      zv[u][0] = r[u][0];
      zv[u][1] = r[u][1];
      zv[u][2] = r[u][2];
      if (a.minv) sym3_mul(m[u], r[u][0], r[u][1], r[u][2], zv[u][0], zv[u][1], zv[u][2]);
      rzn += (double)r[u][0] * zv[u][0] + (double)r[u][1] * zv[u][1] +
             (double)r[u][2] * zv[u][2];
      if constexpr (SPH) {
        const double dx = yv[u][0] - gcx, dy = yv[u][1] - gcy;
        sz[0] += zv[u][0];
        sz[1] += zv[u][1];
        sz[2] += dx * zv[u][1] - dy * zv[u][0];
      }
    }
  }
  ModeFit mz{0.0, 0.0, 0.0};
  if constexpr (SPH) {
    double v[5] = {rn, rzn, sz[0], sz[1], sz[2]};
    block_sums(v, red);
    rn = v[0];
    rzn = v[1];
    mz = mode_fit(v[2], v[3], v[4], inv_n, gww);
  } else {
    double sums[2] = {rn, rzn};
    block_sums(sums, red);
    rn = sums[0];
    rzn = sums[1];
  }
  const float beta = (float)(rzn / rs);
#pragma unroll
  for (int u = 0; u < kRegNodes; ++u) {
    const int64_t i = n0 + threadIdx.x + (int64_t)u * kThreads;
    if (i < n1) {
      if constexpr (SPH) {
        const double dx = yv[u][0] - gcx, dy = yv[u][1] - gcy;
        zv[u][0] = (float)((double)zv[u][0] - mz.tx + mz.om * dy);
        zv[u][1] = (float)((double)zv[u][1] - mz.ty - mz.om * dx);
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) a.p[d * N + i] = zv[u][d] + beta * p[u][d];
    }
  }
  cg_finish(a, s, rn, rzn);
}

// One (preconditioned) CG iteration per active cell, z = M^-1 r (z = r
// without preconditioner): Ap = Hess(Pi) p, alpha = r.z / p.Ap, x += alpha p,
// r -= alpha Ap, beta = r_new.z_new / r.z, p = z_new + beta p.  A cell stops
// at |r| <= max(rel_tol, eta) |r_0| (eta the forcing term of the Newton
// step, 0 without forcing) or on non-positive curvature.  Cells of up to
// kRegNodes * kThreads nodes keep their operands in registers; larger ones
// stream them three times (Ap through memory).  SPH (the sphere indenter):
// the contact Hessian is a 3x3 block per node, and Ap and z are projected
// onto the complement of the lateral translations and the rotation about
// the vertical axis (the residual and the first direction are projected by
// the residual kernel), so the iterates stay there: the CG of the system
// with the centroid held.
template <bool SPH>
__global__ __launch_bounds__(kThreads) void qs_cg_kernel(CgArgs a) {
  __shared__ double red[kThreads];
  const int c = blockIdx.x;
  double* s = a.st + kQsState * c;
  if (s[2] == 0.0) return;  // uniform over the workgroup
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1], N = a.N;
  const double top = a.plate[2 * c], bot = a.plate[2 * c + 1];
  const ShrRange sr = shared_range(a, c, n1);
  if (n1 - n0 <= (int64_t)2 * kThreads) {
    cg_step_regs<2, SPH>(a, s, c, n0, n1, top, bot, red, sr);
    return;
  }
  if constexpr (!SPH) {
    // (the sphere's 4-node variant would exceed 128 VGPRs: its cells of more
    // than 2,048 nodes stream)
    if (n1 - n0 <= (int64_t)kRegNodes * kThreads) {
      cg_step_regs<kRegNodes, SPH>(a, s, c, n0, n1, top, bot, red, sr);
      return;
    }
  }
  double gcx = 0.0, gcy = 0.0, gww = 0.0;
  if constexpr (SPH) {
    gcx = a.ind.geo[3 * c];
    gcy = a.ind.geo[3 * c + 1];
    gww = a.ind.geo[3 * c + 2];
  }
  const double inv_n = 1.0 / (double)(n1 - n0);
  double pap = 0.0, sa[3] = {0.0, 0.0, 0.0};

  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
    float bx, by, bz;
    ybar_of(a, sr, i, bx, by, bz);
    float ax, ay, az;
    if constexpr (SPH) {
      const double yx = a.y[i], yy = a.y[N + i], yz = a.y[2 * N + i];
      const SphereHit hh = sphere_hit(a.ind, c, top, yx, yy, yz);
      double hp[3];
      sphere_hess(hh, a.k, a.p[i], a.p[N + i], a.p[2 * N + i], hp);
      hp[2] += 2.0 * a.k * fmax(bot - yz, 0.0) * (double)a.p[2 * N + i];
      ax = (float)(-(double)bx + hp[0]);
      ay = (float)(-(double)by + hp[1]);
      az = (float)(-(double)bz + hp[2]);
      const double dx = yx - gcx, dy = yy - gcy;
      sa[0] += ax;
      sa[1] += ay;
      sa[2] += dx * ay - dy * ax;
    } else {
      const double z = a.y[2 * N + i];
      const double h = 2.0 * a.k * (fmax(z - top, 0.0) + fmax(bot - z, 0.0));
      ax = -bx;
      ay = -by;
      az = (float)(-(double)bz + h * (double)a.p[2 * N + i]);
    }
    a.Ap[i] = ax; a.Ap[N + i] = ay; a.Ap[2 * N + i] = az;
    pap += (double)a.p[i] * ax + (double)a.p[N + i] * ay + (double)a.p[2 * N + i] * az;
  }
  ModeFit ma{0.0, 0.0, 0.0};
  if constexpr (SPH) {
    double v[4] = {pap, sa[0], sa[1], sa[2]};
    block_sums(v, red);
    pap = v[0];
    ma = mode_fit(v[1], v[2], v[3], inv_n, gww);
  } else {
    pap = block_sum(pap, red);
  }
  const double rs = s[0];
  if (!(pap > 0.0)) {
    if (threadIdx.x == 0) s[2] = 0.0;
    return;
  }
  const float alpha = (float)(rs / pap);
  double rn = 0.0, rzn = 0.0, sz[3] = {0.0, 0.0, 0.0};
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
    float apv[3] = {a.Ap[i], a.Ap[N + i], a.Ap[2 * N + i]};
    double dx = 0.0, dy = 0.0;
    if constexpr (SPH) {
      dx = a.y[i] - gcx;
      dy = a.y[N + i] - gcy;
      apv[0] = (float)((double)apv[0] - ma.tx + ma.om * dy);
      apv[1] = (float)((double)apv[1] - ma.ty - ma.om * dx);
    }
    float rq[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t q = d * N + i;
      a.x[q] += alpha * a.p[q];
      rq[d] = a.r[q] - alpha * apv[d];
      a.r[q] = rq[d];
      rn += (double)rq[d] * rq[d];
    }
    float z[3] = {rq[0], rq[1], rq[2]};
    if (a.minv) apply_minv(a.minv, N, i, rq[0], rq[1], rq[2], z[0], z[1], z[2]);
    rzn += (double)rq[0] * z[0] + (double)rq[1] * z[1] + (double)rq[2] * z[2];
    if constexpr (SPH) {
      sz[0] += z[0];
      sz[1] += z[1];
      sz[2] += dx * z[1] - dy * z[0];
    }
  }
  ModeFit mz{0.0, 0.0, 0.0};
  if constexpr (SPH) {
    double v[5] = {rn, rzn, sz[0], sz[1], sz[2]};
    block_sums(v, red);
    rn = v[0];
    rzn = v[1];
    mz = mode_fit(v[2], v[3], v[4], inv_n, gww);
  } else {
    double sums[2] = {rn, rzn};
    block_sums(sums, red);
    rn = sums[0];
    rzn = sums[1];
  }
  const float beta = (float)(rzn / rs);
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
    float z[3] = {a.r[i], a.r[N + i], a.r[2 * N + i]};
    if (a.minv) apply_minv(a.minv, N, i, z[0], z[1], z[2], z[0], z[1], z[2]);
    if constexpr (SPH) {
      const double dx = a.y[i] - gcx, dy = a.y[N + i] - gcy;
      z[0] = (float)((double)z[0] - mz.tx + mz.om * dy);
      z[1] = (float)((double)z[1] - mz.ty - mz.om * dx);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t q = d * N + i;
      a.p[q] = z[d] + beta * a.p[q];
    }
  }
  cg_finish(a, s, rn, rzn);
}

// Adjoint of the equilibrium for the top-plate force.  At an equilibrium
// f(y; theta) + p(y) = 0 the derivative of F_top = k sum max(0, z - top)^2
// along the parameters is dF_top/dtheta = lam^T df/dtheta with
// Hess(Pi) lam = g, g = dF_top/dy (2 k max(0, z - top) on the z entries, 0
// elsewhere): one more CG solve on the same Hessian-vector products.  This
// kernel starts that solve: r = w_c g (w_c = weight[c], 1 when null), p =
// M^-1 r, x = 0, CG state r . z, |r|^2, active iff |r| > 0, forcing term 0
// (the CG runs to its own tolerance).  g is orthogonal to the symmetry modes
// of the plates (it has z entries only), so the singular system is
// consistent.
struct AdjArgs {
  const int64_t* node_off;
  int64_t N;
  const float* y;
  const double* plate;
  double k;
  const double* weight;
  float *r, *p, *x;
  double* st;
  const float* minv;
  Indenter ind;
};

__global__ __launch_bounds__(kThreads) void qs_adjoint_rhs_kernel(AdjArgs a) {
  __shared__ double red[kThreads];
  const int c = blockIdx.x;
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1], N = a.N;
  const double top = a.plate[2 * c];
  const double w = a.weight ? a.weight[c] : 1.0;
  double rr = 0.0, rz = 0.0;
  if (a.ind.R > 0.0) {  // uniform over the workgroup
    // sphere: F = k sum g^2 m with m = (c_z - z) / d = -n_z, so
    // dF/dy = -k (2 g m n + (g^2 / d)(e_z + m n)); r = w P dF/dy and p = P M^-1 r
    // with P the projection of the held centroid and the rotation symmetry
    // (centroid and sum (dx^2 + dy^2) of the last residual's positions)
    const double gcx = a.ind.geo[3 * c], gcy = a.ind.geo[3 * c + 1];
    const double gww = a.ind.geo[3 * c + 2];
    const double inv_n = 1.0 / (double)(n1 - n0);
    double sg[3] = {0.0, 0.0, 0.0};
    for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
      const double yx = a.y[i], yy = a.y[N + i], yz = a.y[2 * N + i];
      const SphereHit h = sphere_hit(a.ind, c, top, yx, yy, yz);
      double g[3] = {0.0, 0.0, 0.0};
      if (h.g > 0.0) {
        const double m = -h.n[2], q = h.g * h.g / h.d;
#pragma unroll
        for (int d = 0; d < 3; ++d) g[d] = -w * a.k * (2.0 * h.g * m * h.n[d] + q * m * h.n[d]);
        g[2] -= w * a.k * q;
      }
      const float gx = (float)g[0], gy = (float)g[1];
      a.r[i] = gx; a.r[N + i] = gy; a.r[2 * N + i] = (float)g[2];
      const double dx = yx - gcx, dy = yy - gcy;
      sg[0] += gx;
      sg[1] += gy;
      sg[2] += dx * gy - dy * gx;
    }
    block_sums(sg, red);
    const ModeFit mg = mode_fit(sg[0], sg[1], sg[2], inv_n, gww);
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // |r|^2, r . z, mode sums of z
    for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
      const double dx = a.y[i] - gcx, dy = a.y[N + i] - gcy;
      const float rx = (float)((double)a.r[i] - mg.tx + mg.om * dy);
      const float ry = (float)((double)a.r[N + i] - mg.ty - mg.om * dx);
      const float rzv = a.r[2 * N + i];
      float zx = rx, zy = ry, zz = rzv;
      if (a.minv) apply_minv(a.minv, N, i, rx, ry, rzv, zx, zy, zz);
      a.r[i] = rx; a.r[N + i] = ry;
      a.p[i] = zx; a.p[N + i] = zy; a.p[2 * N + i] = zz;
      a.x[i] = 0.f; a.x[N + i] = 0.f; a.x[2 * N + i] = 0.f;
      v[0] += (double)rx * rx + (double)ry * ry + (double)rzv * rzv;
      v[1] += (double)rx * zx + (double)ry * zy + (double)rzv * zz;
      v[2] += zx;
      v[3] += zy;
      v[4] += dx * zy - dy * zx;
    }
    block_sums(v, red);
    const ModeFit mz = mode_fit(v[2], v[3], v[4], inv_n, gww);
    for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
      const double dx = a.y[i] - gcx, dy = a.y[N + i] - gcy;
      a.p[i] = (float)((double)a.p[i] - mz.tx + mz.om * dy);
      a.p[N + i] = (float)((double)a.p[N + i] - mz.ty - mz.om * dx);
    }
    if (threadIdx.x == 0) {
      double* s = a.st + kQsState * c;
      s[0] = v[1];
      s[1] = v[0];
      s[2] = v[0] > 0.0 ? 1.0 : 0.0;
      s[14] = 0.0;
    }
    return;
  }
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
    const double z = a.y[2 * N + i];
    const float g = (float)(w * 2.0 * a.k * fmax(z - top, 0.0));
    float zx = 0.f, zy = 0.f, zz = g;
    if (a.minv) apply_minv(a.minv, N, i, 0.f, 0.f, g, zx, zy, zz);
    a.r[i] = 0.f; a.r[N + i] = 0.f; a.r[2 * N + i] = g;
    a.p[i] = zx; a.p[N + i] = zy; a.p[2 * N + i] = zz;
    a.x[i] = 0.f; a.x[N + i] = 0.f; a.x[2 * N + i] = 0.f;
    rr += (double)g * g;
    rz += (double)g * zz;
  }
  rr = block_sum(rr, red);
  rz = block_sum(rz, red);
  if (threadIdx.x == 0) {
    double* s = a.st + kQsState * c;
    s[0] = rz;
    s[1] = rr;
    s[2] = rr > 0.0 ? 1.0 : 0.0;
    s[14] = 0.0;
  }
}

// Float32 floor of the residual.  Positions held in float32 carry rounding
// errors of up to half a unit in the last place, so the residual of a
// float32 state cannot be resolved below |Hess(Pi) e| for such an error e.
// qs_noise_kernel writes e_q = +-|y_q| 2^-24 with a sign from a fixed hash of
// the index; after the Hessian-vector product ybar = (df/dy)^T e,
// qs_floor_kernel stores rho = |-ybar + penalty diagonal e|_2 per cell.
__global__ __launch_bounds__(kThreads) void qs_noise_kernel(const int64_t* node_off,
                                                            int64_t N, const float* y,
                                                            float* e) {
  const int c = blockIdx.x;
  const int64_t n0 = node_off[c], n1 = node_off[c + 1];
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t q = d * N + i;
      const uint32_t hsh = (uint32_t)q * 2654435761u;
      const float mag = fabsf(y[q]) * 5.9604645e-8f;  // 2^-24
      e[q] = (hsh >> 16) & 1u ? mag : -mag;
    }
}

struct FloorArgs {
  const int64_t* node_off;
  int64_t N;
  const float* y;
  const double* plate;
  double k;
  const float* e;
  const float* ybar;
  double* st;
  Indenter ind;
};

__global__ __launch_bounds__(kThreads) void qs_floor_kernel(FloorArgs a) {
  __shared__ double red[kThreads];
  const int c = blockIdx.x;
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1], N = a.N;
  const double top = a.plate[2 * c], bot = a.plate[2 * c + 1];
  double acc = 0.0;
  const bool sph = a.ind.R > 0.0;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
    const double z = a.y[2 * N + i];
    double hx = -(double)a.ybar[i], hy = -(double)a.ybar[N + i], hz;
    if (sph) {
      const SphereHit hh = sphere_hit(a.ind, c, top, a.y[i], a.y[N + i], z);
      double he[3];
      sphere_hess(hh, a.k, a.e[i], a.e[N + i], a.e[2 * N + i], he);
      hx += he[0];
      hy += he[1];
      hz = -(double)a.ybar[2 * N + i] + he[2] +
           2.0 * a.k * fmax(bot - z, 0.0) * (double)a.e[2 * N + i];
    } else {
      const double h = 2.0 * a.k * (fmax(z - top, 0.0) + fmax(bot - z, 0.0));
      hz = -(double)a.ybar[2 * N + i] + h * (double)a.e[2 * N + i];
    }
    acc += hx * hx + hy * hy + hz * hz;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) a.st[kQsState * c + 7] = sqrt(acc);
}

struct UpdArgs {
  const int64_t* node_off;
  int64_t N;
  const float* x;
  double cap;
  float* y;
  double* st;
};

// y += s x with s = min(1, cap / max |x_i|) per cell (a bounded Newton step);
// the applied scale goes to the state.
__global__ __launch_bounds__(kThreads) void qs_update_kernel(UpdArgs a) {
  __shared__ double red[kThreads];
  const int c = blockIdx.x;
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1], N = a.N;
  double mx = 0.0;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads)
    mx = fmax(mx, fmax(fabs((double)a.x[i]),
                       fmax(fabs((double)a.x[N + i]), fabs((double)a.x[2 * N + i]))));
  mx = block_max(mx, red);
  const float sc = (float)(mx > a.cap ? a.cap / mx : 1.0);
  // a cell that took no step (converged) keeps its last step size
  const bool moved = mx > 0.0;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
    a.y[i] += sc * a.x[i];
    a.y[N + i] += sc * a.x[N + i];
    a.y[2 * N + i] += sc * a.x[2 * N + i];
  }
  if (threadIdx.x == 0 && moved) {
    a.st[kQsState * c + 4] = sc;
    a.st[kQsState * c + 6] = mx * sc;  // largest node move of this step
  }
}

struct LsArgs {
  const int64_t* node_off;
  int64_t N;
  float* x;  // projected in place by the start kernel
  const float* rn;         // Newton residual (-grad Pi, projected)
  const double* plate;
  const double* energy_t;  // E at the trial positions (accept)
  double k, cap, armijo, min_move;
  float* y;
  float* yt;               // trial positions
  double* st;
  const int32_t* ninv_t;   // inverted tetrahedra at y_t (nullable)
  int32_t* ninv;           // inverted tetrahedra at y (nullable)
  Indenter ind;
};

// Start of the line search on Pi along the Newton step x: x loses its
// components along the symmetries of the plates (translations in x and y,
// rotation about z through the centroid of y), which Hess(Pi) annihilates
// and the preconditioned CG therefore never corrects: they change neither
// Pi nor the slope, but they inflate max |x| (a shorter capped step) and a
// finite rotation stretches the cell radially.  Then s = min(1, cap /
// max |x_i|), slope r_N . x (> 0 for a descent direction), y_t = y + s x for
// the cells in equilibrium-search, y_t = y for the others.
__global__ __launch_bounds__(kThreads) void qs_ls_start_kernel(LsArgs a) {
  __shared__ double red[kThreads];
  const int c = blockIdx.x;
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1], N = a.N;
  double* s = a.st + kQsState * c;
  const bool act = s[11] != 0.0;
  double mx = 0.0, rx = 0.0;
  if (act) {  // uniform over the workgroup
    const double inv_n = 1.0 / (double)(n1 - n0);
    double sx = 0.0, sy = 0.0, tx = 0.0, ty = 0.0;
#pragma unroll 1
    for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
      sx += a.y[i];
      sy += a.y[N + i];
      tx += a.x[i];
      ty += a.x[N + i];
    }
    double c4[4] = {sx, sy, tx, ty};
    block_sums(c4, red);
    const double cx = c4[0] * inv_n, cy = c4[1] * inv_n;
    tx = c4[2] * inv_n;
    ty = c4[3] * inv_n;
    // x . w / |w|^2 for w = e_z x (y - c)
    double tq = 0.0, ww = 0.0;
#pragma unroll 1
    for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
      const double dx = a.y[i] - cx, dy = a.y[N + i] - cy;
      tq += dx * a.x[N + i] - dy * a.x[i];
      ww += dx * dx + dy * dy;
    }
    double t2[2] = {tq, ww};
    block_sums(t2, red);
    tq = t2[0];
    ww = t2[1];
    const double om = ww > 0.0 ? tq / ww : 0.0;
#pragma unroll 1
    for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
      const double dx = a.y[i] - cx, dy = a.y[N + i] - cy;
      const float px = (float)((double)a.x[i] - tx + om * dy);
      const float py = (float)((double)a.x[N + i] - ty - om * dx);
      const float pz = a.x[2 * N + i];
      a.x[i] = px;
      a.x[N + i] = py;
      mx = fmax(fmax(mx, fabs((double)px)), fmax(fabs((double)py), fabs((double)pz)));
      rx += (double)a.rn[i] * px + (double)a.rn[N + i] * py + (double)a.rn[2 * N + i] * pz;
    }
  }
  mx = block_max(mx, red);
  rx = block_sum(rx, red);
  const bool go = act && mx > 0.0 && rx > 0.0;
  const double sc = mx > a.cap ? a.cap / mx : 1.0;
  const float scf = go ? (float)sc : 0.f;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t q = d * N + i;
      a.yt[q] = a.y[q] + scf * a.x[q];
    }
  if (threadIdx.x == 0) {
    s[9] = sc;
    s[10] = rx;
    s[12] = go ? 1.0 : 0.0;  // line search pending
    s[13] = mx;
    if (act && !go) s[6] = 0.0;  // no descent step: nothing left to gain
  }
}

// Armijo test per pending cell: accept y_t if Pi(y_t) <= Pi(y) - armijo s
// (r_N . x), copying y_t into y; else halve s and form the next trial, giving
// up (no move) once s max|x| < min_move.  With inverted counts, a trial that
// inverts more tetrahedra than y has is rejected as well: the energy density
// grows without bound as J -> 0, but a finite step can jump over that
// barrier to an inverted state of finite energy.
__global__ __launch_bounds__(kThreads) void qs_ls_accept_kernel(LsArgs a) {
  __shared__ double red[kThreads];
  const int c = blockIdx.x;
  double* s = a.st + kQsState * c;
  if (s[12] == 0.0) return;  // uniform over the workgroup
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1], N = a.N;
  const double top = a.plate[2 * c], bot = a.plate[2 * c + 1];
  double phi = 0.0;
  const bool sph = a.ind.R > 0.0;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
    const double z = a.yt[2 * N + i];
    double dt = fmax(z - top, 0.0);
    const double db = fmax(bot - z, 0.0);
    if (sph) dt = sphere_hit(a.ind, c, top, a.yt[i], a.yt[N + i], z).g;
    phi += dt * dt * dt + db * db * db;
  }
  phi = block_sum(phi, red) * (a.k / 3.0);
  const double pit = a.energy_t[c] + phi;
  const double sc = s[9];
  const bool feasible = !(a.ninv_t && a.ninv) || a.ninv_t[c] <= a.ninv[c];
  const bool ok = feasible && pit <= s[8] - a.armijo * sc * s[10];
  const bool give_up = !ok && 0.5 * sc * s[13] < a.min_move;
  if (ok) {
    for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads)
#pragma unroll
      for (int d = 0; d < 3; ++d) a.y[d * N + i] = a.yt[d * N + i];
  } else {
    const float scf = give_up ? 0.f : (float)(0.5 * sc);
    for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int64_t q = d * N + i;
        a.yt[q] = a.y[q] + scf * a.x[q];
      }
  }
  if (threadIdx.x == 0) {
    if (ok) {
      if (a.ninv_t && a.ninv) a.ninv[c] = a.ninv_t[c];
      s[8] = pit;
      s[4] = sc;
      s[6] = sc * s[13];  // largest node move of this step
      s[12] = 0.0;
    } else if (give_up) {
      s[6] = 0.0;
      s[12] = 0.0;
    } else {
      s[9] = 0.5 * sc;
    }
  }
}

struct PredArgs {
  const int64_t* node_off;
  int64_t N;
  const double* plate_old;
  const double* plate_new;
  float* y;
};

// Predictor for a new plate position: z -> b' + (z - b) s with s = (t' - b')
// / (t - b), and x, y stretched by 1/sqrt(s) about the cell's centroid, an
// affine map of unit determinant (cells are nearly incompressible: a z-only
// compression would start Newton from a large volumetric stress).
__global__ __launch_bounds__(kThreads) void qs_predict_kernel(PredArgs a) {
  __shared__ double red[kThreads];
  const int c = blockIdx.x;
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1], N = a.N;
  const double t0 = a.plate_old[2 * c], b0 = a.plate_old[2 * c + 1];
  const double t1 = a.plate_new[2 * c], b1 = a.plate_new[2 * c + 1];
  const double sc = (t1 - b1) / (t0 - b0);
  const double lat = sc > 0.0 ? 1.0 / sqrt(sc) : 1.0;
  double sx = 0.0, sy = 0.0;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
    sx += a.y[i];
    sy += a.y[N + i];
  }
  const double inv_n = 1.0 / (double)(n1 - n0);
  const double cx = block_sum(sx, red) * inv_n, cy = block_sum(sy, red) * inv_n;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kThreads) {
    a.y[i] = (float)(cx + ((double)a.y[i] - cx) * lat);
    a.y[N + i] = (float)(cy + ((double)a.y[N + i] - cy) * lat);
    a.y[2 * N + i] = (float)(b1 + ((double)a.y[2 * N + i] - b0) * sc);
  }
}

}  // namespace

hipError_t launch_qs_residual(const int64_t* node_off, int64_t N, int32_t n_cells,
                              const float* y, const float* f, const double* energy,
                              const double* plate, double k, double abs_tol,
                              double rel_tol, double step_tol, double floor_factor,
                              double eta_max, int restart, float* r, float* p,
                              float* x, float* rn, double* st, double* force,
                              const float* kel, float* minv, hipStream_t s,
                              const Indenter& ind) {
  ResArgs a{node_off, N, y, f, energy, plate, k, abs_tol, rel_tol, step_tol,
            floor_factor, eta_max, restart, r, p, x, rn, st, force, kel, minv, ind};
  hipLaunchKernelGGL(qs_residual_kernel, dim3(n_cells), dim3(kResThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_qs_adjoint_rhs(const int64_t* node_off, int64_t N, int32_t n_cells,
                                 const float* y, const double* plate, double k,
                                 const double* weight, float* r, float* p, float* x,
                                 double* st, const float* minv, hipStream_t s,
                                 const Indenter& ind) {
  AdjArgs a{node_off, N, y, plate, k, weight, r, p, x, st, minv, ind};
  hipLaunchKernelGGL(qs_adjoint_rhs_kernel, dim3(n_cells), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_qs_cg(const int64_t* node_off, int64_t N, int32_t n_cells,
                        const float* y, const double* plate, double k,
                        double rel_tol, const float* ybar, float* x, float* r,
                        float* p, float* Ap, double* st, const float* minv,
                        hipStream_t s, const DeviceTables* slots, const Indenter& ind) {
  CgArgs a{node_off, N, y, plate, k, rel_tol, ybar, x, r, p, Ap, st, minv,
           slots ? slots->part : nullptr,
           slots ? slots->shared_slot_ptr : nullptr,
           slots ? slots->shared_slots : nullptr,
           slots ? slots->cell_shared_off : nullptr,
           slots ? slots->cell_shared_first : nullptr, ind};
  if (ind.R > 0.0)
    hipLaunchKernelGGL(qs_cg_kernel<true>, dim3(n_cells), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(qs_cg_kernel<false>, dim3(n_cells), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_qs_stiffness(const DeviceTables& T, const Range& r, float* kel,
                               hipStream_t s) {
  if (T.n_tiles <= 0) return hipSuccess;
  for (int pass = 0; pass < 2; ++pass) {
    float* out = kel + (int64_t)pass * 3 * T.n_nodes;
    StiffArgs a{T, pass, out};
    hipLaunchKernelGGL(qs_stiffness_kernel, dim3((unsigned)T.n_tiles), dim3(64),
                       (size_t)16 * T.nloc, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_forward_finalize(T, r, out, nullptr, nullptr, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_qs_update(const int64_t* node_off, int64_t N, int32_t n_cells,
                            const float* x, double cap, float* y, double* st,
                            hipStream_t s) {
  UpdArgs a{node_off, N, x, cap, y, st};
  hipLaunchKernelGGL(qs_update_kernel, dim3(n_cells), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_qs_noise(const int64_t* node_off, int64_t N, int32_t n_cells,
                           const float* y, float* e, hipStream_t s) {
  hipLaunchKernelGGL(qs_noise_kernel, dim3(n_cells), dim3(kThreads), 0, s, node_off, N,
                     y, e);
  return hipGetLastError();
}

hipError_t launch_qs_floor(const int64_t* node_off, int64_t N, int32_t n_cells,
                           const float* y, const double* plate, double k,
                           const float* e, const float* ybar, double* st,
                           hipStream_t s, const Indenter& ind) {
  FloorArgs a{node_off, N, y, plate, k, e, ybar, st, ind};
  hipLaunchKernelGGL(qs_floor_kernel, dim3(n_cells), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_qs_ls_start(const int64_t* node_off, int64_t N, int32_t n_cells,
                              float* x, const float* rn, double cap,
                              const float* y, float* yt, double* st, hipStream_t s) {
  LsArgs a{node_off, N, x, rn, nullptr, nullptr, 0.0, cap, 0.0, 0.0,
           const_cast<float*>(y), yt, st, nullptr, nullptr};
  hipLaunchKernelGGL(qs_ls_start_kernel, dim3(n_cells), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_qs_ls_accept(const int64_t* node_off, int64_t N, int32_t n_cells,
                               const float* x, const double* plate, double k,
                               const double* energy_t, double armijo,
                               double min_move, float* y, float* yt, double* st,
                               const int32_t* ninv_t, int32_t* ninv, hipStream_t s,
                               const Indenter& ind) {
  // the accept kernel only reads x
  LsArgs a{node_off, N, const_cast<float*>(x), nullptr, plate, energy_t, k, 0.0, armijo,
           min_move, y, yt, st, ninv_t, ninv, ind};
  hipLaunchKernelGGL(qs_ls_accept_kernel, dim3(n_cells), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_qs_predict(const int64_t* node_off, int64_t N, int32_t n_cells,
                             const double* plate_old, const double* plate_new,
                             float* y, hipStream_t s) {
  PredArgs a{node_off, N, plate_old, plate_new, y};
  hipLaunchKernelGGL(qs_predict_kernel, dim3(n_cells), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace cm
