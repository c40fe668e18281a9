// Cell-shape diagnostics for gfx950: the Taylor deformation parameter from
// the discretised inertia tensor (Sec. "Taylor deformation parameter", eqs.
// inertia-tensor-discretized, inertia-tensor-ellipsoid-semiaxes and
// taylor-deformation-parameter-definition) and the cell strain (eq.
// cell-strain).
//
//   shape_moments_kernel  one wavefront per tile: the current signed volume
//                         V of every tetrahedron and its centroid r, summed
//                         as V, V r and V r r^T (float64) about a per-cell
//                         origin (the cell's first node), one record per tile,
//                         and the tile's count of tetrahedra with V not > 0;
//   shape_extreme_kernel  per cell, the nodes extreme along the three axes and
//                         the four body diagonals; the largest distance among
//                         these pairs is a lower bound L of d_max (the
//                         distance of two actual nodes) and starts the maximum;
//                         and the cell's count of inverted tetrahedra;
//   shape_bbox_kernel     the bounding box of every candidate block of 256
//                         nodes (below), the nodes of a cell taken candidates
//                         first, each part in Morton order of the reference
//                         positions;
//   pair_max_kernel       the largest squared distance between two candidate
//                         nodes of a cell, over 256 x 256 blocks of node pairs
//                         (float64 differences of the float32 positions are
//                         exact; the maximum of non-negative doubles is an
//                         order-free integer maximum of their bit patterns); a
//                         block pair whose bounding boxes are closer than the
//                         current maximum cannot hold a larger distance and is
//                         skipped (the result is the same, only the work
//                         changes).  The farthest two nodes are convex-hull
//                         vertices, and a node whose faces are all shared by
//                         two tetrahedra on opposite sides lies inside the
//                         image of its star while those keep their orientation
//                         (their solid angles at the node sum to a positive
//                         multiple of 4 pi, so no direction has the node
//                         strictly beyond all its neighbours): the other nodes
//                         are the candidates;
//   pair_all_kernel       cells with an inverted tetrahedron: all node pairs;
//   shape_finalize_kernel per cell (one wavefront): tile records summed in a
//                         fixed order, the inertia tensor about the centre of
//                         mass, its eigenvalues by cyclic Jacobi rotations,
//                         semi-axes, D, d_max and the strain.
// Readings: the tensor is taken about the centre of mass; V is the current
// volume with the reference orientation (negative when inverted); the
// paper's semi-axis formula gives squared semi-axes of a solid ellipsoid, so
// a_i is its square root (0 for a negative radicand); d_ref is the caller's.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_util.h"
#include "aux_kernels.h"

namespace cm {
namespace {

constexpr int kMom = 10;  // V, V r (3), V r r^T (xx yy zz xy xz yz)

struct MomArgs {
  DeviceTables T;
  const int64_t* node_off;
  const float* y;
  double* mom;        // kMom per tile
  int32_t* tile_inv;  // per tile: tetrahedra whose current volume is not > 0
  const uint64_t* chunk_neg;  // per chunk: lanes of negative reference orientation
};

__global__ __launch_bounds__(64) void shape_moments_kernel(MomArgs a) {
  extern __shared__ float4 ys[];
  const int lane = threadIdx.x;
  const int t = blockIdx.x;
  const TileDesc d = a.T.tiles[t];
  const int64_t N = a.T.n_nodes;
  const int64_t o = a.node_off[d.cell];
  const double ox = a.y[o], oy = a.y[N + o], oz = a.y[2 * N + o];
  for (int l = lane; l < d.n_own + d.n_shr; l += 64) {
    const int64_t g = l < d.n_own ? (int64_t)d.own_begin + l
                                  : (int64_t)a.T.slot_node[d.shr_begin + l - d.n_own];
    ys[l] = make_float4(a.y[g], a.y[N + g], a.y[2 * N + g], 0.f);
  }
  wave_sync();
  double m[kMom];
#pragma unroll
  for (int j = 0; j < kMom; ++j) m[j] = 0.0;
  int ninv = 0;
  const TetChunk* ch = a.T.chunks + d.chunk_begin;
  for (int k = 0; k < d.n_chunks; ++k) {
    const uint2 q = make_uint2(ch[k].a[lane][0], ch[k].a[lane][1]);
    const uint64_t neg = a.chunk_neg[d.chunk_begin + k];  // wave-uniform
    if (q.x == kEmptyLane) continue;
    const float4 p[4] = {ys[q.x & 0xffff], ys[q.x >> 16], ys[q.y & 0xffff],
                         ys[q.y >> 16]};
    double e[3][3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      e[v][0] = (double)p[v].x - (double)p[3].x;
      e[v][1] = (double)p[v].y - (double)p[3].y;
      e[v][2] = (double)p[v].z - (double)p[3].z;
    }
    const double det_s = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                         e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                         e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    // current volume with the orientation of the reference vertex order (the
    // sign of the reference edges' determinant for the stored vertex order)
    const double V = (((neg >> lane) & 1ull) ? -det_s : det_s) * (1.0 / 6.0);
    ninv += V > 0.0 ? 0 : 1;
    const double rx = 0.25 * (((double)p[0].x + (double)p[1].x) +
                              ((double)p[2].x + (double)p[3].x)) - ox;
    const double ry = 0.25 * (((double)p[0].y + (double)p[1].y) +
                              ((double)p[2].y + (double)p[3].y)) - oy;
    const double rz = 0.25 * (((double)p[0].z + (double)p[1].z) +
                              ((double)p[2].z + (double)p[3].z)) - oz;
    m[0] += V;
    m[1] += V * rx; m[2] += V * ry; m[3] += V * rz;
    m[4] += V * rx * rx; m[5] += V * ry * ry; m[6] += V * rz * rz;
    m[7] += V * rx * ry; m[8] += V * rx * rz; m[9] += V * ry * rz;
  }
#pragma unroll
  for (int j = 0; j < kMom; ++j) m[j] = wave_sum(m[j]);
  ninv = wave_sum(ninv);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < kMom; ++j) a.mom[(int64_t)kMom * t + j] = m[j];
    a.tile_inv[t] = ninv;
  }
}

struct PairArgs {
  const int4* blocks;  // (cell, row block, column block, first node block of the cell)
  const int64_t* node_off;
  const int32_t* order;  // per cell, node ids in spatial (Morton) order
  const float* y;
  int64_t N;
  const double* bbox;         // per node block: min x y z, max x y z
  unsigned long long* d2max;  // per cell, bits of a non-negative double
};

struct AllArgs {
  const int64_t* node_off;
  const float* y;
  int64_t N;
  const int32_t* cell_inv;
  unsigned long long* d2max;
};

// Cells with an inverted (or degenerate) tetrahedron, which the candidate
// search does not cover: one workgroup per such cell takes the largest
// squared distance over all its node pairs (other cells return at once).
__global__ __launch_bounds__(256) void pair_all_kernel(AllArgs a) {
  __shared__ double red[4];
  const int c = blockIdx.x, tid = threadIdx.x;
  if (a.cell_inv[c] == 0) return;  // uniform over the workgroup
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1], N = a.N;
  double best = 0.0;
  for (int64_t p = n0 + tid; p < n1; p += 256) {
    const double xp = a.y[p], yp = a.y[N + p], zp = a.y[2 * N + p];
    for (int64_t q = p + 1; q < n1; ++q) {
      const double dx = xp - a.y[q], dy = yp - a.y[N + q], dz = zp - a.y[2 * N + q];
      best = fmax(best, dx * dx + dy * dy + dz * dz);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off));
  if ((tid & 63) == 0) red[tid >> 6] = best;
  __syncthreads();
  if (tid == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(&a.d2max[c], (unsigned long long)__double_as_longlong(m));
  }
}

// Directions of the extreme-node search: the axes and the body diagonals.
__constant__ float kDirs[7][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 1},
                                  {1, 1, -1}, {1, -1, 1}, {-1, 1, 1}};

struct ExtArgs {
  DeviceTables T;
  const int64_t* node_off;
  const float* y;
  int64_t N;
  unsigned long long* d2max;
  const int32_t* tile_inv;
  int32_t* cell_inv;  // per cell: tetrahedra whose current volume is not > 0
};

// Per cell: for every direction the node of smallest and of largest
// projection (ties to the smaller index), then d2max = the largest squared
// distance among those pairs; and the cell's count of tetrahedra that are
// inverted (or degenerate) in the current positions.  One pass over the
// nodes: every thread keeps the 14 extremes of its nodes (a largest
// projection as the smallest negated one), then a (value, index)
// lexicographic minimum over the wavefront (butterfly) and the 4 wavefronts.
__global__ __launch_bounds__(256) void shape_extreme_kernel(ExtArgs a) {
  __shared__ double wv[4][14];
  __shared__ int wi[4][14];
  __shared__ int inv[4];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t n0 = a.node_off[c], n1 = a.node_off[c + 1], N = a.N;
  {
    int s = 0;
    const int t0 = a.T.cell_tile_first[c], nt = a.T.cell_tile_count[c];
    for (int k = tid; k < nt; k += 256) s += a.tile_inv[t0 + (int64_t)k * a.T.tile_stride];
    s = wave_sum(s);
    if (lane == 0) inv[w] = s;
  }
  double best[14];
  int arg[14];
#pragma unroll
  for (int k = 0; k < 14; ++k) {
    best[k] = INFINITY;
    arg[k] = -1;
  }
  for (int64_t i = n0 + tid; i < n1; i += 256) {
    const double px = a.y[i], py = a.y[N + i], pz = a.y[2 * N + i];
    const int li = (int)(i - n0);
#pragma unroll
    for (int d = 0; d < 7; ++d) {
      const double pr = (double)kDirs[d][0] * px + (double)kDirs[d][1] * py +
                        (double)kDirs[d][2] * pz;
      // indices grow along a thread's nodes: strict < keeps the smaller one
      if (pr < best[2 * d]) { best[2 * d] = pr; arg[2 * d] = li; }
      if (-pr < best[2 * d + 1]) { best[2 * d + 1] = -pr; arg[2 * d + 1] = li; }
    }
  }
#pragma unroll
  for (int k = 0; k < 14; ++k) {
    double v = best[k];
    int ix = arg[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double v2 = __shfl_xor(v, off);
      const int i2 = __shfl_xor(ix, off);
      if (i2 >= 0 && (ix < 0 || v2 < v || (v2 == v && i2 < ix))) { v = v2; ix = i2; }
    }
    if (lane == 0) { wv[w][k] = v; wi[w][k] = ix; }
  }
  __syncthreads();
  if (tid == 0) {
    a.cell_inv[c] = inv[0] + inv[1] + inv[2] + inv[3];
    int ext[14];
    for (int k = 0; k < 14; ++k) {
      double v = wv[0][k];
      int ix = wi[0][k];
      for (int q = 1; q < 4; ++q) {
        const double v2 = wv[q][k];
        const int i2 = wi[q][k];
        if (i2 >= 0 && (ix < 0 || v2 < v || (v2 == v && i2 < ix))) { v = v2; ix = i2; }
      }
      ext[k] = ix;
    }
    double m = 0.0;
    for (int d = 0; d < 7; ++d) {
      if (ext[2 * d] < 0 || ext[2 * d + 1] < 0) continue;
      const int64_t p = n0 + ext[2 * d], q = n0 + ext[2 * d + 1];
      const double dx = (double)a.y[p] - a.y[q], dy = (double)a.y[N + p] - a.y[N + q],
                   dz = (double)a.y[2 * N + p] - a.y[2 * N + q];
      m = fmax(m, dx * dx + dy * dy + dz * dz);
    }
    a.d2max[c] = (unsigned long long)__double_as_longlong(m);
  }
}

struct BoxArgs {
  const int2* node_blocks;  // (cell, block of the cell)
  const int64_t* node_off;
  const int32_t* order;
  const float* y;
  int64_t N;
  double* bbox;
};

__global__ __launch_bounds__(256) void shape_bbox_kernel(BoxArgs a) {
  __shared__ double red[6][4];
  const int2 nb = a.node_blocks[blockIdx.x];
  const int64_t n1 = a.node_off[nb.x + 1];
  const int64_t i = a.node_off[nb.x] + (int64_t)nb.y * 256 + threadIdx.x;
  const bool in = i < n1;
  const int64_t g = in ? (int64_t)a.order[i] : 0;
  double v[6];
  for (int d = 0; d < 3; ++d) {
    const double q = in ? (double)a.y[d * a.N + g] : 0.0;
    v[d] = in ? q : INFINITY;
    v[3 + d] = in ? q : -INFINITY;
  }
  for (int off = 32; off > 0; off >>= 1)
    for (int d = 0; d < 3; ++d) {
      v[d] = fmin(v[d], __shfl_xor(v[d], off));
      v[3 + d] = fmax(v[3 + d], __shfl_xor(v[3 + d], off));
    }
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    const double r = k < 3 ? fmin(fmin(red[k][0], red[k][1]), fmin(red[k][2], red[k][3]))
                           : fmax(fmax(red[k][0], red[k][1]), fmax(red[k][2], red[k][3]));
    a.bbox[6 * (int64_t)blockIdx.x + k] = r;
  }
}

__global__ __launch_bounds__(256) void pair_max_kernel(PairArgs a) {
  __shared__ double cx[256], cy[256], cz[256];
  __shared__ double red[4];
  __shared__ int skip;
  __shared__ double cur_d2;
  const int4 b = a.blocks[blockIdx.x];
  const int tid = threadIdx.x;
  if (tid == 0) {
    // farthest points of the two bounding boxes vs the current maximum
    const double* r = a.bbox + 6 * (int64_t)(b.w + b.y);
    const double* q = a.bbox + 6 * (int64_t)(b.w + b.z);
    double u = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double e = fmax(r[3 + d] - q[d], q[3 + d] - r[d]);
      u += e * e;
    }
    const unsigned long long cur = __hip_atomic_load(&a.d2max[b.x], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
    cur_d2 = __longlong_as_double((long long)cur);
    // (with a relative margin far above the rounding of the two sums)
    skip = u < cur_d2 * (1.0 - 1e-12);
  }
  __syncthreads();
  if (skip) return;  // uniform over the workgroup
  const int64_t n0 = a.node_off[b.x], n1 = a.node_off[b.x + 1];
  const int64_t j0 = n0 + (int64_t)b.z * 256;
  const int ncol = n1 - j0 < 256 ? (int)(n1 - j0) : 256;
  if (tid < ncol) {
    const int64_t g = a.order[j0 + tid];
    cx[tid] = a.y[g];
    cy[tid] = a.y[a.N + g];
    cz[tid] = a.y[2 * a.N + g];
  }
  __syncthreads();
  const int64_t i = n0 + (int64_t)b.y * 256 + tid;
  double best = 0.0;
  if (i < n1) {
    const int64_t g = a.order[i];
    const double xi = a.y[g], yi = a.y[a.N + g], zi = a.y[2 * a.N + g];
    // the column block's box cannot hold a node farther from this one than
    // the current maximum: nothing to find for this row
    const double* q = a.bbox + 6 * (int64_t)(b.w + b.z);
    const double ex = fmax(xi - q[0], q[3] - xi), ey = fmax(yi - q[1], q[4] - yi),
                 ez = fmax(zi - q[2], q[5] - zi);
    const int ncheck = ex * ex + ey * ey + ez * ez < cur_d2 * (1.0 - 1e-12) ? 0 : ncol;
    for (int k = 0; k < ncheck; ++k) {
      const double dx = xi - cx[k], dy = yi - cy[k], dz = zi - cz[k];
      best = fmax(best, dx * dx + dy * dy + dz * dz);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off));
  if ((tid & 63) == 0) red[tid >> 6] = best;
  __syncthreads();
  if (tid == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(&a.d2max[b.x], (unsigned long long)__double_as_longlong(m));
  }
}

// Eigenvalues of a symmetric 3x3 matrix (A00 A11 A22 A01 A02 A12) by cyclic
// Jacobi rotations; at most 32 sweeps (convergence is quadratic).
__device__ void sym3_eigenvalues(const double s[6], double ev[3]) {
  double A[3][3] = {{s[0], s[3], s[4]}, {s[3], s[1], s[5]}, {s[4], s[5], s[2]}};
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-32 * dia || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + tt * tt), sn = tt * c;
        for (int k = 0; k < 3; ++k) {  // A <- A G (columns p, q)
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  // A <- G^T A (rows p, q)
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        A[p][q] = A[q][p] = 0.0;
      }
  }
  ev[0] = A[0][0]; ev[1] = A[1][1]; ev[2] = A[2][2];
}

struct ShapeFinArgs {
  DeviceTables T;
  const int64_t* node_off;
  const float* y;
  const double* mom;
  const unsigned long long* d2max;
  const double* d_ref;  // nullable
  double* out;          // kShapeFields per cell
};

// One wavefront per cell: lane l sums the tile records l, l + 64, ...,
// then a fixed butterfly; lane 0 finishes the cell.
__global__ __launch_bounds__(256) void shape_finalize_kernel(ShapeFinArgs a) {
  const int c = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= a.T.n_cells) return;  // uniform per wavefront
  double m[kMom];
#pragma unroll
  for (int j = 0; j < kMom; ++j) m[j] = 0.0;
  const int t0 = a.T.cell_tile_first[c], nt = a.T.cell_tile_count[c];
  for (int k = lane; k < nt; k += 64) {
    const int64_t t = t0 + (int64_t)k * a.T.tile_stride;
#pragma unroll
    for (int j = 0; j < kMom; ++j) m[j] += a.mom[kMom * t + j];
  }
#pragma unroll
  for (int j = 0; j < kMom; ++j) m[j] = wave_sum(m[j]);
  if (lane != 0) return;
  const int64_t N = a.T.n_nodes, o = a.node_off[c];
  const double M = m[0];
  const double cx = m[1] / M, cy = m[2] / M, cz = m[3] / M;
  // second moments about the centre of mass, then the inertia tensor
  const double Sxx = m[4] - m[1] * cx, Syy = m[5] - m[2] * cy, Szz = m[6] - m[3] * cz;
  const double Sxy = m[7] - m[1] * cy, Sxz = m[8] - m[1] * cz, Syz = m[9] - m[2] * cz;
  const double tr = Sxx + Syy + Szz;
  const double I[6] = {tr - Sxx, tr - Syy, tr - Szz, -Sxy, -Sxz, -Syz};
  double th[3];
  sym3_eigenvalues(I, th);
  // theta_1 >= theta_2 >= theta_3
  if (th[0] < th[1]) { const double s = th[0]; th[0] = th[1]; th[1] = s; }
  if (th[1] < th[2]) { const double s = th[1]; th[1] = th[2]; th[2] = s; }
  if (th[0] < th[1]) { const double s = th[0]; th[0] = th[1]; th[1] = s; }
  const double f = 5.0 / (2.0 * M);
  const double a1 = sqrt(fmax(f * (-th[0] + th[1] + th[2]), 0.0));
  const double a2 = sqrt(fmax(f * (th[0] - th[1] + th[2]), 0.0));
  const double a3 = sqrt(fmax(f * (th[0] + th[1] - th[2]), 0.0));
  const double dmax = sqrt(__longlong_as_double((long long)a.d2max[c]));
  double* r = a.out + (int64_t)kShapeFields * c;
  r[0] = M;
  r[1] = (double)a.y[o] + cx;
  r[2] = (double)a.y[N + o] + cy;
  r[3] = (double)a.y[2 * N + o] + cz;
  r[4] = a1; r[5] = a2; r[6] = a3;
  r[7] = (a3 - a1) / (a3 + a1);
  r[8] = dmax;
  r[9] = a.d_ref ? (dmax - a.d_ref[c]) / a.d_ref[c] : __builtin_nan("");
}

}  // namespace

size_t shape_lds(int nloc) { return (size_t)16 * nloc; }

hipError_t launch_shape(const DeviceTables& T, const int64_t* node_off,
                        const int4* cand_blocks, int64_t n_cand_blocks,
                        const int2* node_blocks, int64_t n_node_blocks,
                        const int32_t* order, const float* y, const double* d_ref,
                        const uint64_t* chunk_neg, double* mom, int32_t* tile_inv,
                        int32_t* cell_inv,
                        double* bbox, unsigned long long* d2max, double* out,
                        hipStream_t st) {
  const int nc = T.n_cells;
  hipError_t e;
  if (T.n_tiles > 0) {
    MomArgs m{T, node_off, y, mom, tile_inv, chunk_neg};
    hipLaunchKernelGGL(shape_moments_kernel, dim3((unsigned)T.n_tiles), dim3(64),
                       shape_lds(T.nloc), st, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  ExtArgs x{T, node_off, y, T.n_nodes, d2max, tile_inv, cell_inv};
  hipLaunchKernelGGL(shape_extreme_kernel, dim3(nc), dim3(256), 0, st, x);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (n_node_blocks > 0) {
    BoxArgs bx{node_blocks, node_off, order, y, T.n_nodes, bbox};
    hipLaunchKernelGGL(shape_bbox_kernel, dim3((unsigned)n_node_blocks), dim3(256), 0,
                       st, bx);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (n_cand_blocks > 0) {
    PairArgs p{cand_blocks, node_off, order, y, T.n_nodes, bbox, d2max};
    hipLaunchKernelGGL(pair_max_kernel, dim3((unsigned)n_cand_blocks), dim3(256), 0,
                       st, p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  AllArgs al{node_off, y, T.n_nodes, cell_inv, d2max};
  hipLaunchKernelGGL(pair_all_kernel, dim3(nc), dim3(256), 0, st, al);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  ShapeFinArgs f{T, node_off, y, mom, d2max, d_ref, out};
  hipLaunchKernelGGL(shape_finalize_kernel, dim3((nc + 3) / 4), dim3(256), 0, st, f);
  return hipGetLastError();
}

}  // namespace cm
