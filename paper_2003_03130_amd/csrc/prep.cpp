// Host preparation of tetrahedral cells: validation, the FP64 reference
// precompute (B = J^-1 and V0, computed once as the paper prescribes in the
// paragraph defining the Jacobian J_ik = x_i^k - x_i^4), locality ordering,
// tiling and the owned/shared node tables described in layout.h.
#include "prep.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "cellmech.h"

namespace cm {
namespace {

struct CellOut {
  int status = CM_OK;
  std::string err;
  std::vector<TileDesc> tiles;       // chunk_begin, own_begin, shr_begin local
  std::vector<TetChunk> chunks;
  std::vector<uint64_t> chunk_neg;   // per chunk: lanes whose reference
                                     // orientation (det of the edges) is < 0
  std::vector<int32_t> slot_node;    // local internal ids
  std::vector<int32_t> shared_node;  // local internal ids
  std::vector<int32_t> shared_slot_ptr;
  std::vector<int32_t> shared_slots;  // local slot ids
  std::vector<int64_t> new_to_old;    // local
  std::vector<int32_t> space_order;   // local internal ids: candidates of the
                                      // largest node distance first, each part
                                      // in Morton order of the node
  int32_t n_candidates = 0;           // leading entries of space_order
  std::vector<int32_t> tile_region;   // region of every tile
  std::vector<int32_t> region_tile_first, region_tile_count;  // local tiles
  int32_t max_tile_nodes = 0;
  double volume = 0.0, min_v0 = INFINITY, max_cond = 0.0;
};

// Spread the low 10 bits of v so that bit b lands on bit 3b.
inline uint32_t spread3(uint32_t v) {
  v &= 0x3ff;
  v = (v | (v << 16)) & 0x030000ff;
  v = (v | (v << 8)) & 0x0300f00f;
  v = (v | (v << 4)) & 0x030c30c3;
  v = (v | (v << 2)) & 0x09249249;
  return v;
}

// Reference centroids of the tetrahedra (xyz per tet).
void centroids(int64_t m, const int32_t* T, const double* X, std::vector<double>& cen) {
  cen.resize(3 * m);
  for (int64_t t = 0; t < m; ++t)
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
      for (int a = 0; a < 4; ++a) s += X[3 * (int64_t)T[4 * t + a] + i];
      cen[3 * t + i] = 0.25 * s;
    }
}

// Recursive inertial bisection state of one cell.
struct Bisector {
  const int32_t* T;
  const std::vector<double>& cen;     // reference centroids
  const std::vector<int64_t>& rank;   // locality (Morton) rank of every tet
  int64_t tt;                         // tets per tile
  int64_t node_cap;                   // most distinct nodes per tile
  std::vector<int64_t>& perm;
  std::vector<int64_t> ends;          // tile ends (positions in perm)
  std::vector<int32_t> stamp;         // per node: last leaf that counted it
  int32_t gen = 0;

  // Sorts perm[a, b) along the principal axis of the centroids (power
  // iteration on their covariance; ties by rank, so deterministic).
  void sort_principal(int64_t a, int64_t b) {
    const int64_t n = b - a;
    double mu[3] = {0, 0, 0}, cv[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int64_t q = a; q < b; ++q)
      for (int i = 0; i < 3; ++i) mu[i] += cen[3 * perm[q] + i];
    for (int i = 0; i < 3; ++i) mu[i] /= (double)n;
    for (int64_t q = a; q < b; ++q) {
      double d[3];
      for (int i = 0; i < 3; ++i) d[i] = cen[3 * perm[q] + i] - mu[i];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) cv[i][j] += d[i] * d[j];
    }
    double v[3] = {0.6, 0.5, 0.4};
    for (int it = 0; it < 40; ++it) {
      double w[3] = {0, 0, 0};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) w[i] += cv[i][j] * v[j];
      const double nw = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
      if (!(nw > 0)) break;
      for (int i = 0; i < 3; ++i) v[i] = w[i] / nw;
    }
    std::vector<std::pair<double, int64_t>> key(n);
    for (int64_t q = 0; q < n; ++q) {
      const double* c = &cen[3 * perm[a + q]];
      key[q] = {c[0] * v[0] + c[1] * v[1] + c[2] * v[2], rank[perm[a + q]]};
    }
    std::vector<int64_t> idx(perm.begin() + a, perm.begin() + b), ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return key[x] < key[y]; });
    for (int64_t q = 0; q < n; ++q) perm[a + q] = idx[ord[q]];
  }

  int64_t distinct_nodes(int64_t a, int64_t b) {
    ++gen;
    int64_t cnt = 0;
    for (int64_t q = a; q < b; ++q)
      for (int k = 0; k < 4; ++k) {
        const int32_t v = T[4 * perm[q] + k];
        if (stamp[v] != gen) { stamp[v] = gen; ++cnt; }
      }
    return cnt;
  }

  // perm[a, b) into tiles: whole tiles of tt tets (the last one ragged) by
  // halving along the principal axis, the first part taking floor(k/2)
  // tiles; a tile touching more than node_cap nodes (thin or boundary-heavy
  // parts) is halved again.  Tets keep their locality order inside a tile.
  void split(int64_t a, int64_t b) {
    const int64_t n = b - a;
    const int64_t k = (n + tt - 1) / tt;
    if (k <= 1 && (n <= kChunk || distinct_nodes(a, b) <= node_cap)) {
      std::sort(perm.begin() + a, perm.begin() + b,
                [&](int64_t x, int64_t y) { return rank[x] < rank[y]; });
      ends.push_back(b);
      return;
    }
    sort_principal(a, b);
    const int64_t mid = k > 1 ? a + (k / 2) * tt : a + n / 2;
    split(a, mid);
    split(mid, b);
  }
};

// Tet order by the Morton (Z-order) code of the reference centroid.
void morton_order(int64_t m, const int32_t* T, const double* X,
                  std::vector<int64_t>& perm) {
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  std::vector<double> cen(3 * m);
  for (int64_t t = 0; t < m; ++t)
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
      for (int a = 0; a < 4; ++a) s += X[3 * (int64_t)T[4 * t + a] + i];
      cen[3 * t + i] = 0.25 * s;
      lo[i] = std::min(lo[i], cen[3 * t + i]);
      hi[i] = std::max(hi[i], cen[3 * t + i]);
    }
  std::vector<uint32_t> code(m);
  for (int64_t t = 0; t < m; ++t) {
    uint32_t c = 0;
    for (int i = 0; i < 3; ++i) {
      double span = hi[i] - lo[i];
      double q = span > 0 ? (cen[3 * t + i] - lo[i]) / span : 0.0;
      uint32_t qi = (uint32_t)std::min(1023.0, std::max(0.0, std::floor(q * 1024.0)));
      c |= spread3(qi) << i;
    }
    code[t] = c;
  }
  perm.resize(m);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int64_t a, int64_t b) { return code[a] < code[b]; });
}

// Tet order by the smallest reverse Cuthill-McKee label of its vertices.
void rcm_order(int64_t n, int64_t m, const int32_t* T,
               std::vector<int64_t>& perm) {
  static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  std::vector<std::pair<int32_t, int32_t>> edges;
  edges.reserve(12 * m);
  for (int64_t t = 0; t < m; ++t)
    for (auto& e : E) {
      int32_t a = T[4 * t + e[0]], b = T[4 * t + e[1]];
      edges.emplace_back(a, b);
      edges.emplace_back(b, a);
    }
  std::sort(edges.begin(), edges.end());
  edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
  std::vector<int64_t> ptr(n + 1, 0);
  for (auto& e : edges) ptr[e.first + 1]++;
  for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  std::vector<int32_t> adj(edges.size());
  for (size_t q = 0; q < edges.size(); ++q) adj[q] = edges[q].second;
  auto deg = [&](int32_t v) { return ptr[v + 1] - ptr[v]; };

  std::vector<int32_t> label(n, -1), order;
  order.reserve(n);
  std::vector<int32_t> level(n, -1);
  auto bfs_last = [&](int32_t s, std::vector<int32_t>& seen) {
    // returns a minimum-degree vertex of the last BFS level from s
    std::vector<int32_t> cur{s}, nxt, last{s};
    seen[s] = s;
    while (!cur.empty()) {
      last = cur;
      nxt.clear();
      for (int32_t v : cur)
        for (int64_t q = ptr[v]; q < ptr[v + 1]; ++q)
          if (seen[adj[q]] != s) { seen[adj[q]] = s; nxt.push_back(adj[q]); }
      cur.swap(nxt);
    }
    return *std::min_element(last.begin(), last.end(), [&](int32_t a, int32_t b) {
      return deg(a) < deg(b) || (deg(a) == deg(b) && a < b);
    });
  };
  std::vector<int32_t> seen(n, -1);
  for (int32_t start = 0; start < n; ++start) {
    if (label[start] >= 0) continue;
    // pseudo-peripheral start vertex of this component
    int32_t s = start;
    for (int it = 0; it < 2; ++it) s = bfs_last(s, seen);
    size_t head = order.size();
    order.push_back(s);
    label[s] = 0;
    std::vector<int32_t> nb;
    while (head < order.size()) {
      int32_t v = order[head++];
      nb.clear();
      for (int64_t q = ptr[v]; q < ptr[v + 1]; ++q)
        if (label[adj[q]] < 0) { label[adj[q]] = 0; nb.push_back(adj[q]); }
      std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
        return deg(a) < deg(b) || (deg(a) == deg(b) && a < b);
      });
      for (int32_t u : nb) order.push_back(u);
    }
  }
  for (int64_t k = 0; k < n; ++k) label[order[k]] = (int32_t)(n - 1 - k);
  std::vector<int32_t> key(m);
  for (int64_t t = 0; t < m; ++t) {
    int32_t k = label[T[4 * t]];
    for (int a = 1; a < 4; ++a) k = std::min(k, label[T[4 * t + a]]);
    key[t] = k;
  }
  perm.resize(m);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int64_t a, int64_t b) { return key[a] < key[b]; });
}

// FP64 reference data of one tetrahedron with vertices v[0..3] (v[3] is the
// local origin): J_ik = x_i^(v_k) - x_i^(v_3), B = J^-1 (row-major, B[k][j]),
// returns det J.  Also the 1-norm condition number of J.
double reference_inverse(const double* X, const int32_t v[4], double B[9],
                         double* cond1) {
  double Jm[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) Jm[i][k] = X[3 * (int64_t)v[k] + i] - X[3 * (int64_t)v[3] + i];
  double adj[3][3];
  adj[0][0] = Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1];
  adj[0][1] = Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2];
  adj[0][2] = Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1];
  adj[1][0] = Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2];
  adj[1][1] = Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0];
  adj[1][2] = Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2];
  adj[2][0] = Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0];
  adj[2][1] = Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1];
  adj[2][2] = Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0];
  const double det = Jm[0][0] * adj[0][0] + Jm[0][1] * adj[1][0] + Jm[0][2] * adj[2][0];
  double n1J = 0.0, n1B = 0.0;
  for (int k = 0; k < 3; ++k) {
    double sJ = 0.0, sB = 0.0;
    for (int i = 0; i < 3; ++i) {
      B[3 * k + i] = adj[k][i] / det;
      sJ += std::fabs(Jm[i][k]);
      sB += std::fabs(adj[i][k] / det);
    }
    n1J = std::max(n1J, sJ);
    n1B = std::max(n1B, sB);
  }
  if (cond1) *cond1 = n1J * n1B;
  return det;
}

// The 24 assignments of the 4 vertices of a tetrahedron to the 4 slots.
struct Perms {
  int p[24][4];
  Perms() {
    int k = 0, a[4] = {0, 1, 2, 3};
    do {
      for (int i = 0; i < 4; ++i) p[k][i] = a[i];
      ++k;
    } while (std::next_permutation(a, a + 4));
  }
};
const Perms kPerms;

void prepare_cell(int32_t c, int64_t n, int64_t m, const double* X,
                  const int32_t* T, const uint8_t* region, int32_t n_regions,
                  const PrepOptions& opt, CellOut& out) {
  auto fail = [&](int st, const std::string& msg) {
    out.status = st;
    out.err = "cell " + std::to_string(c) + ": " + msg;
  };
  if (m <= 0) return fail(CM_EINVAL, "has no tetrahedra");
  if (n < 4) return fail(CM_EINVAL, "has fewer than 4 nodes");
  if (n > 0x7fffffffLL || m > 0x7fffffffLL) return fail(CM_EINVAL, "too large");
  for (int64_t t = 0; t < m; ++t) {
    const int32_t* v = T + 4 * t;
    for (int a = 0; a < 4; ++a) {
      if (v[a] < 0 || v[a] >= n)
        return fail(CM_EINVAL, "tetrahedron " + std::to_string(t) +
                                   " has a vertex index out of range");
      for (int b = 0; b < a; ++b)
        if (v[a] == v[b])
          return fail(CM_EINVAL, "tetrahedron " + std::to_string(t) +
                                     " repeats a vertex");
    }
  }
  for (int64_t q = 0; q < 3 * n; ++q)
    if (!std::isfinite(X[q])) return fail(CM_EINVAL, "non-finite reference position");
  if (region)
    for (int64_t t = 0; t < m; ++t)
      if ((int32_t)region[t] >= n_regions)
        return fail(CM_EINVAL, "tetrahedron " + std::to_string(t) +
                                   " has a region id >= n_regions");

  // FP64 precompute: J_ik = x_i^k - x_i^4, B = J^-1, V0 = |det J| / 6
  // (checked and summarised here in the input vertex order; recomputed for
  // the slot order when the chunks are packed).
  std::vector<double> absdet(m);
  double hsum = 0.0;
  static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  for (int64_t t = 0; t < m; ++t) {
    const int32_t* v = T + 4 * t;
    double Bt[9], cond1;
    absdet[t] = std::fabs(reference_inverse(X, v, Bt, &cond1));
    out.max_cond = std::max(out.max_cond, cond1);
    for (auto& e : E) {
      double d2 = 0.0;
      for (int i = 0; i < 3; ++i) {
        double d = X[3 * (int64_t)v[e[0]] + i] - X[3 * (int64_t)v[e[1]] + i];
        d2 += d * d;
      }
      hsum += std::sqrt(d2);
    }
  }
  double h = hsum / (6.0 * (double)m);
  double thr = opt.degenerate_tol * h * h * h;
  for (int64_t t = 0; t < m; ++t) {
    if (!(absdet[t] > thr))
      return fail(CM_EDEGENERATE, "tetrahedron " + std::to_string(t) +
                                      " is degenerate (|det J| = " +
                                      std::to_string(absdet[t]) + ")");
    out.volume += absdet[t] / 6.0;
    out.min_v0 = std::min(out.min_v0, absdet[t] / 6.0);
  }

  // Locality order of the tetrahedra.
  std::vector<int64_t> perm;
  if (opt.order == CM_ORDER_MORTON || opt.order == CM_ORDER_BISECT) {
    morton_order(m, T, X, perm);
  } else if (opt.order == CM_ORDER_RCM) {
    rcm_order(n, m, T, perm);
  } else {
    perm.resize(m);
    std::iota(perm.begin(), perm.end(), 0);
  }

  // Material regions: the tetrahedra of each region are contiguous in the
  // order (stable, so the locality order holds inside a region) and no tile
  // spans two regions, so every tile has one material.
  if (region && n_regions > 1)
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) {
      return region[a] < region[b];
    });
  const int64_t TT = opt.tile_tets;
  std::vector<int64_t> tlo, thi;  // tet range [tlo, thi) of every tile in the order
  out.region_tile_first.assign(n_regions, 0);
  out.region_tile_count.assign(n_regions, 0);
  std::vector<double> cen;
  std::vector<int64_t> rank;
  if (opt.order == CM_ORDER_BISECT) {
    centroids(m, T, X, cen);
    rank.resize(m);
    for (int64_t p = 0; p < m; ++p) rank[perm[p]] = p;
  }
  for (int64_t p = 0; p < m;) {
    const int32_t r = region ? (int32_t)region[perm[p]] : 0;
    int64_t e = p;
    while (e < m && (region ? (int32_t)region[perm[e]] : 0) == r) ++e;
    out.region_tile_first[r] = (int32_t)tlo.size();
    if (opt.order == CM_ORDER_BISECT) {
      // compact tiles by recursive bisection inside the region, Morton
      // order inside every tile; at most 5/12 tile_tets nodes per tile
      Bisector bs{T, cen, rank, TT, std::max<int64_t>(TT * 5 / 12, 4 * kChunk), perm, {},
                  std::vector<int32_t>(n, -1)};
      bs.split(p, e);
      int64_t a = p;
      for (int64_t b : bs.ends) {
        tlo.push_back(a);
        thi.push_back(b);
        out.tile_region.push_back(r);
        a = b;
      }
    } else {
      for (int64_t a = p; a < e; a += TT) {
        tlo.push_back(a);
        thi.push_back(std::min(e, a + TT));
        out.tile_region.push_back(r);
      }
    }
    out.region_tile_count[r] = (int32_t)tlo.size() - out.region_tile_first[r];
    p = e;
  }
  const int64_t n_tiles = (int64_t)tlo.size();
  // Number of distinct tiles touching each node.
  std::vector<int32_t> last(n, -1), ntile(n, 0);
  for (int64_t k = 0; k < n_tiles; ++k)
    for (int64_t p = tlo[k]; p < thi[k]; ++p) {
      const int32_t* v = T + 4 * perm[p];
      for (int a = 0; a < 4; ++a)
        if (last[v[a]] != (int32_t)k) { last[v[a]] = (int32_t)k; ntile[v[a]]++; }
    }
  // Internal numbering: owned nodes tile by tile, then shared nodes in order
  // of first appearance, then nodes no tetrahedron uses.
  std::vector<int32_t> newid(n, -1);
  std::vector<int32_t> own_begin(n_tiles), n_own(n_tiles);
  int32_t next = 0;
  for (int64_t k = 0; k < n_tiles; ++k) {
    own_begin[k] = next;
    for (int64_t p = tlo[k]; p < thi[k]; ++p) {
      const int32_t* v = T + 4 * perm[p];
      for (int a = 0; a < 4; ++a)
        if (ntile[v[a]] == 1 && newid[v[a]] < 0) newid[v[a]] = next++;
    }
    n_own[k] = next - own_begin[k];
  }
  const int32_t n_owned = next;
  for (int64_t p = 0; p < m; ++p) {
    const int32_t* v = T + 4 * perm[p];
    for (int a = 0; a < 4; ++a)
      if (newid[v[a]] < 0) newid[v[a]] = next++;
  }
  for (int64_t v = 0; v < n; ++v)
    if (newid[v] < 0) newid[v] = next++;
  const int32_t n_shared = (int32_t)n - n_owned;

  out.new_to_old.resize(n);
  for (int64_t v = 0; v < n; ++v) out.new_to_old[newid[v]] = v;
  {
    // nodes in Morton order of their reference position (spatially compact
    // blocks of nodes for the shape kernels' pair search)
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t v = 0; v < n; ++v)
      for (int i = 0; i < 3; ++i) {
        lo[i] = std::min(lo[i], X[3 * v + i]);
        hi[i] = std::max(hi[i], X[3 * v + i]);
      }
    std::vector<uint32_t> code(n);
    for (int64_t v = 0; v < n; ++v) {
      uint32_t cd = 0;
      for (int i = 0; i < 3; ++i) {
        const double span = hi[i] - lo[i];
        const double q = span > 0 ? (X[3 * v + i] - lo[i]) / span : 0.0;
        cd |= spread3((uint32_t)std::min(1023.0, std::max(0.0, std::floor(q * 1024.0)))) << i;
      }
      code[newid[v]] = cd;
    }
    // Candidates for the largest node distance: the two nodes of a cell that
    // are farthest apart are vertices of the convex hull of its nodes, and a
    // node whose faces are each shared by exactly two tetrahedra on opposite
    // sides (its link is a closed, consistently oriented surface) lies inside
    // the image of its star while all those tetrahedra keep their
    // orientation, so it is no hull vertex.  The others (on a boundary face,
    // a face of one orientation shared more than once, or in no tetrahedron)
    // come first.
    std::vector<uint8_t> cand(n, 0);
    {
      // per face: sorted vertex triple and its orientation induced by the
      // tetrahedron (the reference orientation of the tetrahedron, the sign
      // of the face in its boundary, and the parity of the sort)
      struct Face { std::array<int32_t, 3> k; int8_t o; };
      std::vector<Face> faces((size_t)4 * m);
      for (int64_t t = 0; t < m; ++t) {
        const int32_t* v = T + 4 * t;
        double e[3][3];
        for (int a = 0; a < 3; ++a)
          for (int i = 0; i < 3; ++i) e[a][i] = X[3 * v[a + 1] + i] - X[3 * v[0] + i];
        const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                           e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                           e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
        const int so = det > 0 ? 1 : -1;
        for (int f = 0; f < 4; ++f) {
          std::array<int32_t, 3> k;
          for (int a = 0, q = 0; a < 4; ++a)
            if (a != f) k[q++] = v[a];
          int par = 1;  // parity of the sort of three entries
          if (k[0] > k[1]) { std::swap(k[0], k[1]); par = -par; }
          if (k[1] > k[2]) { std::swap(k[1], k[2]); par = -par; }
          if (k[0] > k[1]) { std::swap(k[0], k[1]); par = -par; }
          faces[(size_t)4 * t + f] = Face{k, (int8_t)(so * (f % 2 ? -1 : 1) * par)};
        }
      }
      std::sort(faces.begin(), faces.end(),
                [](const Face& a, const Face& b) { return a.k < b.k; });
      std::vector<uint8_t> referenced(n, 0);
      for (int64_t q = 0; q < 4 * m; ++q) referenced[T[q]] = 1;
      for (size_t i = 0; i < faces.size();) {
        size_t j = i + 1;
        while (j < faces.size() && faces[j].k == faces[i].k) ++j;
        if (!(j - i == 2 && faces[i].o != faces[i + 1].o))
          for (int a = 0; a < 3; ++a) cand[faces[i].k[a]] = 1;
        i = j;
      }
      for (int64_t v = 0; v < n; ++v)
        if (!referenced[v]) cand[v] = 1;
    }
    std::vector<uint8_t> cand_new(n);
    for (int64_t v = 0; v < n; ++v) cand_new[newid[v]] = cand[v];
    out.space_order.resize(n);
    std::iota(out.space_order.begin(), out.space_order.end(), 0);
    std::stable_sort(out.space_order.begin(), out.space_order.end(),
                     [&](int32_t a, int32_t b) {
                       if (cand_new[a] != cand_new[b]) return cand_new[a] > cand_new[b];
                       return code[a] < code[b];
                     });
    out.n_candidates = 0;
    for (int64_t v = 0; v < n; ++v) out.n_candidates += cand[v];
  }

  // Tiles, slots and chunks.
  out.tiles.resize(n_tiles);
  std::vector<int32_t> stamp(n, -1), loc(n, 0);
  std::vector<std::vector<uint8_t>> used;  // per chunk: slot mask per tile node
  std::vector<int32_t> cnt;
  struct Placed { int32_t chunk, lane; int32_t v[4]; };
  std::vector<Placed> placed;
  for (int64_t k = 0; k < n_tiles; ++k) {
    const int64_t p0 = tlo[k], p1 = thi[k];
    TileDesc& d = out.tiles[k];
    d.chunk_begin = (int32_t)out.chunks.size();
    d.n_tets = (int32_t)(p1 - p0);
    d.own_begin = own_begin[k];
    d.n_own = n_own[k];
    d.shr_begin = (int32_t)out.slot_node.size();
    d.cell = c;
    int32_t nsh = 0;
    for (int64_t p = p0; p < p1; ++p) {
      const int32_t* v = T + 4 * perm[p];
      for (int a = 0; a < 4; ++a) {
        int32_t u = v[a];
        if (ntile[u] == 1) {
          loc[u] = newid[u] - own_begin[k];
        } else if (stamp[u] != (int32_t)k) {
          stamp[u] = (int32_t)k;
          loc[u] = n_own[k] + nsh++;
          out.slot_node.push_back(newid[u]);
        }
      }
    }
    d.n_shr = nsh;
    // The tile's shared nodes in the order of their internal ids (first
    // appearance over the tiles), local indices following: the slots of
    // consecutive shared nodes then form runs inside every tile, so the
    // finalize reads the partials of neighbouring nodes from the same cache
    // lines.  The chunk assignment below only compares node identities, so
    // it and every sum stay the same.
    std::sort(out.slot_node.begin() + d.shr_begin, out.slot_node.end());
    for (int32_t j = 0; j < nsh; ++j)
      loc[out.new_to_old[out.slot_node[d.shr_begin + j]]] = n_own[k] + j;
    const int32_t nloc = d.n_own + d.n_shr;
    out.max_tile_nodes = std::max(out.max_tile_nodes, nloc);

    // Chunk assignment: tetrahedron p prefers chunk p mod nmin (neighbours
    // in the locality order land in different chunks) and takes the first
    // chunk with a free lane in which some assignment of its vertices to
    // the 4 slots uses nodes not yet used in those slots; if none exists a
    // chunk is added.
    const int nmin = (int)((p1 - p0 + kChunk - 1) / kChunk);
    used.assign(nmin, std::vector<uint8_t>(nloc, 0));
    cnt.assign(nmin, 0);
    placed.clear();
    for (int64_t p = p0; p < p1; ++p) {
      const int32_t* v = T + 4 * perm[p];
      int32_t lv[4];
      for (int a = 0; a < 4; ++a) lv[a] = loc[v[a]];
      const int nc = (int)used.size();
      const int c0 = (int)((p - p0) % nmin);
      int chosen = -1, pi = -1;
      for (int dc = 0; dc < nc && chosen < 0; ++dc) {
        const int ch = (c0 + dc) % nc;
        if (cnt[ch] >= kChunk) continue;
        uint8_t mk[4];
        for (int a = 0; a < 4; ++a) mk[a] = used[ch][lv[a]];
        for (int q = 0; q < 24; ++q) {
          const int* pm = kPerms.p[q];
          if (!((mk[0] >> pm[0]) & 1) && !((mk[1] >> pm[1]) & 1) &&
              !((mk[2] >> pm[2]) & 1) && !((mk[3] >> pm[3]) & 1)) {
            chosen = ch;
            pi = q;
            break;
          }
        }
      }
      if (chosen < 0) {
        used.emplace_back(nloc, 0);
        cnt.push_back(0);
        chosen = (int)used.size() - 1;
        pi = 0;
      }
      const int* pm = kPerms.p[pi];
      Placed pl;
      pl.chunk = chosen;
      pl.lane = cnt[chosen]++;
      for (int a = 0; a < 4; ++a) {
        used[chosen][lv[a]] |= (uint8_t)(1u << pm[a]);
        pl.v[pm[a]] = v[a];  // vertex a goes to slot pm[a]
      }
      placed.push_back(pl);
    }
    d.n_chunks = (int32_t)used.size();
    const size_t base = out.chunks.size();
    out.chunks.resize(base + used.size());
    out.chunk_neg.resize(base + used.size(), 0);
    for (size_t q = base; q < out.chunks.size(); ++q) {
      TetChunk& ch = out.chunks[q];
      std::memset(&ch, 0, sizeof(TetChunk));
      for (int l = 0; l < kChunk; ++l) ch.a[l][0] = ch.a[l][1] = kEmptyLane;
    }
    for (const Placed& pl : placed) {
      TetChunk& ch = out.chunks[base + pl.chunk];
      ch.a[pl.lane][0] = (uint32_t)loc[pl.v[0]] | ((uint32_t)loc[pl.v[1]] << 16);
      ch.a[pl.lane][1] = (uint32_t)loc[pl.v[2]] | ((uint32_t)loc[pl.v[3]] << 16);
      double Bt[9];
      const double det = reference_inverse(X, pl.v, Bt, nullptr);
      const float v0f = (float)(std::fabs(det) / 6.0), b0f = (float)Bt[0];
      std::memcpy(&ch.a[pl.lane][2], &v0f, sizeof(float));
      std::memcpy(&ch.a[pl.lane][3], &b0f, sizeof(float));
      for (int q = 1; q < 5; ++q) ch.b[pl.lane][q - 1] = (float)Bt[q];
      for (int q = 5; q < 9; ++q) ch.c[pl.lane][q - 5] = (float)Bt[q];
      if (det < 0) out.chunk_neg[base + pl.chunk] |= 1ull << pl.lane;
    }
  }
  // Shared node -> its slots, in tile order.
  out.shared_node.resize(n_shared);
  for (int32_t s = 0; s < n_shared; ++s) out.shared_node[s] = n_owned + s;
  out.shared_slot_ptr.assign(n_shared + 1, 0);
  for (int32_t node : out.slot_node) out.shared_slot_ptr[node - n_owned + 1]++;
  for (int32_t s = 0; s < n_shared; ++s)
    out.shared_slot_ptr[s + 1] += out.shared_slot_ptr[s];
  out.shared_slots.resize(out.slot_node.size());
  std::vector<int32_t> fill(out.shared_slot_ptr.begin(), out.shared_slot_ptr.end() - 1);
  for (size_t q = 0; q < out.slot_node.size(); ++q)
    out.shared_slots[fill[out.slot_node[q] - n_owned]++] = (int32_t)q;
}

}  // namespace

int prepare_batch(int32_t n_cells, const int64_t* node_off,
                  const int64_t* tet_off, const double* ref_xyz,
                  const int32_t* tets, const uint8_t* tet_region,
                  int32_t n_regions, const PrepOptions& opt, Prepared* P,
                  std::string* err) {
  if (n_cells <= 0 || !node_off || !tet_off || !ref_xyz || !tets) {
    *err = "null pointer or n_cells <= 0";
    return CM_EINVAL;
  }
  if (n_regions < 1 || n_regions > kMaxRegions || (n_regions > 1 && !tet_region)) {
    *err = "n_regions must be in [1, " + std::to_string(kMaxRegions) +
           "] (with a region array when > 1)";
    return CM_EINVAL;
  }
  if ((int64_t)n_cells * n_regions >= 0x7fffffffLL) {
    *err = "too many material slots";
    return CM_EINVAL;
  }
  if (opt.tile_tets < kChunk || opt.tile_tets > kMaxTileTets || opt.tile_tets % kChunk) {
    *err = "tile_tets must be a multiple of 64 in [64, 4096]";
    return CM_EINVAL;
  }
  if (opt.order < 0 || opt.order > 3) {
    *err = "unknown order";
    return CM_EINVAL;
  }
  if (node_off[0] != 0 || tet_off[0] != 0) {
    *err = "offsets must start at 0";
    return CM_EINVAL;
  }
  for (int32_t c = 0; c < n_cells; ++c)
    if (node_off[c + 1] < node_off[c] || tet_off[c + 1] < tet_off[c]) {
      *err = "offsets must be non-decreasing";
      return CM_EINVAL;
    }
  if (node_off[n_cells] >= 0x7fffffffLL) {
    *err = "more than 2^31 - 1 nodes";
    return CM_EINVAL;
  }

  std::vector<CellOut> cells(n_cells);
  std::atomic<int32_t> next_cell(0);
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nt = std::min<unsigned>(nt, (unsigned)n_cells);
  auto work = [&]() {
    for (;;) {
      int32_t c = next_cell.fetch_add(1);
      if (c >= n_cells) break;
      prepare_cell(c, node_off[c + 1] - node_off[c], tet_off[c + 1] - tet_off[c],
                   ref_xyz + 3 * node_off[c], tets + 4 * tet_off[c],
                   tet_region ? tet_region + tet_off[c] : nullptr, n_regions, opt,
                   cells[c]);
    }
  };
  std::vector<std::thread> pool;
  for (unsigned i = 1; i < nt; ++i) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
  for (auto& cell : cells)
    if (cell.status != CM_OK) {
      *err = cell.err;
      return cell.status;
    }

  // Concatenate with global offsets.
  int64_t n_tiles = 0, n_chunks = 0, n_slots = 0, n_shared = 0;
  for (auto& cell : cells) {
    n_tiles += cell.tiles.size();
    n_chunks += cell.chunks.size();
    n_slots += cell.slot_node.size();
    n_shared += cell.shared_node.size();
  }
  if (n_chunks >= 0x7fffffffLL || n_slots >= 0x7fffffffLL) {
    *err = "batch too large for 32-bit tile tables";
    return CM_EINVAL;
  }
  P->n_cells = n_cells;
  P->n_nodes = node_off[n_cells];
  P->n_tets = tet_off[n_cells];
  P->tiles.resize(n_tiles);
  P->chunks.resize(n_chunks);
  P->chunk_neg.resize(n_chunks);
  P->slot_node.resize(n_slots);
  P->shared_node.resize(n_shared);
  P->shared_slot_ptr.resize(n_shared + 1);
  P->shared_slots.resize(n_slots);
  P->cell_tile_off.resize(n_cells + 1);
  P->cell_shared_off.resize(n_cells + 1);
  P->node_off.assign(node_off, node_off + n_cells + 1);
  P->new_to_old.resize(P->n_nodes);
  P->space_order.resize(P->n_nodes);
  P->cell_candidates.resize(n_cells);
  P->n_regions = n_regions;
  P->tile_mat.resize(n_tiles);
  P->mat_tile_first.resize((size_t)n_cells * n_regions);
  P->mat_tile_count.resize((size_t)n_cells * n_regions);
  P->volume = 0.0;
  P->min_v0 = INFINITY;
  P->max_cond = 0.0;
  P->max_tile_nodes = 0;
  int64_t tb = 0, cb = 0, sb = 0, hb = 0;
  P->shared_slot_ptr[0] = 0;
  for (int32_t c = 0; c < n_cells; ++c) {
    CellOut& cell = cells[c];
    const int32_t nb = (int32_t)node_off[c];
    P->cell_tile_off[c] = (int32_t)tb;
    P->cell_shared_off[c] = (int32_t)hb;
    for (size_t k = 0; k < cell.tiles.size(); ++k) {
      TileDesc d = cell.tiles[k];
      d.chunk_begin += (int32_t)cb;
      d.own_begin += nb;
      d.shr_begin += (int32_t)sb;
      P->tiles[tb + k] = d;
      P->tile_mat[tb + k] = c * n_regions + cell.tile_region[k];
    }
    for (int32_t r = 0; r < n_regions; ++r) {
      P->mat_tile_first[(size_t)c * n_regions + r] = (int32_t)tb + cell.region_tile_first[r];
      P->mat_tile_count[(size_t)c * n_regions + r] = cell.region_tile_count[r];
    }
    std::copy(cell.chunk_neg.begin(), cell.chunk_neg.end(), P->chunk_neg.begin() + cb);
    std::memcpy(P->chunks.data() + cb, cell.chunks.data(),
                sizeof(TetChunk) * cell.chunks.size());
    for (size_t q = 0; q < cell.slot_node.size(); ++q) {
      P->slot_node[sb + q] = cell.slot_node[q] + nb;
      P->shared_slots[sb + q] = cell.shared_slots[q] + (int32_t)sb;
    }
    for (size_t s = 0; s < cell.shared_node.size(); ++s) {
      P->shared_node[hb + s] = cell.shared_node[s] + nb;
      P->shared_slot_ptr[hb + s + 1] = cell.shared_slot_ptr[s + 1] + (int32_t)sb;
    }
    for (size_t v = 0; v < cell.new_to_old.size(); ++v)
      P->new_to_old[nb + v] = cell.new_to_old[v] + nb;
    for (size_t v = 0; v < cell.space_order.size(); ++v)
      P->space_order[nb + v] = cell.space_order[v] + nb;
    P->cell_candidates[c] = cell.n_candidates;
    P->volume += cell.volume;
    P->min_v0 = std::min(P->min_v0, cell.min_v0);
    P->max_cond = std::max(P->max_cond, cell.max_cond);
    P->max_tile_nodes = std::max(P->max_tile_nodes, cell.max_tile_nodes);
    tb += cell.tiles.size();
    cb += cell.chunks.size();
    sb += cell.slot_node.size();
    hb += cell.shared_node.size();
    std::vector<TetChunk>().swap(cell.chunks);
  }
  P->cell_tile_off[n_cells] = (int32_t)tb;
  P->cell_shared_off[n_cells] = (int32_t)hb;
  P->cell_tile_first.resize(n_cells);
  P->cell_tile_count.resize(n_cells);
  for (int32_t c = 0; c < n_cells; ++c) {
    P->cell_tile_first[c] = P->cell_tile_off[c];
    P->cell_tile_count[c] = P->cell_tile_off[c + 1] - P->cell_tile_off[c];
  }
  P->tile_stride = 1;
  return CM_OK;
}

int prepare_template(int32_t n_cells, int64_t n_nodes, int64_t n_tets,
                     const double* ref_xyz, const int32_t* tets,
                     const uint8_t* tet_region, int32_t n_regions,
                     const PrepOptions& opt, Prepared* P, std::string* err) {
  if (n_cells <= 0) {
    *err = "n_cells must be positive";
    return CM_EINVAL;
  }
  const int64_t no[2] = {0, n_nodes}, to[2] = {0, n_tets};
  Prepared one;
  int rc = prepare_batch(1, no, to, ref_xyz, tets, tet_region, n_regions, opt,
                         &one, err);
  if (rc != CM_OK) return rc;
  const int64_t C = n_cells, N = n_nodes;
  const int64_t T1 = (int64_t)one.tiles.size(), S1 = (int64_t)one.slot_node.size();
  const int64_t H1 = (int64_t)one.shared_node.size();
  const int64_t R = n_regions;
  if (C * N >= 0x7fffffffLL || C * T1 >= 0x7fffffffLL || C * S1 >= 0x7fffffffLL ||
      C * R >= 0x7fffffffLL) {
    *err = "template batch too large for 32-bit tables";
    return CM_EINVAL;
  }
  P->n_cells = C;
  P->n_nodes = C * N;
  P->n_tets = C * n_tets;
  P->chunks = std::move(one.chunks);
  P->chunk_neg = std::move(one.chunk_neg);
  P->tiles.resize(C * T1);
  P->tile_mat.resize(C * T1);
  for (int64_t k = 0; k < T1; ++k)
    for (int64_t c = 0; c < C; ++c) {
      TileDesc d = one.tiles[k];
      d.own_begin += (int32_t)(c * N);
      d.shr_begin += (int32_t)(c * S1);
      d.cell = (int32_t)c;
      P->tiles[k * C + c] = d;
      P->tile_mat[k * C + c] = (int32_t)(c * R) + one.tile_mat[k];
    }
  P->n_regions = n_regions;
  P->mat_tile_first.resize(C * R);
  P->mat_tile_count.resize(C * R);
  for (int64_t c = 0; c < C; ++c)
    for (int64_t r = 0; r < R; ++r) {
      P->mat_tile_first[c * R + r] = (int32_t)(c + one.mat_tile_first[r] * C);
      P->mat_tile_count[c * R + r] = one.mat_tile_count[r];
    }
  P->slot_node.resize(C * S1);
  P->shared_slots.resize(C * S1);
  P->shared_node.resize(C * H1);
  P->shared_slot_ptr.resize(C * H1 + 1);
  P->new_to_old.resize(C * N);
  P->space_order.resize(C * N);
  P->cell_candidates.assign(C, one.cell_candidates[0]);
  P->node_off.resize(C + 1);
  P->cell_shared_off.resize(C + 1);
  P->cell_tile_first.resize(C);
  P->cell_tile_count.assign(C, (int32_t)T1);
  P->shared_slot_ptr[0] = 0;
  for (int64_t c = 0; c < C; ++c) {
    for (int64_t q = 0; q < S1; ++q) {
      P->slot_node[c * S1 + q] = one.slot_node[q] + (int32_t)(c * N);
      P->shared_slots[c * S1 + q] = one.shared_slots[q] + (int32_t)(c * S1);
    }
    for (int64_t h = 0; h < H1; ++h) {
      P->shared_node[c * H1 + h] = one.shared_node[h] + (int32_t)(c * N);
      P->shared_slot_ptr[c * H1 + h + 1] = one.shared_slot_ptr[h + 1] + (int32_t)(c * S1);
    }
    for (int64_t v = 0; v < N; ++v) P->new_to_old[c * N + v] = one.new_to_old[v] + c * N;
    for (int64_t v = 0; v < N; ++v)
      P->space_order[c * N + v] = one.space_order[v] + (int32_t)(c * N);
    P->node_off[c] = c * N;
    P->cell_shared_off[c] = (int32_t)(c * H1);
    P->cell_tile_first[c] = (int32_t)c;
  }
  P->node_off[C] = C * N;
  P->cell_shared_off[C] = (int32_t)(C * H1);
  P->cell_tile_off.clear();
  P->tile_stride = (int32_t)C;
  P->max_tile_nodes = one.max_tile_nodes;
  P->volume = one.volume * (double)C;
  P->min_v0 = one.min_v0;
  P->max_cond = one.max_cond;
  return CM_OK;
}

}  // namespace cm
