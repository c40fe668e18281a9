// C ABI of libcellmech (declared in include/cellmech.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "cellmech.h"
#include "aux_kernels.h"
#include "handle.h"
#include "kernels.h"
#include "prep.h"

namespace {

thread_local std::string g_err;

int fail(int st, const std::string& msg) {
  g_err = msg;
  return st;
}

}  // namespace

int cm::api_fail(int st, const std::string& msg) { return fail(st, msg); }

namespace {

int check_handle(cm_batch h) {
  if (!h) return fail(CM_EINVAL, "null handle");
  return CM_OK;
}

cm::Range full_range(const cm_batch_s* h) {
  return cm::Range{0, (int32_t)h->n_tiles, 0, (int32_t)h->n_shared, 0,
                   (int32_t)h->n_cells};
}

cm::Range cell_range(const cm_batch_s* h, int32_t c) {
  return cm::Range{h->cell_tile_off[c], h->cell_tile_off[c + 1],
                   h->cell_shared_off[c], h->cell_shared_off[c + 1], c, c + 1};
}

int select_device(cm_batch h) {
  int cur = 0;
  CM_HIP(hipGetDevice(&cur));
  if (cur != h->device) CM_HIP(hipSetDevice(h->device));
  return CM_OK;
}

bool lds_fits(const cm_batch_s* h, int waves, bool backward) {
  size_t per = backward ? cm::backward_lds_per_wave(h->T.nloc)
                        : cm::forward_lds_per_wave(h->T.nloc);
  return per * (size_t)waves <= 65536;
}

// The fused forward + backward pass needs more LDS per wave than either
// pass: it runs with the handle's launch shape, its waves per workgroup
// halved until its LDS fits (results do not depend on the launch shape).
bool fused_cfg(const cm_batch_s* h, cm::LaunchCfg* cfg) {
  *cfg = h->cfg;
  while (cfg->waves > 1 &&
         cm::forward_backward_lds_per_wave(h->T.nloc) * (size_t)cfg->waves > 65536)
    cfg->waves /= 2;
  return cm::forward_backward_lds_per_wave(h->T.nloc) * (size_t)cfg->waves <= 65536;
}

}  // namespace

extern "C" {

const char* cm_last_error(void) { return g_err.c_str(); }

int cm_version(void) { return 1; }

void cm_options_default(cm_options* opt) {
  if (!opt) return;
  opt->order = CM_ORDER_BISECT;
  opt->tile_tets = 768;
  opt->degenerate_tol = 1e-12;
}

static cm::PrepOptions prep_options(const cm_options* opt) {
  cm::PrepOptions po;
  if (opt) {
    po.order = opt->order;
    po.tile_tets = opt->tile_tets ? opt->tile_tets : 768;
    po.degenerate_tol = opt->degenerate_tol > 0 ? opt->degenerate_tol : 1e-12;
  }
  return po;
}

// Uploads a prepared layout and builds the handle.
static int create_from(cm::Prepared& P, const cm::PrepOptions& po,
                       hipStream_t stream, cm_batch* out) {
  int rc = CM_OK;
  cm_batch_s* h = new (std::nothrow) cm_batch_s();
  if (!h) return fail(CM_ENOMEM, "host allocation failed");
  auto bail = [&](int st) { delete h; return st; };
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) return bail(fail(CM_EHIP, hipGetErrorString(e)));
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, h->device);
  if (e != hipSuccess) return bail(fail(CM_EHIP, hipGetErrorString(e)));
  h->n_cu = prop.multiProcessorCount;

  h->n_cells = P.n_cells;
  h->n_regions = P.n_regions;
  h->n_mat = P.n_cells * (int64_t)P.n_regions;
  h->n_nodes = P.n_nodes;
  h->n_tets = P.n_tets;
  h->n_slots = (int64_t)P.slot_node.size();
  h->n_shared = (int64_t)P.shared_node.size();
  h->n_tiles = (int64_t)P.tiles.size();
  h->n_chunks = (int64_t)P.chunks.size();
  h->tile_tets = po.tile_tets;
  h->max_tile_nodes = P.max_tile_nodes;
  h->volume = P.volume;
  h->min_v0 = P.min_v0;
  h->max_cond = P.max_cond;
  h->cell_tile_off = P.cell_tile_off;
  h->cell_shared_off = P.cell_shared_off;
  h->is_template = P.tile_stride != 1;
  h->new_to_old = std::move(P.new_to_old);

  cm::DeviceTables& T = h->T;
  // host tables built here are copied asynchronously: they live until the
  // stream synchronisation below
  std::vector<int32_t> shared_cell, orphan_off, orphan, slot_first, shared_first;
  std::vector<int4> pc;
  std::vector<int2> nbk;
  {
    cm::TileDesc* tiles;
    cm::TetChunk* chunks;
    int32_t *slot_node, *shared_node, *ssp, *ss, *ctf, *ctc, *tmat, *mtf, *mtc, *scell;
    int32_t *orph_off, *orph, *sfirst, *cso;
    int64_t* noff;
    // cell of every shared node; slot_node with bit 31 on the first slot of
    // every shared node; shared nodes in no slot (nodes of no tetrahedron),
    // grouped by cell
    const size_t n_shr = P.shared_node.size();
    shared_cell.assign(n_shr, 0);
    orphan_off.assign(h->n_cells + 1, 0);
    slot_first.assign(P.slot_node.begin(), P.slot_node.end());
    for (size_t s = 0; s < n_shr; ++s) {
      shared_cell[s] = (int32_t)(std::upper_bound(P.node_off.begin(), P.node_off.end(),
                                                  (int64_t)P.shared_node[s]) -
                                 P.node_off.begin() - 1);
      if (P.shared_slot_ptr[s] < P.shared_slot_ptr[s + 1])
        slot_first[P.shared_slots[P.shared_slot_ptr[s]]] |= INT32_MIN;
      else
        ++orphan_off[shared_cell[s] + 1];
    }
    for (int64_t c = 0; c < h->n_cells; ++c) orphan_off[c + 1] += orphan_off[c];
    orphan.resize(orphan_off[h->n_cells]);
    {
      std::vector<int32_t> fill(orphan_off.begin(), orphan_off.end() - 1);
      for (size_t s = 0; s < n_shr; ++s)
        if (P.shared_slot_ptr[s] == P.shared_slot_ptr[s + 1])
          orphan[fill[shared_cell[s]]++] = P.shared_node[s];
    }
    if ((rc = h->upload(&tiles, P.tiles, stream)) ||
        (rc = h->upload(&chunks, P.chunks, stream)) ||
        (rc = h->upload(&slot_node, P.slot_node, stream)) ||
        (rc = h->upload(&shared_node, P.shared_node, stream)) ||
        (rc = h->upload(&ssp, P.shared_slot_ptr, stream)) ||
        (rc = h->upload(&ss, P.shared_slots, stream)) ||
        (rc = h->upload(&scell, shared_cell, stream)) ||
        (rc = h->upload(&sfirst, slot_first, stream)) ||
        (rc = h->upload(&orph_off, orphan_off, stream)) ||
        (rc = h->upload(&orph, orphan, stream)) ||
        (rc = h->upload(&ctf, P.cell_tile_first, stream)) ||
        (rc = h->upload(&ctc, P.cell_tile_count, stream)) ||
        (rc = h->upload(&tmat, P.tile_mat, stream)) ||
        (rc = h->upload(&mtf, P.mat_tile_first, stream)) ||
        (rc = h->upload(&mtc, P.mat_tile_count, stream)) ||
        (rc = h->upload(&noff, P.node_off, stream)) ||
        (rc = h->upload(&cso, P.cell_shared_off, stream)))
      return bail(rc);
    T.cell_shared_off = cso;
    // first shared node of every cell (its shared nodes are contiguous)
    shared_first.resize(h->n_cells);
    for (int32_t c = 0; c < h->n_cells; ++c)
      shared_first[c] = P.cell_shared_off[c + 1] > P.cell_shared_off[c]
                            ? P.shared_node[P.cell_shared_off[c]]
                            : (int32_t)P.node_off[c + 1];
    int32_t* csf;
    if ((rc = h->upload(&csf, shared_first, stream))) return bail(rc);
    T.cell_shared_first = csf;
    h->d_node_off = noff;
    T.tiles = tiles;
    T.chunks = chunks;
    T.slot_node = slot_node;
    T.shared_node = shared_node;
    T.shared_slot_ptr = ssp;
    T.shared_slots = ss;
    T.shared_cell = scell;
    T.slot_node_first = sfirst;
    T.orphan_off = orph_off;
    T.orphan_node = orph;
    T.cell_tile_first = ctf;
    T.cell_tile_count = ctc;
    T.tile_stride = P.tile_stride;
    T.tile_mat = tmat;
    T.mat_tile_first = mtf;
    T.mat_tile_count = mtc;
    double* params;
    float *part, *part_b;
    double *tile_acc, *tile_acc_b, *tile_plate;
    int32_t *tile_ninv, *tile_nonfin;
    if ((rc = h->alloc(&params, 3 * (size_t)h->n_mat)) ||
        (rc = h->alloc(&tile_nonfin, (size_t)h->n_tiles)) ||
        (rc = h->alloc(&part, 3 * (size_t)h->n_slots)) ||
        (rc = h->alloc(&part_b, 3 * (size_t)h->n_slots)) ||
        (rc = h->alloc(&tile_acc, (size_t)h->n_tiles)) ||
        (rc = h->alloc(&tile_acc_b, 3 * (size_t)h->n_tiles)) ||
        (rc = h->alloc(&tile_plate, (size_t)h->n_tiles)) ||
        (rc = h->alloc(&tile_ninv, (size_t)h->n_tiles)))
      return bail(rc);
    // 256 x 256 node-pair blocks of every cell (row block <= column block);
    // the cell's nodes are ordered candidates first, so the pairs of the
    // first ceil(candidates / 256) blocks hold every candidate pair
    // pc: the candidate pair blocks; nbk: the candidate node blocks of every cell
    for (int64_t c = 0; c < h->n_cells; ++c) {
      const int64_t nb = (P.node_off[c + 1] - P.node_off[c] + 255) / 256;
      int64_t bc = ((int64_t)P.cell_candidates[c] + 255) / 256;
      if (bc <= 0) bc = nb;
      const int base = (int)nbk.size();
      for (int64_t i = 0; i < bc; ++i) {
        nbk.push_back(make_int2((int)c, (int)i));
        for (int64_t j = i; j < bc; ++j)
          pc.push_back(make_int4((int)c, (int)i, (int)j, base));
      }
    }
    int4* pcd;
    int2* nbd;
    int32_t *sord, *tinv, *cinv;
    uint64_t* cneg;
    double *mom, *bbox;
    unsigned long long* d2;
    if ((rc = h->upload(&pcd, pc, stream)) ||
        (rc = h->upload(&sord, P.space_order, stream)) ||
        (rc = h->upload(&cneg, P.chunk_neg, stream)) ||
        (rc = h->upload(&nbd, nbk, stream)) ||
        (rc = h->alloc(&bbox, 6 * nbk.size())) ||
        (rc = h->alloc(&mom, 10 * (size_t)h->n_tiles)) ||
        (rc = h->alloc(&tinv, (size_t)h->n_tiles)) ||
        (rc = h->alloc(&cinv, (size_t)h->n_cells)) ||
        (rc = h->alloc(&d2, (size_t)h->n_cells)))
      return bail(rc);
    h->cand_blocks = pcd;
    h->n_cand_blocks = (int64_t)pc.size();
    h->shape_tile_inv = tinv;
    h->chunk_neg = cneg;
    h->shape_cell_inv = cinv;
    h->node_blocks = nbd;
    h->n_node_blocks = (int64_t)nbk.size();
    h->shape_bbox = bbox;
    h->space_order = sord;
    h->shape_mom = mom;
    h->d2max = d2;
    T.params = params;
    T.part = part;
    T.tile_acc = tile_acc;
    T.tile_plate = tile_plate;
    T.tile_ninv = tile_ninv;
    T.tile_nonfin = tile_nonfin;
    h->Tb = T;
    h->Tb.part = part_b;
    h->Tb.tile_acc = tile_acc_b;
    h->Tb.tile_ninv = nullptr;
    h->Tb.tile_nonfin = nullptr;
  }
  for (cm::DeviceTables* t : {&h->T, &h->Tb}) {
    t->n_nodes = h->n_nodes;
    t->n_slots = h->n_slots;
    t->n_tiles = h->n_tiles;
    t->n_cells = (int32_t)h->n_cells;
    t->n_regions = h->n_regions;
    t->n_mat = (int32_t)h->n_mat;
    t->nloc = (h->max_tile_nodes + 3) & ~3;
    if (t->nloc == 0) t->nloc = 4;
  }
  e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) return bail(fail(CM_EHIP, hipGetErrorString(e)));
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return bail(fail(CM_EHIP, hipGetErrorString(e)));
  h->cfg.waves = 1;
  h->cfg.blocks = 0;
  *out = h;
  return CM_OK;
}

int cm_batch_create(int32_t n_cells, const int64_t* node_off,
                    const int64_t* tet_off, const double* ref_xyz,
                    const int32_t* tets, const cm_options* opt,
                    hipStream_t stream, cm_batch* out) {
  g_err.clear();
  if (!out) return fail(CM_EINVAL, "out is null");
  *out = nullptr;
  const cm::PrepOptions po = prep_options(opt);
  cm::Prepared P;
  std::string err;
  int rc = cm::prepare_batch(n_cells, node_off, tet_off, ref_xyz, tets, nullptr, 1,
                             po, &P, &err);
  if (rc != CM_OK) return fail(rc, err);
  return create_from(P, po, stream, out);
}

int cm_batch_create_regions(int32_t n_cells, const int64_t* node_off,
                            const int64_t* tet_off, const double* ref_xyz,
                            const int32_t* tets, const uint8_t* tet_region,
                            int32_t n_regions, const cm_options* opt,
                            hipStream_t stream, cm_batch* out) {
  g_err.clear();
  if (!out) return fail(CM_EINVAL, "out is null");
  *out = nullptr;
  const cm::PrepOptions po = prep_options(opt);
  cm::Prepared P;
  std::string err;
  int rc = cm::prepare_batch(n_cells, node_off, tet_off, ref_xyz, tets, tet_region,
                             n_regions, po, &P, &err);
  if (rc != CM_OK) return fail(rc, err);
  return create_from(P, po, stream, out);
}

int cm_template_create(int32_t n_cells, int64_t n_nodes, int64_t n_tets,
                       const double* ref_xyz, const int32_t* tets,
                       const cm_options* opt, hipStream_t stream,
                       cm_batch* out) {
  g_err.clear();
  if (!out) return fail(CM_EINVAL, "out is null");
  *out = nullptr;
  if (!ref_xyz || !tets || n_nodes < 0 || n_tets < 0)
    return fail(CM_EINVAL, "null pointer or negative size");
  const cm::PrepOptions po = prep_options(opt);
  cm::Prepared P;
  std::string err;
  int rc = cm::prepare_template(n_cells, n_nodes, n_tets, ref_xyz, tets, nullptr, 1,
                                po, &P, &err);
  if (rc != CM_OK) return fail(rc, err);
  return create_from(P, po, stream, out);
}

int cm_template_create_regions(int32_t n_cells, int64_t n_nodes, int64_t n_tets,
                               const double* ref_xyz, const int32_t* tets,
                               const uint8_t* tet_region, int32_t n_regions,
                               const cm_options* opt, hipStream_t stream,
                               cm_batch* out) {
  g_err.clear();
  if (!out) return fail(CM_EINVAL, "out is null");
  *out = nullptr;
  if (!ref_xyz || !tets || n_nodes < 0 || n_tets < 0)
    return fail(CM_EINVAL, "null pointer or negative size");
  const cm::PrepOptions po = prep_options(opt);
  cm::Prepared P;
  std::string err;
  int rc = cm::prepare_template(n_cells, n_nodes, n_tets, ref_xyz, tets, tet_region,
                                n_regions, po, &P, &err);
  if (rc != CM_OK) return fail(rc, err);
  return create_from(P, po, stream, out);
}

int cm_mesh_create(int64_t n_nodes, int64_t n_tets, const double* ref_xyz,
                   const int32_t* tets, const cm_options* opt,
                   hipStream_t stream, cm_mesh* out) {
  int64_t no[2] = {0, n_nodes}, to[2] = {0, n_tets};
  if (n_nodes < 0 || n_tets < 0) return fail(CM_EINVAL, "negative size");
  return cm_batch_create(1, no, to, ref_xyz, tets, opt, stream, out);
}

int cm_destroy(cm_batch h) {
  if (!h) return CM_OK;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  delete h;
  return CM_OK;
}

int cm_get_info(cm_batch h, cm_info* o) {
  if (int rc = check_handle(h)) return rc;
  if (!o) return fail(CM_EINVAL, "out is null");
  o->n_cells = h->n_cells;
  o->n_nodes = h->n_nodes;
  o->n_tets = h->n_tets;
  o->n_tiles = h->n_tiles;
  o->n_shared = h->n_shared;
  o->n_slots = h->n_slots;
  o->n_chunks = h->n_chunks;
  o->tile_tets = h->tile_tets;
  o->max_tile_nodes = h->max_tile_nodes;
  o->device_bytes = h->device_bytes;
  o->volume = h->volume;
  o->min_v0 = h->min_v0;
  o->max_cond = h->max_cond;
  o->n_regions = h->n_regions;
  return CM_OK;
}

int cm_permutation(cm_batch h, int64_t* new_to_old) {
  if (int rc = check_handle(h)) return rc;
  if (!new_to_old) return fail(CM_EINVAL, "out is null");
  std::memcpy(new_to_old, h->new_to_old.data(), sizeof(int64_t) * h->n_nodes);
  return CM_OK;
}

int cm_set_params(cm_batch h, const double* mu, const double* kappa,
                  const double* w, int on_device, hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!mu || !kappa || !w) return fail(CM_EINVAL, "null parameter array");
  if (int rc = select_device(h)) return rc;
  const size_t n = (size_t)h->n_mat;
  double* dst = const_cast<double*>(h->T.params);
  if (on_device) {
    CM_HIP(hipMemcpyAsync(dst, mu, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
    CM_HIP(hipMemcpyAsync(dst + n, kappa, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
    CM_HIP(hipMemcpyAsync(dst + 2 * n, w, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
  } else {
    std::vector<double> buf(3 * n);
    for (size_t c = 0; c < n; ++c) {
      if (!std::isfinite(mu[c]) || !std::isfinite(kappa[c]) || !std::isfinite(w[c]) ||
          mu[c] < 0 || kappa[c] < 0 || w[c] < 0 || w[c] > 1)
        return fail(CM_EINVAL, "material slot " + std::to_string(c) +
                                   ": parameters must be finite with mu >= 0, "
                                   "kappa >= 0, 0 <= w <= 1");
      buf[c] = mu[c];
      buf[n + c] = kappa[c];
      buf[2 * n + c] = w[c];
    }
    CM_HIP(hipMemcpyAsync(dst, buf.data(), 3 * n * sizeof(double),
                          hipMemcpyHostToDevice, stream));
    // the staging buffer is pageable and local: wait for the copy
    CM_HIP(hipStreamSynchronize(stream));
  }
  h->params_set = true;
  return CM_OK;
}

static int forces_impl(cm_batch h, const float* y, float* f, double* energy,
                       int32_t* ninv, hipStream_t st, bool percell,
                       int32_t* nonfin = nullptr) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !f) return fail(CM_EINVAL, "y and f must be device pointers");
  if (!h->params_set) return fail(CM_ESTATE, "cm_set_params was not called");
  if (!lds_fits(h, h->cfg.waves, false))
    return fail(CM_EINVAL, "launch configuration exceeds 64 KiB of LDS");
  if (int rc = select_device(h)) return rc;
  if (percell && h->is_template)
    return fail(CM_EINVAL, "per-cell launches need contiguous tiles (not a template batch)");
  if (!percell) {
    CM_HIP(cm::launch_forward(h->T, full_range(h), h->cfg, y, f, energy, ninv, st,
                              cm::PlateFwd{}, nonfin));
  } else {
    cm::LaunchCfg one{h->cfg.waves, 0};
    for (int32_t c = 0; c < (int32_t)h->n_cells; ++c)
      CM_HIP(cm::launch_forward(h->T, cell_range(h, c), one, y, f, energy, ninv, st,
                                cm::PlateFwd{}, nonfin));
  }
  return CM_OK;
}

static int backward_impl(cm_batch h, const float* y, const float* fbar,
                         const double* ebar, float* ybar, double* thetabar,
                         hipStream_t st, bool percell,
                         const cm::CellMask& mask = cm::CellMask{}) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !ybar) return fail(CM_EINVAL, "y and ybar must be device pointers");
  if (!h->params_set) return fail(CM_ESTATE, "cm_set_params was not called");
  if (!lds_fits(h, h->cfg.waves, true))
    return fail(CM_EINVAL, "launch configuration exceeds 64 KiB of LDS");
  if (int rc = select_device(h)) return rc;
  if (percell && h->is_template)
    return fail(CM_EINVAL, "per-cell launches need contiguous tiles (not a template batch)");
  if (!percell) {
    CM_HIP(cm::launch_backward(h->Tb, full_range(h), h->cfg, y, fbar, ebar, ybar,
                               thetabar, st, mask));
  } else {
    cm::LaunchCfg one{h->cfg.waves, 0};
    for (int32_t c = 0; c < (int32_t)h->n_cells; ++c)
      CM_HIP(cm::launch_backward(h->Tb, cell_range(h, c), one, y, fbar, ebar,
                                 ybar, thetabar, st));
  }
  return CM_OK;
}

static int forward_backward_impl(cm_batch h, const float* y, float* f,
                                 double* energy, int32_t* ninv, const float* fbar,
                                 const double* ebar, float* ybar, double* thetabar,
                                 hipStream_t st) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !f || !ybar) return fail(CM_EINVAL, "y, f and ybar must be device pointers");
  // the outputs are written while other tiles still read the inputs
  if (f == ybar || f == y || ybar == y || (fbar && (f == fbar || ybar == fbar)))
    return fail(CM_EINVAL, "f and ybar must not alias each other, y or fbar");
  if (!h->params_set) return fail(CM_ESTATE, "cm_set_params was not called");
  cm::LaunchCfg cfg;
  if (!fused_cfg(h, &cfg))
    return fail(CM_EINVAL, "fused pass: one tile's nodes exceed 64 KiB of LDS");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_forward_backward(h->T, h->Tb, full_range(h), cfg, y, f, energy, ninv,
                                     fbar, ebar, ybar, thetabar, st));
  return CM_OK;
}

int cm_forces_and_backward(cm_batch h, const float* y, float* f, double* energy,
                           int32_t* n_inverted, const float* fbar, const double* ebar,
                           float* ybar, double* thetabar, hipStream_t stream) {
  return forward_backward_impl(h, y, f, energy, n_inverted, fbar, ebar, ybar, thetabar,
                               stream);
}

int cm_forces(cm_batch h, const float* y, float* f, double* energy,
              int32_t* n_inverted, hipStream_t stream) {
  return forces_impl(h, y, f, energy, n_inverted, stream, false);
}

int cm_forces_checked(cm_batch h, const float* y, float* f, double* energy,
                      int32_t* n_inverted, int32_t* n_nonfinite, hipStream_t stream) {
  if (!n_nonfinite) return fail(CM_EINVAL, "n_nonfinite must be a device pointer");
  return forces_impl(h, y, f, energy, n_inverted, stream, false, n_nonfinite);
}

int cm_forces_percell(cm_batch h, const float* y, float* f, double* energy,
                      int32_t* n_inverted, hipStream_t stream) {
  return forces_impl(h, y, f, energy, n_inverted, stream, true);
}

int cm_forces_backward(cm_batch h, const float* y, const float* fbar,
                       const double* ebar, float* ybar, double* thetabar,
                       hipStream_t stream) {
  return backward_impl(h, y, fbar, ebar, ybar, thetabar, stream, false);
}

int cm_forces_backward_percell(cm_batch h, const float* y, const float* fbar,
                               const double* ebar, float* ybar,
                               double* thetabar, hipStream_t stream) {
  return backward_impl(h, y, fbar, ebar, ybar, thetabar, stream, true);
}

int cm_forces_backward_cells(cm_batch h, const float* y, const float* fbar,
                             const double* ebar, const double* cell_flags,
                             int64_t flag_stride, float* ybar, double* thetabar,
                             hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!cell_flags) return fail(CM_EINVAL, "cell_flags must be a device pointer");
  if (flag_stride < 1) return fail(CM_EINVAL, "flag_stride must be >= 1");
  cm::CellMask mask{cell_flags, flag_stride};
  return backward_impl(h, y, fbar, ebar, ybar, thetabar, stream, false, mask);
}

int cm_set_launch(cm_batch h, int32_t waves, int32_t blocks_per_cu) {
  if (int rc = check_handle(h)) return rc;
  if (waves != 1 && waves != 2 && waves != 4 && waves != 8)
    return fail(CM_EINVAL, "waves_per_block must be 1, 2, 4 or 8");
  if (blocks_per_cu < 0 || blocks_per_cu > 64)
    return fail(CM_EINVAL, "blocks_per_cu must be in [0, 64]");
  if (!lds_fits(h, waves, true) || !lds_fits(h, waves, false))
    return fail(CM_EINVAL, "launch configuration exceeds 64 KiB of LDS");
  h->cfg.waves = waves;
  h->cfg.blocks = blocks_per_cu * h->n_cu;
  return CM_OK;
}

int cm_get_launch(cm_batch h, int32_t* waves, int32_t* blocks_per_cu) {
  if (int rc = check_handle(h)) return rc;
  if (waves) *waves = h->cfg.waves;
  if (blocks_per_cu) *blocks_per_cu = h->n_cu ? h->cfg.blocks / h->n_cu : 0;
  return CM_OK;
}

// Autotuner cache: one JSON object, one entry per line,
//   "<key>": {"waves": W, "blocks_per_cu": B, "ms": T},
static bool cache_lookup(const char* path, const std::string& key, int* w, int* b) {
  std::ifstream in(path);
  if (!in) return false;
  std::string line, pre = "\"" + key + "\":";
  while (std::getline(in, line)) {
    size_t p = line.find(pre);
    if (p == std::string::npos) continue;
    return std::sscanf(line.c_str() + p + pre.size(),
                       " {\"waves\": %d, \"blocks_per_cu\": %d", w, b) == 2;
  }
  return false;
}

static void cache_store(const char* path, const std::string& key, int w, int b,
                        double ms) {
  std::vector<std::string> entries;
  {
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
      // every entry line (launch entries and tuned-creation entries)
      if (line.find("\": {\"") == std::string::npos) continue;
      if (line.find("\"" + key + "\":") != std::string::npos) continue;
      while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
      entries.push_back(line);
    }
  }
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "  \"%s\": {\"waves\": %d, \"blocks_per_cu\": %d, \"ms\": %.6f}",
                key.c_str(), w, b, ms);
  entries.push_back(buf);
  std::ofstream out(path, std::ios::trunc);
  out << "{\n";
  for (size_t i = 0; i < entries.size(); ++i)
    out << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
  out << "}\n";
}

// Entries of the tuned creation: "<key>": {"tile": T, "waves": W,
// "blocks_per_cu": B, "ms": M}, in the same file format.
static bool cache_lookup_tile(const char* path, const std::string& key, int* w, int* b,
                              int* t) {
  std::ifstream in(path);
  if (!in) return false;
  std::string line, pre = "\"" + key + "\":";
  while (std::getline(in, line)) {
    size_t p = line.find(pre);
    if (p == std::string::npos) continue;
    return std::sscanf(line.c_str() + p + pre.size(),
                       " {\"tile\": %d, \"waves\": %d, \"blocks_per_cu\": %d", t, w,
                       b) == 3;
  }
  return false;
}

static void cache_store_tile(const char* path, const std::string& key, int w, int b,
                             int t, double ms) {
  std::vector<std::string> entries;
  {
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
      if (line.find("\": {\"") == std::string::npos) continue;
      if (line.find("\"" + key + "\":") != std::string::npos) continue;
      while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
      entries.push_back(line);
    }
  }
  char buf[768];
  std::snprintf(buf, sizeof buf,
                "  \"%s\": {\"tile\": %d, \"waves\": %d, \"blocks_per_cu\": %d, "
                "\"ms\": %.6f}",
                key.c_str(), t, w, b, ms);
  entries.push_back(buf);
  std::ofstream out(path, std::ios::trunc);
  out << "{\n";
  for (size_t i = 0; i < entries.size(); ++i)
    out << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
  out << "}\n";
}

// Times forward + backward for every launch configuration that fits in LDS
// (waves per block x persistent blocks per CU, two rounds, the better round
// of each), leaves h->cfg at the fastest and returns its time in *best_ms.
static int tune_launch(cm_batch h, const float* y, hipStream_t stream,
                       double* best_ms_out) {
  const size_t n3 = 3 * (size_t)h->n_nodes;
  float *f = nullptr, *ybar = nullptr;
  double *energy = nullptr, *tb = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = CM_OK;
  double best_ms = INFINITY;
  int best_w = h->cfg.waves, best_b = h->n_cu ? h->cfg.blocks / h->n_cu : 0;
  const cm::LaunchCfg saved = h->cfg;
  auto cleanup = [&]() {
    if (f) (void)hipFree(f);
    if (ybar) (void)hipFree(ybar);
    if (energy) (void)hipFree(energy);
    if (tb) (void)hipFree(tb);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc((void**)&f, n3 * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&ybar, n3 * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&energy, h->n_cells * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&tb, 3 * h->n_mat * sizeof(double)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(CM_ENOMEM, "autotune scratch allocation failed");
  }
  const int waves[4] = {1, 2, 4, 8};
  const int bpcu[6] = {0, 1, 2, 4, 8, 16};
  // the objective is one full forward + backward evaluation: the fused pass
  // (the fastest route) where its LDS fits, else the two separate passes
  auto run = [&]() {
    cm::LaunchCfg fc;
    if (fused_cfg(h, &fc))
      return forward_backward_impl(h, y, f, energy, nullptr, y, nullptr, ybar, tb, stream);
    int r = forces_impl(h, y, f, energy, nullptr, stream, false);
    if (r == CM_OK) r = backward_impl(h, y, y, energy, ybar, tb, stream, false);
    return r;
  };
  // bring the clocks to their loaded state before measuring
  h->cfg = saved;
  if (!lds_fits(h, h->cfg.waves, true) || !lds_fits(h, h->cfg.waves, false))
    h->cfg.waves = 1;
  for (int k = 0; k < 20 && rc == CM_OK; ++k) rc = run();
  double ms_of[4][6];
  for (int wi = 0; wi < 4; ++wi)
    for (int bi = 0; bi < 6; ++bi) ms_of[wi][bi] = INFINITY;
  // two rounds over all candidates; a candidate's time is its better round
  for (int round = 0; round < 2 && rc == CM_OK; ++round)
    for (int wi = 0; wi < 4 && rc == CM_OK; ++wi) {
      if (!lds_fits(h, waves[wi], true) || !lds_fits(h, waves[wi], false)) continue;
      for (int bi = 0; bi < 6 && rc == CM_OK; ++bi) {
        h->cfg.waves = waves[wi];
        h->cfg.blocks = bpcu[bi] * h->n_cu;
        rc = run();
        if (rc != CM_OK) break;
        const int reps = 4;
        if (hipEventRecord(e0, stream) != hipSuccess) { rc = fail(CM_EHIP, "event"); break; }
        for (int k = 0; k < reps && rc == CM_OK; ++k) rc = run();
        if (rc != CM_OK) break;
        float ms = 0.f;
        if (hipEventRecord(e1, stream) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = fail(CM_EHIP, "autotune timing failed");
          break;
        }
        ms_of[wi][bi] = std::min(ms_of[wi][bi], (double)ms / reps);
      }
    }
  for (int wi = 0; wi < 4; ++wi)
    for (int bi = 0; bi < 6; ++bi)
      if (ms_of[wi][bi] < best_ms) {
        best_ms = ms_of[wi][bi];
        best_w = waves[wi];
        best_b = bpcu[bi];
      }
  cleanup();
  h->cfg = saved;
  if (rc != CM_OK) return rc;
  if (best_ms_out) *best_ms_out = best_ms;
  return cm_set_launch(h, best_w, best_b);
}

static std::string device_key(cm_batch h) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, h->device) != hipSuccess) return "unknown";
  return std::string(prop.gcnArchName) + "|cu" + std::to_string(h->n_cu);
}

// Names what a cached timing measured (one fused forward + backward
// evaluation), so that entries timed with another objective are not reused.
static const char* const kTuneObjective = "|fused-fwd-bwd";

static std::string sanitize_key(std::string key) {
  for (char& ch : key)
    if (ch == '"' || ch == '\\') ch = '_';
  return key;
}

int cm_autotune(cm_batch h, const float* y, const char* cache_path,
                hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y) return fail(CM_EINVAL, "y must be a device pointer");
  if (!h->params_set) return fail(CM_ESTATE, "cm_set_params was not called");
  if (int rc = select_device(h)) return rc;
  const std::string key = sanitize_key(
      device_key(h) + "|tets" + std::to_string(h->n_tets) + "|tiles" +
      std::to_string(h->n_tiles) + "|tile" + std::to_string(h->tile_tets) + "|nloc" +
      std::to_string(h->T.nloc) + (h->is_template ? "|template" : "") + kTuneObjective);
  int w = 0, b = 0;
  if (cache_path && cache_lookup(cache_path, key, &w, &b))
    return cm_set_launch(h, w, b);
  double best_ms = INFINITY;
  if (int rc = tune_launch(h, y, stream, &best_ms)) return rc;
  if (cache_path) {
    cm_get_launch(h, &w, &b);
    cache_store(cache_path, key, w, b, best_ms);
  }
  return CM_OK;
}

int cm_batch_create_tuned(int32_t n_cells, const int64_t* node_off,
                          const int64_t* tet_off, const double* ref_xyz,
                          const int32_t* tets, const cm_options* opt,
                          const int32_t* tile_candidates, int32_t n_candidates,
                          const char* cache_path, double* candidate_ms,
                          hipStream_t stream, cm_batch* out) {
  g_err.clear();
  if (!out) return fail(CM_EINVAL, "out is null");
  *out = nullptr;
  static const int32_t kDefault[5] = {512, 640, 768, 896, 1024};
  if (!tile_candidates) {
    tile_candidates = kDefault;
    n_candidates = 5;
  }
  if (n_candidates < 1 || n_candidates > 64)
    return fail(CM_EINVAL, "n_candidates must lie in [1, 64]");
  for (int32_t k = 0; k < n_candidates; ++k) {
    const int32_t t = tile_candidates[k];
    if (t < 64 || t > cm::kMaxTileTets || t % 64 != 0)
      return fail(CM_EINVAL, "tile candidates must be multiples of 64 in [64, 4096]");
  }
  if (candidate_ms)
    for (int32_t k = 0; k < n_candidates; ++k) candidate_ms[k] = INFINITY;
  if (n_cells < 1 || !node_off || !tet_off)
    return fail(CM_EINVAL, "null offsets or no cell");
  const cm::PrepOptions base = prep_options(opt);
  // cache key: device, mesh sizes, ordering and the candidate list
  int dev = 0;
  CM_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  CM_HIP(hipGetDeviceProperties(&prop, dev));
  std::string key = std::string(prop.gcnArchName) + "|cu" +
                    std::to_string(prop.multiProcessorCount) + "|cells" +
                    std::to_string(n_cells) + "|nodes" + std::to_string(node_off[n_cells]) +
                    "|tets" + std::to_string(tet_off[n_cells]) + "|order" +
                    std::to_string(base.order) + "|cand";
  for (int32_t k = 0; k < n_candidates; ++k) key += "," + std::to_string(tile_candidates[k]);
  key = sanitize_key(key + kTuneObjective);
  int cw = 0, cb = 0, ct = 0;
  if (cache_path && cache_lookup_tile(cache_path, key, &cw, &cb, &ct)) {
    cm::PrepOptions po = base;
    po.tile_tets = ct;
    cm::Prepared P;
    std::string err;
    int rc = cm::prepare_batch(n_cells, node_off, tet_off, ref_xyz, tets, nullptr, 1, po,
                               &P, &err);
    if (rc != CM_OK) return fail(rc, err);
    cm_batch h = nullptr;
    if ((rc = create_from(P, po, stream, &h)) != CM_OK) return rc;
    if ((rc = cm_set_launch(h, cw, cb)) != CM_OK) {
      cm_destroy(h);
      return rc;
    }
    *out = h;
    return CM_OK;
  }
  cm_batch best = nullptr;
  double best_ms = INFINITY;
  float* y = nullptr;
  for (int32_t k = 0; k < n_candidates; ++k) {
    cm::PrepOptions po = base;
    po.tile_tets = tile_candidates[k];
    cm::Prepared P;
    std::string err;
    int rc = cm::prepare_batch(n_cells, node_off, tet_off, ref_xyz, tets, nullptr, 1, po,
                               &P, &err);
    if (rc != CM_OK) {
      if (best) cm_destroy(best);
      return fail(rc, err);
    }
    cm_batch h = nullptr;
    if ((rc = create_from(P, po, stream, &h)) != CM_OK) {
      if (best) cm_destroy(best);
      return rc;
    }
    // timing input: the reference positions (float32, internal order) and
    // unit parameters; neither changes the work done per tetrahedron
    const size_t N = (size_t)h->n_nodes;
    std::vector<float> ys(3 * N);
    for (size_t g = 0; g < N; ++g)
      for (int c = 0; c < 3; ++c) ys[c * N + g] = (float)ref_xyz[3 * h->new_to_old[g] + c];
    std::vector<double> mu(h->n_mat, 1.0), ka(h->n_mat, 10.0), w(h->n_mat, 0.5);
    double ms = INFINITY;
    if (hipMalloc((void**)&y, 3 * N * sizeof(float)) != hipSuccess) {
      y = nullptr;
      rc = fail(CM_ENOMEM, "autotune input allocation failed");
    } else if (hipMemcpy(y, ys.data(), 3 * N * sizeof(float), hipMemcpyHostToDevice) !=
               hipSuccess) {
      rc = fail(CM_EHIP, "autotune input copy failed");
    } else if ((rc = cm_set_params(h, mu.data(), ka.data(), w.data(), 0, stream)) == CM_OK) {
      rc = tune_launch(h, y, stream, &ms);
    }
    if (y) (void)hipFree(y);
    y = nullptr;
    h->params_set = false;  // the caller sets the real parameters
    if (rc == CM_EINVAL && k + 1 < n_candidates) {
      // a candidate whose tiles exceed the LDS for every launch is skipped
      cm_destroy(h);
      continue;
    }
    if (rc != CM_OK) {
      cm_destroy(h);
      if (best) cm_destroy(best);
      return rc;
    }
    if (candidate_ms) candidate_ms[k] = ms;
    if (ms < best_ms) {
      if (best) cm_destroy(best);
      best = h;
      best_ms = ms;
    } else {
      cm_destroy(h);
    }
  }
  if (!best) return fail(CM_EINVAL, "no tile candidate fits in LDS");
  if (cache_path) {
    int bw = 0, bb = 0;
    cm_get_launch(best, &bw, &bb);
    cache_store_tile(cache_path, key, bw, bb, best->tile_tets, best_ms);
  }
  *out = best;
  return CM_OK;
}

int cm_plate_step(cm_batch h, const float* y, const float* f,
                  const double* plate, double k_plate, double mobility,
                  float* y_next, double* force, hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !f || !plate || !y_next)
    return fail(CM_EINVAL, "y, f, plate and y_next must be device pointers");
  if (y_next == y || y_next == f)
    return fail(CM_EINVAL, "y_next may not alias y or f");
  if (!std::isfinite(k_plate) || !std::isfinite(mobility) || k_plate < 0 || mobility < 0)
    return fail(CM_EINVAL, "k_plate and mobility must be finite and >= 0");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_plate_step(h->d_node_off, h->n_nodes, (int32_t)h->n_cells, y,
                               f, plate, k_plate, mobility, y_next, force, stream));
  return CM_OK;
}

int cm_qs_set_indenter(cm_batch h, double radius, const double* axis_xy,
                       hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!(radius >= 0.0) || !std::isfinite(radius))
    return fail(CM_EINVAL, "radius must be finite and >= 0");
  if (radius > 0.0 && !axis_xy)
    return fail(CM_EINVAL, "a sphere needs axis_xy (device float64[2 n_cells])");
  if (int rc = select_device(h)) return rc;
  if (radius > 0.0) {
    if (!h->qs_ind.axis) {
      double *ax, *geo;
      int rc;
      if ((rc = h->alloc(&ax, 2 * (size_t)h->n_cells)) ||
          (rc = h->alloc(&geo, 3 * (size_t)h->n_cells)))
        return rc;
      CM_HIP(hipMemsetAsync(geo, 0, 3 * (size_t)h->n_cells * sizeof(double), stream));
      h->qs_ind.axis = ax;
      h->qs_ind.geo = geo;
    }
    CM_HIP(hipMemcpyAsync(const_cast<double*>(h->qs_ind.axis), axis_xy,
                          2 * (size_t)h->n_cells * sizeof(double), hipMemcpyDeviceToDevice,
                          stream));
  }
  h->qs_ind.R = radius;
  return CM_OK;
}

int cm_qs_residual(cm_batch h, const float* y, const float* f, const double* energy,
                   const double* plate, double k_plate, double abs_tol,
                   double rel_tol, double step_tol, double floor_factor,
                   double eta_max, int32_t restart, float* r, float* p, float* x,
                   float* r_newton, double* state, double* force, const float* k_el,
                   float* minv, hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !f || !plate || !r || !p || !x || !state)
    return fail(CM_EINVAL, "y, f, plate, r, p, x and state must be device pointers");
  if ((k_el == nullptr) != (minv == nullptr))
    return fail(CM_EINVAL, "k_el and minv must both be given or both be null");
  if (!std::isfinite(k_plate) || k_plate < 0 || !(abs_tol >= 0) || !(rel_tol >= 0) ||
      !(step_tol >= 0) || !(floor_factor >= 0))
    return fail(CM_EINVAL, "k_plate and tolerances must be finite and >= 0");
  if (!(eta_max >= 0 && eta_max < 1))
    return fail(CM_EINVAL, "eta_max must lie in [0, 1)");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_qs_residual(h->d_node_off, h->n_nodes, (int32_t)h->n_cells, y, f,
                                energy, plate, k_plate, abs_tol, rel_tol, step_tol,
                                floor_factor, eta_max, restart ? 1 : 0, r, p, x,
                                r_newton, state, force, k_el, minv, stream, h->qs_ind));
  return CM_OK;
}

int cm_qs_ls_start(cm_batch h, float* x, const float* r_newton, double cap,
                   const float* y, float* y_trial, double* state,
                   hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!x || !r_newton || !y || !y_trial || !state || y_trial == y)
    return fail(CM_EINVAL, "x, r_newton, y, y_trial (distinct from y) and state "
                           "must be device pointers");
  if (!(cap > 0) || !std::isfinite(cap)) return fail(CM_EINVAL, "cap must be finite and > 0");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_qs_ls_start(h->d_node_off, h->n_nodes, (int32_t)h->n_cells, x,
                                r_newton, cap, y, y_trial, state, stream));
  return CM_OK;
}

int cm_qs_ls_accept(cm_batch h, const float* x, const double* plate, double k_plate,
                    const double* energy_trial, double armijo, double min_move,
                    float* y, float* y_trial, double* state,
                    const int32_t* n_inverted_trial, int32_t* n_inverted,
                    hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!x || !plate || !energy_trial || !y || !y_trial || !state || y_trial == y)
    return fail(CM_EINVAL, "x, plate, energy_trial, y, y_trial (distinct from y) "
                           "and state must be device pointers");
  if ((n_inverted_trial == nullptr) != (n_inverted == nullptr))
    return fail(CM_EINVAL, "n_inverted_trial and n_inverted must both be given or "
                           "both be null");
  if (!std::isfinite(k_plate) || k_plate < 0 || !(armijo >= 0) || !(armijo < 1) ||
      !(min_move >= 0))
    return fail(CM_EINVAL, "k_plate >= 0, 0 <= armijo < 1 and min_move >= 0 required");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_qs_ls_accept(h->d_node_off, h->n_nodes, (int32_t)h->n_cells, x,
                                 plate, k_plate, energy_trial, armijo, min_move, y,
                                 y_trial, state, n_inverted_trial, n_inverted, stream,
                                 h->qs_ind));
  return CM_OK;
}

int cm_qs_noise(cm_batch h, const float* y, float* e, hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !e || e == y) return fail(CM_EINVAL, "y and e must be distinct device pointers");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_qs_noise(h->d_node_off, h->n_nodes, (int32_t)h->n_cells, y, e, stream));
  return CM_OK;
}

int cm_qs_floor(cm_batch h, const float* y, const double* plate, double k_plate,
                const float* e, const float* ybar, double* state, hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !plate || !e || !ybar || !state)
    return fail(CM_EINVAL, "y, plate, e, ybar and state must be device pointers");
  if (!std::isfinite(k_plate) || k_plate < 0)
    return fail(CM_EINVAL, "k_plate must be finite and >= 0");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_qs_floor(h->d_node_off, h->n_nodes, (int32_t)h->n_cells, y, plate,
                             k_plate, e, ybar, state, stream, h->qs_ind));
  return CM_OK;
}

int cm_qs_adjoint_rhs(cm_batch h, const float* y, const double* plate, double k_plate,
                      const double* weight, float* r, float* p, float* x, double* state,
                      const float* minv, hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !plate || !r || !p || !x || !state)
    return fail(CM_EINVAL, "y, plate, r, p, x and state must be device pointers");
  if (!std::isfinite(k_plate) || k_plate < 0)
    return fail(CM_EINVAL, "k_plate must be finite and >= 0");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_qs_adjoint_rhs(h->d_node_off, h->n_nodes, (int32_t)h->n_cells, y,
                                   plate, k_plate, weight, r, p, x, state, minv, stream,
                                   h->qs_ind));
  return CM_OK;
}

int cm_qs_stiffness(cm_batch h, float* k_el, hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!k_el) return fail(CM_EINVAL, "k_el must be a device pointer");
  if (!h->params_set) return fail(CM_ESTATE, "cm_set_params was not called");
  if ((size_t)16 * h->T.nloc > 65536)
    return fail(CM_EINVAL, "tiles too large for the stiffness kernel's LDS");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_qs_stiffness(h->T, full_range(h), k_el, stream));
  return CM_OK;
}

int cm_qs_cg_step(cm_batch h, const float* y, const double* plate, double k_plate,
                  double rel_tol, const float* ybar, float* x, float* r, float* p,
                  float* Ap, double* state, const float* minv, hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !plate || !ybar || !x || !r || !p || !Ap || !state)
    return fail(CM_EINVAL, "all arrays must be device pointers");
  if (!std::isfinite(k_plate) || k_plate < 0 || !(rel_tol >= 0))
    return fail(CM_EINVAL, "k_plate and rel_tol must be finite and >= 0");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_qs_cg(h->d_node_off, h->n_nodes, (int32_t)h->n_cells, y, plate,
                          k_plate, rel_tol, ybar, x, r, p, Ap, state, minv, stream,
                          nullptr, h->qs_ind));
  return CM_OK;
}

int cm_qs_cg_iteration(cm_batch h, const float* y, const double* plate, double k_plate,
                       double rel_tol, float* ybar, float* x, float* r, float* p,
                       float* Ap, double* state, const float* minv, hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !plate || !ybar || !x || !r || !p || !Ap || !state)
    return fail(CM_EINVAL, "y, plate, ybar, x, r, p, Ap and state must be device pointers");
  if (!std::isfinite(k_plate) || k_plate < 0 || !(rel_tol >= 0))
    return fail(CM_EINVAL, "k_plate and rel_tol must be finite and >= 0");
  if (!h->params_set) return fail(CM_ESTATE, "cm_set_params was not called");
  if (!lds_fits(h, h->cfg.waves, true))
    return fail(CM_EINVAL, "launch configuration exceeds 64 KiB of LDS");
  if (int rc = select_device(h)) return rc;
  // the Hessian-vector product of the cells still in CG (state column 2),
  // tile pass only: owned nodes into ybar, shared nodes as slot partials
  const cm::CellMask mask{state + 2, cm::kQsState};
  CM_HIP(cm::launch_backward_main(h->Tb, full_range(h), h->cfg, y, p, nullptr, ybar,
                                  stream, mask, cm::PlateBwd{}, false));
  CM_HIP(cm::launch_qs_cg(h->d_node_off, h->n_nodes, (int32_t)h->n_cells, y, plate,
                          k_plate, rel_tol, ybar, x, r, p, Ap, state, minv, stream,
                          &h->Tb, h->qs_ind));
  return CM_OK;
}

int cm_qs_update(cm_batch h, const float* x, double cap, float* y, double* state,
                 hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!x || !y || !state) return fail(CM_EINVAL, "x, y and state must be device pointers");
  if (!(cap > 0) || !std::isfinite(cap)) return fail(CM_EINVAL, "cap must be finite and > 0");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_qs_update(h->d_node_off, h->n_nodes, (int32_t)h->n_cells, x, cap, y,
                              state, stream));
  return CM_OK;
}

int cm_qs_predict(cm_batch h, const double* plate_old, const double* plate_new,
                  float* y, hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!plate_old || !plate_new || !y)
    return fail(CM_EINVAL, "plate_old, plate_new and y must be device pointers");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_qs_predict(h->d_node_off, h->n_nodes, (int32_t)h->n_cells,
                               plate_old, plate_new, y, stream));
  return CM_OK;
}

int cm_plate_step_adjoint(cm_batch h, const float* y, const float* lam_next,
                          const float* ybar_el, const double* plate,
                          double k_plate, double mobility,
                          const double* F_meas, const double* F_target,
                          double scale, const double* thetabar_el,
                          double* thetabar_acc, float* lam,
                          hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !lam_next || !ybar_el || !plate || !lam)
    return fail(CM_EINVAL, "y, lam_next, ybar_el, plate and lam must be device pointers");
  if (lam == lam_next || lam == ybar_el || lam == y)
    return fail(CM_EINVAL, "lam may not alias the inputs");
  if (F_target && !F_meas) return fail(CM_EINVAL, "F_target needs F_meas");
  if ((thetabar_el == nullptr) != (thetabar_acc == nullptr))
    return fail(CM_EINVAL, "thetabar_el and thetabar_acc go together");
  if (!std::isfinite(k_plate) || !std::isfinite(mobility) || k_plate < 0 || mobility < 0)
    return fail(CM_EINVAL, "k_plate and mobility must be finite and >= 0");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_plate_adjoint(h->d_node_off, h->n_nodes, (int32_t)h->n_cells,
                                  y, lam_next, ybar_el, plate, k_plate, mobility,
                                  F_meas, F_target, scale, thetabar_el,
                                  thetabar_acc, h->n_regions, lam, stream));
  return CM_OK;
}

int cm_plate_forces_step(cm_batch h, const float* y, const double* plate,
                         double k_plate, double mobility, float* y_next,
                         double* force, double* energy, int32_t* n_inverted,
                         hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !plate || !y_next)
    return fail(CM_EINVAL, "y, plate and y_next must be device pointers");
  if (y_next == y) return fail(CM_EINVAL, "y_next may not alias y");
  if (!std::isfinite(k_plate) || !std::isfinite(mobility) || k_plate < 0 || mobility < 0)
    return fail(CM_EINVAL, "k_plate and mobility must be finite and >= 0");
  if (!h->params_set) return fail(CM_ESTATE, "cm_set_params was not called");
  if (!lds_fits(h, h->cfg.waves, false))
    return fail(CM_EINVAL, "launch configuration exceeds 64 KiB of LDS");
  if (int rc = select_device(h)) return rc;
  cm::PlateFwd pl;
  pl.plate = plate;
  pl.k = (float)k_plate;
  pl.m = (float)mobility;
  pl.y_next = y_next;
  pl.force = force;
  CM_HIP(cm::launch_forward(h->T, full_range(h), h->cfg, y, nullptr, energy, n_inverted,
                            stream, pl));
  return CM_OK;
}

int cm_plate_backward_step(cm_batch h, const float* y, const float* lam_next,
                           const double* plate, double k_plate, double mobility,
                           const double* F_meas, const double* F_target,
                           double scale, double* thetabar_acc, float* lam,
                           hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !lam_next || !plate || !lam)
    return fail(CM_EINVAL, "y, lam_next, plate and lam must be device pointers");
  if (lam == lam_next || lam == y) return fail(CM_EINVAL, "lam may not alias the inputs");
  if (F_target && !F_meas) return fail(CM_EINVAL, "F_target needs F_meas");
  if (!std::isfinite(k_plate) || !std::isfinite(mobility) || k_plate < 0 ||
      mobility < 0 || !std::isfinite(scale))
    return fail(CM_EINVAL, "k_plate and mobility must be finite and >= 0, scale finite");
  if (!h->params_set) return fail(CM_ESTATE, "cm_set_params was not called");
  if (!lds_fits(h, h->cfg.waves, true))
    return fail(CM_EINVAL, "launch configuration exceeds 64 KiB of LDS");
  if (int rc = select_device(h)) return rc;
  cm::PlateBwd pl;
  pl.plate = plate;
  pl.k = (float)k_plate;
  pl.m = (float)mobility;
  pl.m64 = mobility;
  pl.F_meas = F_meas;
  pl.F_target = F_target;
  pl.scale = scale;
  pl.thetabar_acc = thetabar_acc;
  pl.lam = lam;
  CM_HIP(cm::launch_backward(h->Tb, full_range(h), h->cfg, y, lam_next, nullptr, nullptr,
                             nullptr, stream, cm::CellMask{}, pl));
  return CM_OK;
}

int cm_shape(cm_batch h, const float* y, const double* d_ref, double* out,
             hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !out) return fail(CM_EINVAL, "y and out must be device pointers");
  if (cm::shape_lds(h->T.nloc) > 65536)
    return fail(CM_EINVAL, "tiles too large for the shape kernel's LDS");
  if (int rc = select_device(h)) return rc;
  CM_HIP(cm::launch_shape(h->T, h->d_node_off, h->cand_blocks, h->n_cand_blocks,
                          h->node_blocks, h->n_node_blocks, h->space_order, y, d_ref,
                          h->chunk_neg, h->shape_mom, h->shape_tile_inv, h->shape_cell_inv,
                          h->shape_bbox, h->d2max, out, stream));
  return CM_OK;
}

int cm_profile_kernels(cm_batch h, const float* y, float* f, double* energy,
                       const float* fbar, const double* ebar, float* ybar,
                       double* thetabar, int32_t reps, double* ms,
                       hipStream_t st) {
  if (int rc = check_handle(h)) return rc;
  if (!y || !f || !ybar || !ms || reps <= 0)
    return fail(CM_EINVAL, "y, f, ybar, ms must be non-null and reps > 0");
  if (!h->params_set) return fail(CM_ESTATE, "cm_set_params was not called");
  if (!lds_fits(h, h->cfg.waves, true) || !lds_fits(h, h->cfg.waves, false))
    return fail(CM_EINVAL, "launch configuration exceeds 64 KiB of LDS");
  if (int rc = select_device(h)) return rc;
  const cm::Range r = full_range(h);
  cm::LaunchCfg fcfg;
  const bool fused = fused_cfg(h, &fcfg) && f != ybar && f != y && ybar != y &&
                     (!fbar || (f != fbar && ybar != fbar));
  hipEvent_t ev[7];
  for (int i = 0; i < 7; ++i) CM_HIP(hipEventCreate(&ev[i]));
  int rc = CM_OK;
  for (int k = 0; k < 6 && rc == CM_OK; ++k) {
    if (k >= 4 && !fused) {
      ms[k] = NAN;
      continue;
    }
    auto once = [&]() -> hipError_t {
      switch (k) {
        case 0: return cm::launch_forward_main(h->T, r, h->cfg, y, f, st);
        case 1: return cm::launch_forward_finalize(h->T, r, f, energy, nullptr, st);
        case 2: return cm::launch_backward_main(h->Tb, r, h->cfg, y, fbar, ebar, ybar, st);
        case 3: return cm::launch_backward_finalize(h->Tb, r, ybar, thetabar, st);
        case 4:
          return cm::launch_forward_backward_main(h->T, h->Tb, r, fcfg, y, f, fbar, ebar,
                                                  ybar, st);
        default:
          return cm::launch_forward_backward_finalize(h->T, h->Tb, r, f, energy, nullptr,
                                                      ybar, thetabar, st);
      }
    };
    hipError_t e = once();  // warm-up
    if (e == hipSuccess) e = hipEventRecord(ev[k], st);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = once();
    if (e == hipSuccess) e = hipEventRecord(ev[k + 1], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[k + 1]);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
    if (e != hipSuccess) rc = fail(CM_EHIP, std::string("profile: ") + hipGetErrorString(e));
    ms[k] = (double)t / reps;
  }
  for (int i = 0; i < 7; ++i) (void)hipEventDestroy(ev[i]);
  return rc;
}

int cm_graph_capture(cm_batch h, int mode, const float* y, float* f,
                     double* energy, int32_t* n_inverted, const float* fbar,
                     const double* ebar, float* ybar, double* thetabar,
                     hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (mode < 0 || mode > 6) return fail(CM_EINVAL, "mode must be 0..6");
  if (!stream) return fail(CM_EINVAL, "capture needs a non-null stream");
  if (int rc = select_device(h)) return rc;
  if (h->graph_exec) { (void)hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; }
  if (h->graph) { (void)hipGraphDestroy(h->graph); h->graph = nullptr; }
  CM_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  const bool percell = mode == 2 || mode == 3 || mode == 5;
  const bool bwd = mode == 1 || mode == 3 || mode == 4 || mode == 5;
  const bool fork = mode == 4 || mode == 5;
  const bool fused = mode == 6;
  int rc = CM_OK;
  hipError_t e = hipSuccess;
  if (fused) {
    rc = forward_backward_impl(h, y, f, energy, n_inverted, fbar, ebar, ybar, thetabar,
                               stream);
  } else if (fork) {
    // The backward pass reads y, fbar, ebar only (never the forward's
    // outputs) and uses its own scratch, so it can be a parallel branch.
    e = hipEventRecord(h->ev_fork, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->side, h->ev_fork, 0);
    if (e == hipSuccess)
      rc = backward_impl(h, y, fbar, ebar, ybar, thetabar, h->side, percell);
  }
  if (!fused && e == hipSuccess && rc == CM_OK)
    rc = forces_impl(h, y, f, energy, n_inverted, stream, percell);
  if (bwd && !fork && rc == CM_OK)
    rc = backward_impl(h, y, fbar, ebar, ybar, thetabar, stream, percell);
  if (fork && e == hipSuccess) {
    e = hipEventRecord(h->ev_join, h->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(stream, h->ev_join, 0);
  }
  if (e != hipSuccess && rc == CM_OK)
    rc = fail(CM_EHIP, std::string("graph fork/join: ") + hipGetErrorString(e));
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(stream, &g);
  if (rc != CM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(CM_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  h->graph = g;
  CM_HIP(hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0));
  return CM_OK;
}

int cm_graph_launch(cm_batch h, hipStream_t stream) {
  if (int rc = check_handle(h)) return rc;
  if (!h->graph_exec) return fail(CM_ESTATE, "no graph captured");
  CM_HIP(hipGraphLaunch(h->graph_exec, stream));
  return CM_OK;
}

struct cm_layout_s {
  cm::Prepared P;
  int32_t tile_tets;
};

int cm_layout_create(int32_t n_cells, const int64_t* node_off,
                     const int64_t* tet_off, const double* ref_xyz,
                     const int32_t* tets, const cm_options* opt,
                     cm_layout* out) {
  return cm_layout_create_regions(n_cells, node_off, tet_off, ref_xyz, tets,
                                  nullptr, 1, opt, out);
}

int cm_layout_create_regions(int32_t n_cells, const int64_t* node_off,
                             const int64_t* tet_off, const double* ref_xyz,
                             const int32_t* tets, const uint8_t* tet_region,
                             int32_t n_regions, const cm_options* opt,
                             cm_layout* out) {
  g_err.clear();
  if (!out) return fail(CM_EINVAL, "out is null");
  *out = nullptr;
  cm_layout_s* l = new (std::nothrow) cm_layout_s();
  if (!l) return fail(CM_ENOMEM, "host allocation failed");
  const cm::PrepOptions po = prep_options(opt);
  std::string err;
  int rc = cm::prepare_batch(n_cells, node_off, tet_off, ref_xyz, tets, tet_region,
                             n_regions, po, &l->P, &err);
  if (rc != CM_OK) {
    delete l;
    return fail(rc, err);
  }
  l->tile_tets = po.tile_tets;
  *out = l;
  return CM_OK;
}

int cm_layout_create_template(int32_t n_cells, int64_t n_nodes, int64_t n_tets,
                              const double* ref_xyz, const int32_t* tets,
                              const cm_options* opt, cm_layout* out) {
  g_err.clear();
  if (!out) return fail(CM_EINVAL, "out is null");
  *out = nullptr;
  if (!ref_xyz || !tets || n_nodes < 0 || n_tets < 0)
    return fail(CM_EINVAL, "null pointer or negative size");
  cm_layout_s* l = new (std::nothrow) cm_layout_s();
  if (!l) return fail(CM_ENOMEM, "host allocation failed");
  const cm::PrepOptions po = prep_options(opt);
  std::string err;
  int rc = cm::prepare_template(n_cells, n_nodes, n_tets, ref_xyz, tets, nullptr, 1,
                                po, &l->P, &err);
  if (rc != CM_OK) {
    delete l;
    return fail(rc, err);
  }
  l->tile_tets = po.tile_tets;
  *out = l;
  return CM_OK;
}

int cm_layout_sizes(cm_layout l, int64_t* s) {
  if (!l || !s) return fail(CM_EINVAL, "null argument");
  s[0] = (int64_t)l->P.tiles.size();
  s[1] = (int64_t)l->P.chunks.size();
  s[2] = (int64_t)l->P.slot_node.size();
  s[3] = (int64_t)l->P.shared_node.size();
  s[4] = l->P.n_nodes;
  s[5] = l->P.n_cells;
  s[6] = l->P.max_tile_nodes;
  s[7] = l->tile_tets;
  return CM_OK;
}

int cm_layout_export(cm_layout l, int32_t* tiles, void* chunks,
                     int32_t* slot_node, int32_t* shared_node,
                     int32_t* shared_slot_ptr, int32_t* shared_slots,
                     int32_t* cell_tile_off, int32_t* cell_shared_off,
                     int64_t* new_to_old) {
  if (!l) return fail(CM_EINVAL, "null layout");
  const cm::Prepared& P = l->P;
  auto cp = [](void* dst, const void* src, size_t bytes) {
    if (dst && bytes) std::memcpy(dst, src, bytes);
  };
  cp(tiles, P.tiles.data(), P.tiles.size() * sizeof(cm::TileDesc));
  cp(chunks, P.chunks.data(), P.chunks.size() * sizeof(cm::TetChunk));
  cp(slot_node, P.slot_node.data(), P.slot_node.size() * 4);
  cp(shared_node, P.shared_node.data(), P.shared_node.size() * 4);
  cp(shared_slot_ptr, P.shared_slot_ptr.data(), P.shared_slot_ptr.size() * 4);
  cp(shared_slots, P.shared_slots.data(), P.shared_slots.size() * 4);
  cp(cell_tile_off, P.cell_tile_off.data(), P.cell_tile_off.size() * 4);
  cp(cell_shared_off, P.cell_shared_off.data(), P.cell_shared_off.size() * 4);
  cp(new_to_old, P.new_to_old.data(), P.new_to_old.size() * 8);
  return CM_OK;
}

int cm_layout_export_regions(cm_layout l, int32_t* tile_mat,
                             int32_t* mat_tile_first, int32_t* mat_tile_count) {
  if (!l) return fail(CM_EINVAL, "null layout");
  const cm::Prepared& P = l->P;
  auto cp = [](void* dst, const void* src, size_t bytes) {
    if (dst && bytes) std::memcpy(dst, src, bytes);
  };
  cp(tile_mat, P.tile_mat.data(), P.tile_mat.size() * 4);
  cp(mat_tile_first, P.mat_tile_first.data(), P.mat_tile_first.size() * 4);
  cp(mat_tile_count, P.mat_tile_count.data(), P.mat_tile_count.size() * 4);
  return CM_OK;
}

int cm_layout_destroy(cm_layout l) {
  delete l;
  return CM_OK;
}

}  // extern "C"
