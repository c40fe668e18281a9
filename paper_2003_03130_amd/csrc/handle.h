// Handle of a prepared batch (internal to the library; the C ABI sees an
// opaque pointer).  Shared by the translation units that implement entry
// points.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "cellmech.h"
#include "kernels.h"

namespace cm {

// Records `msg` as this thread's last error (cm_last_error) and returns st.
int api_fail(int st, const std::string& msg);

}  // namespace cm

#define CM_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return cm::api_fail(CM_EHIP, std::string(#call) + ": " +               \
                                       hipGetErrorString(e_));              \
  } while (0)

struct cm_batch_s {
  int device = 0;
  int n_cu = 256;
  int64_t n_cells = 0, n_nodes = 0, n_tets = 0, n_slots = 0, n_shared = 0;
  int64_t n_tiles = 0, n_chunks = 0;
  int32_t n_regions = 1;
  int64_t n_mat = 0;  // material slots: n_cells * n_regions
  // shape diagnostics scratch
  const int4* cand_blocks = nullptr;  // block pairs among candidate nodes
  int64_t n_cand_blocks = 0;
  int32_t* shape_tile_inv = nullptr;
  const uint64_t* chunk_neg = nullptr;  // per chunk: lanes of negative orientation
  int32_t* shape_cell_inv = nullptr;
  const int2* node_blocks = nullptr;
  int64_t n_node_blocks = 0;
  const int32_t* space_order = nullptr;
  double* shape_bbox = nullptr;
  double* shape_mom = nullptr;
  unsigned long long* d2max = nullptr;
  int32_t tile_tets = 0, max_tile_nodes = 0;
  double volume = 0, min_v0 = 0, max_cond = 0;
  std::vector<int32_t> cell_tile_off, cell_shared_off;
  const int64_t* d_node_off = nullptr;  // device copy of the cell node offsets
  std::vector<int64_t> new_to_old;
  std::vector<void*> allocs;
  int64_t device_bytes = 0;
  cm::DeviceTables T;   // tables + forward scratch
  cm::DeviceTables Tb;  // same tables + backward scratch
  cm::LaunchCfg cfg;
  bool params_set = false;
  bool is_template = false;  // cells share one chunk array (tiles interleaved)
  cm::Indenter qs_ind;       // top contact of the quasi-static entry points
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // fork/join of the forward and backward branches of a captured graph
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  ~cm_batch_s() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
    for (void* p : allocs) (void)hipFree(p);
  }

  template <class T>
  int alloc(T** p, size_t count) {
    size_t bytes = std::max<size_t>(sizeof(T) * count, 256);
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e != hipSuccess)
      return cm::api_fail(e == hipErrorOutOfMemory ? CM_ENOMEM : CM_EHIP,
                  std::string("hipMalloc: ") + hipGetErrorString(e));
    allocs.push_back(*p);
    device_bytes += (int64_t)bytes;
    return CM_OK;
  }

  template <class T>
  int upload(T** p, const std::vector<T>& v, hipStream_t st) {
    int rc = alloc(p, v.size());
    if (rc) return rc;
    if (!v.empty())
      CM_HIP(hipMemcpyAsync(*p, v.data(), sizeof(T) * v.size(),
                            hipMemcpyHostToDevice, st));
    return CM_OK;
  }
};
