// cm_forces_noalloc: cm_forces with its scratch memory (the shared-node
// slot partials, the per-tile energies and the per-tile inverted counts) in
// a file-scope device array of fixed size instead of the handle's own
// scratch, for callers that cannot allocate.  Same kernels, same summation
// order: results are bitwise those of cm_forces.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "cellmech.h"
#include "handle.h"
#include "kernels.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;  // CM_NOALLOC_SCRATCH_BYTES

// One copy per GPU, held from module load until the process ends.  In host
// code the name `scratch` is only a host-side stand-in for the symbol: its
// device address comes from hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static_assert(kScratchBytes == CM_NOALLOC_SCRATCH_BYTES, "header constant");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up on the
// first call on that device (with it current) and kept per device.
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" int cm_forces_noalloc(cm_batch h, const float* y, float* f,
                                 double* energy, int32_t* n_inverted,
                                 hipStream_t stream) {
  if (!h) return cm::api_fail(CM_EINVAL, "null handle");
  if (!y || !f) return cm::api_fail(CM_EINVAL, "y and f must be device pointers");
  if (!h->params_set) return cm::api_fail(CM_ESTATE, "cm_set_params was not called");
  if (cm::forward_lds_per_wave(h->T.nloc) * (size_t)h->cfg.waves > 65536)
    return cm::api_fail(CM_EINVAL, "launch configuration exceeds 64 KiB of LDS");
  // scratch: slot partials (3 float per slot), tile energies (float64) and
  // tile inverted counts (int32), each starting on a 256-byte boundary
  const size_t off_acc = align256((size_t)h->n_slots * 3 * sizeof(float));
  const size_t off_ninv = align256(off_acc + (size_t)h->n_tiles * sizeof(double));
  const size_t need = off_ninv + (size_t)h->n_tiles * sizeof(int32_t);
  if (need > kScratchBytes)
    return cm::api_fail(CM_EINVAL,
                        "cm_forces_noalloc: the handle needs " + std::to_string(need) +
                            " bytes of scratch (" + std::to_string(h->n_slots) +
                            " slots, " + std::to_string(h->n_tiles) +
                            " tiles); the static scratch holds " +
                            std::to_string(kScratchBytes) + " bytes (use cm_forces)");
  if (h->device < 0 || h->device >= kMaxDevices)
    return cm::api_fail(CM_EINVAL, "device ordinal beyond the scratch table");
  int cur = 0;
  CM_HIP(hipGetDevice(&cur));
  if (cur != h->device) CM_HIP(hipSetDevice(h->device));
  void* base = nullptr;
  CM_HIP(scratch_address(h->device, &base));
  unsigned char* b = static_cast<unsigned char*>(base);
  cm::DeviceTables T = h->T;  // same read-only tables, scratch replaced
  T.part = reinterpret_cast<float*>(b);
  T.tile_acc = reinterpret_cast<double*>(b + off_acc);
  T.tile_ninv = reinterpret_cast<int32_t*>(b + off_ninv);
  T.tile_plate = nullptr;  // written only by the plate-step pass
  T.tile_nonfin = nullptr;  // written only by the checked pass
  const cm::Range r{0, (int32_t)h->n_tiles, 0, (int32_t)h->n_shared, 0,
                    (int32_t)h->n_cells};
  CM_HIP(cm::launch_forward(T, r, h->cfg, y, f, energy, n_inverted, stream));
  return CM_OK;
}
