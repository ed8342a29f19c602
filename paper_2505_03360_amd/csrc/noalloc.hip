// bz_collide_batch_noalloc: the collision evaluation of bz_collide_batch with
// its workspace in a static device array instead of a bound workspace, for
// callers that cannot allocate device memory.
#include <algorithm>
#include <mutex>

#include "bz_internal.hpp"

// Workspace of bz_collide_batch_noalloc: one static array per device, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (in host code the name is a host-side stand-in); it uses the device
// address hipGetSymbolAddress returns, looked up once per device with that
// device current.
static constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

bz_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return bz::fail(BZ_ERR_DEVICE, "bz_collide_batch_noalloc: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return bz::fail(BZ_ERR_UNSUPPORTED, "bz_collide_batch_noalloc: device %d", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return bz::fail(BZ_ERR_DEVICE, "bz_collide_batch_noalloc: scratch address: %s", hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return BZ_OK;
}

}  // namespace

extern "C" bz_status bz_collide_batch_noalloc(const bz_plan* p, const void* f, int32_t f_dtype, const int32_t* idx,
                                              int32_t ncells, const int32_t* ncells_dev, void* q, int32_t flags,
                                              void* stream) {
  bz::clear_error();
  if (!p) return bz::fail(BZ_ERR_ARG, "bz_collide_batch_noalloc: null plan");
  if (ncells < 0) return bz::fail(BZ_ERR_ARG, "bz_collide_batch_noalloc: ncells < 0");
  if (ncells == 0) return BZ_OK;
  if (!f || !q) return bz::fail(BZ_ERR_ARG, "bz_collide_batch_noalloc: null f or q");
  if (f_dtype != BZ_FP32 && f_dtype != BZ_FP64) return bz::fail(BZ_ERR_ARG, "bz_collide_batch_noalloc: bad f_dtype");
  if (flags & ~int32_t(BZ_SCATTER)) return bz::fail(BZ_ERR_ARG, "bz_collide_batch_noalloc: unknown flags");
  if ((flags & BZ_SCATTER) && !idx) return bz::fail(BZ_ERR_ARG, "bz_collide_batch_noalloc: BZ_SCATTER needs idx");
  const size_t need = p->ws_fixed + p->ws_per_cell * size_t(ncells);
  if (need > kScratchBytes)
    return bz::fail(BZ_ERR_NOMEM, "bz_collide_batch_noalloc: %d cells need %zu workspace bytes, above the %zu-byte "
                    "static scratch (at most %zu cells of this plan)", int(ncells), need, kScratchBytes,
                    (kScratchBytes - std::min(kScratchBytes, p->ws_fixed)) / p->ws_per_cell);
  if (!p->tables_dev) return bz::fail(BZ_ERR_STATE, "bz_collide_batch_noalloc: plan tables not bound");
  void* ws = nullptr;
  const bz_status st = scratch_address(&ws);
  if (st != BZ_OK) return st;
  const bz::Binding b = bz::make_binding(p, p->tables_dev, ws, need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  bz::launch_clear_status(b.ws, b.lay, s);  // the one region that must start at zero
  return bz::launch_collide(p, b, f, f_dtype == BZ_FP32, idx, ncells, ncells_dev, q, (flags & BZ_SCATTER) != 0, s,
                            false);
}
