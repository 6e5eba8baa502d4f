// Staging of launch descriptors that the host builds (batched render views, batched ICP
// requests): a small ring of slots per device, each a pinned host block, a device block and
// an event.  A call fills the host block, copies it to the device block on its stream,
// launches the kernels that read it and records the slot's event behind them; the slot is
// handed out again only once that event has completed.  The host memory handed to the
// asynchronous copy therefore lives until the copy has run, whatever the caller does after
// the call returns, and the descriptors of calls in flight on different streams never share
// memory.
#include <mutex>

#include "dtsdf_internal.hpp"

namespace dtsdf {

namespace {

constexpr int kStageSlots = 8;
constexpr int kMaxDevices = 64;

struct Ring {
  Stage slot[kStageSlots];
  int next = 0;
  bool ready = false;
};

std::mutex g_mu;
Ring g_rings[kMaxDevices];

dtsdf_status init_ring(Ring& r) {
  for (Stage& s : r.slot) {
    if (hipHostMalloc((void**)&s.host, kStageHostBytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&s.dev, kStageDevBytes) != hipSuccess ||
        hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
      return DTSDF_E_NOMEM;
  }
  r.ready = true;
  return DTSDF_OK;
}

}  // namespace

dtsdf_status stage_acquire(Stage** out) {
  *out = nullptr;
  int dev = 0;
  DTSDF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return DTSDF_E_INVAL;
  Stage* s = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    Ring& r = g_rings[dev];
    if (!r.ready) {
      const dtsdf_status st = init_ring(r);
      if (st != DTSDF_OK) return st;
    }
    for (int i = 0; i < kStageSlots && !s; ++i) {
      Stage& c = r.slot[(r.next + i) % kStageSlots];
      if (!c.busy) {
        c.busy = true;
        s = &c;
        r.next = (r.next + i + 1) % kStageSlots;
      }
    }
  }
  // every slot is held by a call between acquire and release (other host threads)
  if (!s) return DTSDF_E_BUSY;
  if (s->recorded && hipEventSynchronize(s->done) != hipSuccess) {
    std::lock_guard<std::mutex> lock(g_mu);
    s->busy = false;
    return DTSDF_E_HIP;
  }
  *out = s;
  return DTSDF_OK;
}

dtsdf_status stage_release(Stage* s, hipStream_t st) {
  const hipError_t e = hipEventRecord(s->done, st);
  std::lock_guard<std::mutex> lock(g_mu);
  s->recorded = e == hipSuccess;
  s->busy = false;
  return e == hipSuccess ? DTSDF_OK : DTSDF_E_HIP;
}

}  // namespace dtsdf
