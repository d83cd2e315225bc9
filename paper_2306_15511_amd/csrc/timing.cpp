// Optional per-kernel timing with HIP events (crsht_timing_enable /
// crsht_timing_read): the launchers bracket each launch of a tracked kernel
// with two events on the launch stream when timing is on.
#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"

namespace crsht {

void timing_begin(const crsht_plan* Pc, int id, hipStream_t s) {
  crsht_plan* P = const_cast<crsht_plan*>(Pc);
  if (!P->timing.on || id < 0 || id >= kTimedKernels) return;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return;
  }
  (void)hipEventRecord(a, s);
  P->timing.open[id] = a;
  P->timing.open_end[id] = b;
}

void timing_end(const crsht_plan* Pc, int id, hipStream_t s) {
  crsht_plan* P = const_cast<crsht_plan*>(Pc);
  if (!P->timing.on || id < 0 || id >= kTimedKernels || !P->timing.open[id]) return;
  (void)hipEventRecord(P->timing.open_end[id], s);
  P->timing.events[id].push_back({P->timing.open[id], P->timing.open_end[id]});
  P->timing.open[id] = nullptr;
  P->timing.open_end[id] = nullptr;
}

void timing_clear(crsht_plan* P) {
  for (int k = 0; k < kTimedKernels; ++k) {
    for (auto& e : P->timing.events[k]) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    P->timing.events[k].clear();
    P->timing.total_ms[k] = 0.0;
    P->timing.count[k] = 0;
  }
}

}  // namespace crsht

extern "C" int crsht_timing_enable(const crsht_plan* Pc, int on) {
  if (!Pc) return CR_EINVAL;
  crsht_plan* P = const_cast<crsht_plan*>(Pc);
  (void)hipDeviceSynchronize();
  crsht::timing_clear(P);
  P->timing.on = on != 0;
  return CR_OK;
}

extern "C" int crsht_timing_read(const crsht_plan* Pc, int kernel, double* total_ms, int64_t* launches) {
  if (!Pc || !total_ms || !launches || kernel < 0 || kernel >= crsht::kTimedKernels) return CR_EINVAL;
  crsht_plan* P = const_cast<crsht_plan*>(Pc);
  auto& ev = P->timing.events[kernel];
  for (auto& e : ev) {
    if (hipEventSynchronize(e.second) != hipSuccess) return CR_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.first, e.second) != hipSuccess) return CR_EDEVICE;
    P->timing.total_ms[kernel] += ms;
    P->timing.count[kernel] += 1;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  ev.clear();
  *total_ms = P->timing.total_ms[kernel];
  *launches = P->timing.count[kernel];
  return CR_OK;
}
