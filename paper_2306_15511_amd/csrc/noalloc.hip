// sht_synth_noalloc: the synthesis Y of sht_synth for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc). The intermediate buffers of the transform
// (the per-coefficient scaled a_lm and the Legendre sums between the Legendre
// and the ring kernels) live in one file-scope device array instead of the
// plan workspace; the kernels are those of sht_synth.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

using namespace crsht;

namespace {

constexpr size_t kScratchBytes = size_t(96) << 20;   // CRSHT_NOALLOC_SCRATCH_BYTES of crsht.h
constexpr int kMaxDevices = 64;

// One copy per GPU, allocated when the library's code object is loaded on that
// GPU and held until the process ends. In host code `scratch` is only the
// host-side stand-in of the symbol: its device address comes from
// hipGetSymbolAddress (per device) and only that address is used.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
bool g_tried[kMaxDevices] = {};

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

namespace crsht {

// Set-up: the device address of `scratch` on the current device, looked up
// once per device (plan creation calls this with the plan's device current).
int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return CR_ENOTSUP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return CR_OK;
  if (g_tried[device]) return CR_EDEVICE;
  g_tried[device] = true;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return CR_EDEVICE;
  }
  g_ptr[device] = p;
  return CR_OK;
}

}  // namespace crsht

extern "C" int sht_synth_noalloc(const crsht_plan* P, int nrhs, const double* alm, double* map, cr_prec prec,
                                 void* stream) {
  if (!P || !alm || !map) return CR_EINVAL;
  if (nrhs < 1 || nrhs > P->nrhs_max) return CR_EINVAL;
  if (prec != CR_F64 && prec != CR_MIXED) return CR_EINVAL;
  if (P->ncomp != 1) return CR_ENOTSUP;
  if (P->timing.on) return CR_EINVAL;   // kernel timing creates events per launch
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return CR_EDEVICE;
  if (dev != P->device || dev < 0 || dev >= kMaxDevices) return CR_EINVAL;
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    base = g_ptr[dev];
  }
  if (!base) return CR_EDEVICE;   // set-up at plan creation failed on this device
  const Geometry& g = P->g;
  const int64_t eo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;   // complex entries per column
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  unsigned char* sp = static_cast<unsigned char*>(base);
  if (prec == CR_MIXED) {
    // Legendre sums as float2; the a_lm scaling is folded into the operand preparation
    const size_t need = (size_t)nrhs * eo_stride * sizeof(float2);
    if (need > kScratchBytes) return CR_ESCRATCH;
    float2* eo = reinterpret_cast<float2*>(sp);
    if (launch_legendre_synth_mixed(P, nrhs, reinterpret_cast<const double2*>(alm), P->t.rec_kappa, eo, s) !=
        hipSuccess)
      return CR_EDEVICE;
    if (launch_ring(P, nrhs, RING_SYNTH, eo, map, nullptr, nullptr, true, s) != hipSuccess) return CR_EDEVICE;
    return CR_OK;
  }
  const size_t alm_bytes = align256((size_t)nrhs * g.nalm * sizeof(double2));
  const size_t need = alm_bytes + (size_t)nrhs * eo_stride * sizeof(double2);
  if (need > kScratchBytes) return CR_ESCRATCH;
  double2* scaled = reinterpret_cast<double2*>(sp);
  double2* eo = reinterpret_cast<double2*>(sp + alm_bytes);
  if (launch_scale_alm(P, nrhs, reinterpret_cast<const double2*>(alm), P->t.rec_kappa, scaled, s) != hipSuccess)
    return CR_EDEVICE;
  if (launch_legendre_synth(P, nrhs, scaled, eo, s) != hipSuccess) return CR_EDEVICE;
  if (launch_ring(P, nrhs, RING_SYNTH, eo, map, nullptr, nullptr, false, s) != hipSuccess) return CR_EDEVICE;
  return CR_OK;
}
