// Gaussian white draws on the device for the random terms of the
// constrained-realization equation (w0 in harmonic space, w1 in pixel space):
// the counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011) and the Box-Muller
// transform. Every output element is a pure function of (seed, counter,
// column, element), so draws are reproducible and independent of the launch
// shape.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace crsht {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

struct U4 {
  uint32_t x, y, z, w;
};

// ten rounds; round r uses the key bumped r times by (W0, W1)
__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x, p1 = (uint64_t)kPhiloxM1 * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return c;
}

// two standard normals from one block: two uniforms of 53 bits in (0, 1)
// (the high 53 bits of (hi, lo) plus half a unit), Box-Muller
__device__ __forceinline__ void box_muller(U4 b, double& g0, double& g1) {
  const uint64_t a = ((uint64_t)b.x << 32) | b.y, c = ((uint64_t)b.z << 32) | b.w;
  const double u1 = ((double)(a >> 11) + 0.5) * 0x1p-53;
  const double u2 = ((double)(c >> 11) + 0.5) * 0x1p-53;
  const double r = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  g0 = r * cs;
  g1 = r * sn;
}

// counter words: (element, column | purpose << 31, counter lo, counter hi); key = seed
// w0: element i of column c -> (Re, Im) = (g0, g1) / sqrt 2, m = 0: (g0, 0)
__global__ void k_white_alm(int64_t nalm, int nrhs, const int* __restrict__ idx_m, uint32_t k0, uint32_t k1,
                            uint32_t c2, uint32_t c3, double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= nalm || c >= nrhs) return;
  double g0, g1;
  box_muller(philox4x32_10(U4{(uint32_t)i, (uint32_t)c, c2, c3}, k0, k1), g0, g1);
  const double h = 0.70710678118654752440;
  out[(int64_t)c * nalm + i] = idx_m[i] == 0 ? make_double2(g0, 0.0) : make_double2(g0 * h, g1 * h);
}

// w1: pixels 2 j and 2 j + 1 of column c from block j
__global__ void k_white_map(int64_t npix, int nrhs, uint32_t k0, uint32_t k1, uint32_t c2, uint32_t c3,
                            double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (2 * j >= npix || c >= nrhs) return;
  double g0, g1;
  box_muller(philox4x32_10(U4{(uint32_t)j, (uint32_t)c | 0x80000000u, c2, c3}, k0, k1), g0, g1);
  double* o = out + (int64_t)c * npix + 2 * j;
  o[0] = g0;
  if (2 * j + 1 < npix) o[1] = g1;
}

}  // namespace

hipError_t launch_white(const crsht_plan* P, int nrhs, uint64_t seed, uint64_t counter, double2* w0, double* w1,
                        hipStream_t s) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const uint32_t c2 = (uint32_t)counter, c3 = (uint32_t)(counter >> 32);
  const int tb = 256;
  if (w0) {
    const int64_t na = P->g.nalm;
    hipLaunchKernelGGL(k_white_alm, dim3((unsigned)((na + tb - 1) / tb), nrhs), dim3(tb), 0, s, na, nrhs,
                       P->t.idx_m, k0, k1, c2, c3, w0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (w1) {
    const int64_t np = P->g.npix, half = (np + 1) / 2;
    hipLaunchKernelGGL(k_white_map, dim3((unsigned)((half + tb - 1) / tb), nrhs), dim3(tb), 0, s, np, nrhs, k0, k1,
                       c2, c3, w1);
  }
  return hipGetLastError();
}

}  // namespace crsht
