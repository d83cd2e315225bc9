// Legendre step of the spherical-harmonic transforms, FP64 vector-ALU form.
//
// lambda_lm(z) = Delta_lm P_lm(z) (paper App. A) is evaluated by the standard
// three-term recurrence written for mu_l = lambda_l / kappa_l, which needs one
// multiply and one FMA per step:
//     mu_m = lambda_mm,  mu_{m-1} = 0,  mu_l = (alpha_lm z) mu_{l-1} - mu_{l-2}.
// kappa_lm is folded into the a_lm before synthesis and into the outputs of
// the adjoint. lambda_mm ~ sin^m(theta) underflows near the poles at large m;
// values there carry an integer scale (see kScaleBits) and contribute only
// once they reach the double range.
//
// North/south symmetry lambda_lm(-z) = (-1)^{l+m} lambda_lm(z) (App. A,
// parity of P_lm) lets one recurrence serve a ring and its mirror: synthesis
// produces E (sum over even l-m) and O (odd l-m) per ring pair, the ring
// kernel forms F_N = E + O and F_S = E - O; the adjoint consumes
// G_N + G_S (even l-m) and G_N - G_S (odd l-m).
#include "internal.h"

namespace crsht {
namespace {

constexpr int kSynthBlock = 64;   // ring pairs per block (one wavefront)
constexpr int kSynthMT = 4;       // consecutive m per thread: 4 x (E,O) = 128 contiguous bytes per column
constexpr int kAdjBlock = 256;    // threads per block of the adjoint (one m per block)
constexpr int kAdjOutputs = 16;   // doubles reduced across the block per chunk

__device__ __forceinline__ void rescale(double& v0, double& v1, int& k) {
  if (k < 0 && fabs(v1) > kRescaleAbove) {
    v0 *= kRescaleBy;
    v1 *= kRescaleBy;
    ++k;
  }
}

// ------------------------------------------------------------------ synthesis
template <int NR>
__global__ __launch_bounds__(kSynthBlock) void k_legendre_synth(
    int lmax, int mmax, int npairs, const double* __restrict__ pair_z, const double* __restrict__ alpha,
    const double* __restrict__ lmm_v, const int* __restrict__ lmm_k, const int64_t* __restrict__ mstart,
    const double2* __restrict__ alms, int64_t alm_stride, double2* __restrict__ eo, int64_t eo_stride) {
  const int p = blockIdx.y * kSynthBlock + threadIdx.x;
  const bool valid = p < npairs;
  const int pp = valid ? p : npairs - 1;
  const double z = pair_z[pp];
  const int mfirst = blockIdx.x * kSynthMT;
#pragma unroll 1
  for (int mi = 0; mi < kSynthMT; ++mi) {
    const int m = mfirst + mi;
    if (m > mmax) break;
    const int64_t base = mstart[m];
    const double* __restrict__ al = alpha + base - m;  // al[l] = alpha_lm
    double2 E[NR], O[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) E[c] = O[c] = make_double2(0.0, 0.0);
    double v0 = 0.0;
    double v1 = lmm_v[(size_t)m * npairs + pp];
    int k = lmm_k[(size_t)m * npairs + pp];
    {
      const double w = (k == 0) ? v1 : 0.0;
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        const double2 a = alms[c * alm_stride + base];
        E[c].x = fma(w, a.x, E[c].x);
        E[c].y = fma(w, a.y, E[c].y);
      }
    }
    int l = m + 1;
    // steps while some lane of the wavefront still carries a scaled value
    while (l <= lmax && __any(k < 0)) {
      const double mu = fma(al[l] * z, v1, -v0);
      v0 = v1;
      v1 = mu;
      rescale(v0, v1, k);
      const double w = (k == 0) ? v1 : 0.0;
      const double2* __restrict__ a = alms + base + (l - m);
      if ((l - m) & 1) {
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          O[c].x = fma(w, a[c * alm_stride].x, O[c].x);
          O[c].y = fma(w, a[c * alm_stride].y, O[c].y);
        }
      } else {
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          E[c].x = fma(w, a[c * alm_stride].x, E[c].x);
          E[c].y = fma(w, a[c * alm_stride].y, E[c].y);
        }
      }
      ++l;
    }
    // ordinary doubles from here on; align so each iteration is (odd, even)
    if (l <= lmax && ((l - m) & 1) == 0) {
      const double mu = fma(al[l] * z, v1, -v0);
      v0 = v1;
      v1 = mu;
      const double2* __restrict__ a = alms + base + (l - m);
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        E[c].x = fma(v1, a[c * alm_stride].x, E[c].x);
        E[c].y = fma(v1, a[c * alm_stride].y, E[c].y);
      }
      ++l;
    }
#pragma unroll 2
    for (; l + 1 <= lmax; l += 2) {
      const double a1 = al[l], a2 = al[l + 1];
      const double2* __restrict__ a = alms + base + (l - m);
      const double mu1 = fma(a1 * z, v1, -v0);
      const double mu2 = fma(a2 * z, mu1, -v1);
      v0 = mu1;
      v1 = mu2;
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        const double2 ao = a[c * alm_stride], ae = a[c * alm_stride + 1];
        O[c].x = fma(mu1, ao.x, O[c].x);
        O[c].y = fma(mu1, ao.y, O[c].y);
        E[c].x = fma(mu2, ae.x, E[c].x);
        E[c].y = fma(mu2, ae.y, E[c].y);
      }
    }
    if (l <= lmax) {  // one odd step left
      const double mu = fma(al[l] * z, v1, -v0);
      const double2* __restrict__ a = alms + base + (l - m);
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        O[c].x = fma(mu, a[c * alm_stride].x, O[c].x);
        O[c].y = fma(mu, a[c * alm_stride].y, O[c].y);
      }
    }
    if (valid) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        double2* dst = eo + c * eo_stride + ((size_t)p * (mmax + 1) + m) * 2;
        dst[0] = E[c];
        dst[1] = O[c];
      }
    }
  }
}

// -------------------------------------------------------------------- adjoint
// One block per m. Thread t owns ring pairs t, t + 256, ...; each step adds
// mu_lm(z_p) * G_p over its pairs, and every C steps the block reduces the
// per-thread partial sums through LDS. Output modes:
//   MODE_PLAIN : out = oscale * raw  (oscale = kappa gives Y^T, b kappa gives B Y^T)
//   MODE_AXPY  : out = sinv * pin + bk * raw; partial[c][m] = w_m <pin, out>_m
//   MODE_DIAG  : dout = kept ? sinv + bk^2 * raw : 1   (raw = sum mu^2 W_p)
enum { MODE_PLAIN = 0, MODE_AXPY = 1, MODE_DIAG = 2 };

__device__ __forceinline__ int block_to_m(int b) {
  // blocks are dealt to the 8 XCDs round-robin; give each XCD four
  // consecutive m so the 128-byte lines of G they share stay in one L2
  const int xcd = b & 7, q = b >> 3;
  return (q >> 2) * 32 + xcd * 4 + (q & 3);
}

template <int NR, int RPT, int MODE>
__global__ __launch_bounds__(kAdjBlock) void k_legendre_adj(
    int lmax, int mmax, int npairs, const double* __restrict__ pair_z, const double* __restrict__ alpha,
    const double* __restrict__ lmm_v, const int* __restrict__ lmm_k, const int64_t* __restrict__ mstart,
    const double* __restrict__ oscale, const double2* __restrict__ geo, int64_t geo_stride,
    const double* __restrict__ ringw, double2* __restrict__ out, double* __restrict__ dout, int64_t out_stride,
    const double2* __restrict__ pin, const double* __restrict__ sinv, const double* __restrict__ bk,
    double* __restrict__ partial, int npart) {
  constexpr int C = kAdjOutputs / (2 * NR);          // l steps per reduction chunk
  constexpr int TPO = kAdjBlock / kAdjOutputs;        // threads per reduced output
  __shared__ double red[kAdjOutputs][kAdjBlock];
  __shared__ double redq[kAdjBlock];

  const int m = block_to_m(blockIdx.x);
  if (m > mmax) return;
  const int t = threadIdx.x;
  const int64_t base = mstart[m];
  const double* __restrict__ al = alpha + base - m;

  double z[RPT], v0[RPT], v1[RPT];
  int k[RPT];
  double2 ge[RPT][NR], go[RPT][NR];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int p = t + j * kAdjBlock;
    const bool ok = p < npairs;
    const int pp = ok ? p : 0;
    z[j] = pair_z[pp];
    v0[j] = 0.0;
    v1[j] = ok ? lmm_v[(size_t)m * npairs + pp] : 0.0;
    k[j] = ok ? lmm_k[(size_t)m * npairs + pp] : 0;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      if (MODE == MODE_DIAG) {
        const double wgt = ok ? ringw[pp] : 0.0;
        ge[j][c] = make_double2(wgt, 0.0);
        go[j][c] = ge[j][c];
      } else {
        const double2* g = geo + c * geo_stride + ((size_t)pp * (mmax + 1) + m) * 2;
        ge[j][c] = ok ? g[0] : make_double2(0.0, 0.0);
        go[j][c] = ok ? g[1] : make_double2(0.0, 0.0);
      }
    }
  }

  const int o = t / TPO;        // output this thread reduces: (jj, c, re/im)
  const int s = t % TPO;
  const int o_jj = o / (2 * NR), o_c = (o / 2) % NR, o_ri = o & 1;
  const double wm = (m == 0) ? 1.0 : 2.0;
  double accq = 0.0;

  for (int l0 = m; l0 <= lmax; l0 += C) {
    double2 part[C][NR];
#pragma unroll
    for (int jj = 0; jj < C; ++jj)
#pragma unroll
      for (int c = 0; c < NR; ++c) part[jj][c] = make_double2(0.0, 0.0);

    bool anyneg = false;
#pragma unroll
    for (int j = 0; j < RPT; ++j) anyneg |= (k[j] < 0);
    const bool scaled = __any(anyneg);

#pragma unroll
    for (int jj = 0; jj < C; ++jj) {
      const int l = l0 + jj;
      if (l > lmax) break;
      const bool odd = (l - m) & 1;
      const double a = (l > m) ? al[l] : 0.0;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        if (l > m) {
          const double mu = fma(a * z[j], v1[j], -v0[j]);
          v0[j] = v1[j];
          v1[j] = mu;
          if (scaled) rescale(v0[j], v1[j], k[j]);
        }
        double w = v1[j];
        if (scaled) w = (k[j] == 0) ? w : 0.0;
        if (MODE == MODE_DIAG) w = w * w;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          const double2 g = odd ? go[j][c] : ge[j][c];
          part[jj][c].x = fma(w, g.x, part[jj][c].x);
          part[jj][c].y = fma(w, g.y, part[jj][c].y);
        }
      }
    }

    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < C; ++jj)
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        red[(jj * NR + c) * 2 + 0][t] = part[jj][c].x;
        red[(jj * NR + c) * 2 + 1][t] = part[jj][c].y;
      }
    __syncthreads();
    double sum = 0.0;
#pragma unroll 4
    for (int i = 0; i < kAdjBlock / TPO; ++i) sum += red[o][s + TPO * i];
#pragma unroll
    for (int off = TPO / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, TPO);
    const int l = l0 + o_jj;
    if (s == 0 && l <= lmax) {
      const int64_t idx = base + (l - m);
      if (MODE == MODE_PLAIN) {
        reinterpret_cast<double*>(out + o_c * out_stride + idx)[o_ri] = oscale[idx] * sum;
      } else if (MODE == MODE_AXPY) {
        const double pv = reinterpret_cast<const double*>(pin + o_c * out_stride + idx)[o_ri];
        const double val = sinv[idx] * pv + bk[idx] * sum;
        reinterpret_cast<double*>(out + o_c * out_stride + idx)[o_ri] = val;
        accq = fma(wm * pv, val, accq);
      } else {
        if (o_ri == 0) {
          const double b = bk[idx];
          dout[idx] = (b != 0.0 || sinv[idx] != 0.0) ? sinv[idx] + b * b * sum : 1.0;
        }
      }
    }
  }

  if (MODE == MODE_AXPY) {
    __syncthreads();
    redq[t] = accq;
    __syncthreads();
    if (t < NR) {
      // threads owning column c: o = (jj*NR + c)*2 + ri, s == 0
      double tot = 0.0;
      for (int jj = 0; jj < C; ++jj)
        for (int ri = 0; ri < 2; ++ri) tot += redq[((jj * NR + t) * 2 + ri) * TPO];
      partial[(size_t)t * 4 * npart + m] = tot;
    }
  }
}

int pick_nr(int n) { return n >= 8 ? 8 : n >= 4 ? 4 : n >= 2 ? 2 : 1; }

template <int NR>
hipError_t synth_pass(const crsht_plan* P, const double2* alms, double2* eo, hipStream_t s) {
  const Geometry& g = P->g;
  dim3 grid((g.mmax + kSynthMT) / kSynthMT, (g.npairs + kSynthBlock - 1) / kSynthBlock);
  const int64_t eo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  timing_begin(P, 0, s);
  hipLaunchKernelGGL(k_legendre_synth<NR>, grid, dim3(kSynthBlock), 0, s, g.lmax, g.mmax, g.npairs, P->t.pair_z,
                     P->t.rec_alpha, P->t.lmm_v, P->t.lmm_k, P->t.mstart, alms, (int64_t)g.nalm, eo, eo_stride);
  timing_end(P, 0, s);
  return hipGetLastError();
}

template <int NR, int RPT>
hipError_t adj_pass_rpt(const crsht_plan* P, const double2* geo, double2* out, double* dout, int mode,
                        const double2* pin, const double* sinv, const double* bk, double* partial,
                        hipStream_t s) {
  const double* oscale = (mode == MODE_PLAIN && sinv) ? sinv : P->t.rec_kappa;
  const Geometry& g = P->g;
  const int nb = ((g.mmax + 1 + 31) / 32) * 32;
  const int64_t geo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  const int64_t os = g.nalm;
#define CRSHT_ADJ_LAUNCH(MD)                                                                                 \
  hipLaunchKernelGGL((k_legendre_adj<NR, RPT, MD>), dim3(nb), dim3(kAdjBlock), 0, s, g.lmax, g.mmax,        \
                     g.npairs, P->t.pair_z, P->t.rec_alpha, P->t.lmm_v, P->t.lmm_k, P->t.mstart,             \
                     oscale, geo, geo_stride, P->w.ring_w, out, dout, os, pin, sinv, bk, partial,            \
                     P->w.npart)
  timing_begin(P, 1, s);
  if (mode == MODE_PLAIN)
    CRSHT_ADJ_LAUNCH(MODE_PLAIN);
  else if (mode == MODE_AXPY)
    CRSHT_ADJ_LAUNCH(MODE_AXPY);
  else
    CRSHT_ADJ_LAUNCH(MODE_DIAG);
  timing_end(P, 1, s);
#undef CRSHT_ADJ_LAUNCH
  return hipGetLastError();
}

// ring pairs per thread of the adjoint, and the widest column group that
// keeps the per-thread G values (RPT x NR x 2 complex) within registers
int adj_rpt(const crsht_plan* P) {
  const int r = (P->g.npairs + kAdjBlock - 1) / kAdjBlock;
  return r <= 1 ? 1 : r <= 2 ? 2 : r <= 4 ? 4 : r <= 8 ? 8 : 16;
}
int adj_max_nr(int rpt) { return rpt >= 16 ? 1 : rpt >= 8 ? 2 : rpt >= 4 ? 4 : 8; }

template <int NR>
hipError_t adj_pass(const crsht_plan* P, const double2* geo, double2* out, double* dout, int mode,
                    const double2* pin, const double* sinv, const double* bk, double* partial, hipStream_t s) {
  const int rpt = adj_rpt(P);
  if (rpt == 1) return adj_pass_rpt<NR, 1>(P, geo, out, dout, mode, pin, sinv, bk, partial, s);
  if (rpt == 2) return adj_pass_rpt<NR, 2>(P, geo, out, dout, mode, pin, sinv, bk, partial, s);
  if constexpr (NR <= 4)
    if (rpt == 4) return adj_pass_rpt<NR, 4>(P, geo, out, dout, mode, pin, sinv, bk, partial, s);
  if constexpr (NR <= 2)
    if (rpt == 8) return adj_pass_rpt<NR, 8>(P, geo, out, dout, mode, pin, sinv, bk, partial, s);
  if constexpr (NR == 1)
    if (rpt == 16) return adj_pass_rpt<NR, 16>(P, geo, out, dout, mode, pin, sinv, bk, partial, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_legendre_synth(const crsht_plan* P, int nrhs, const double2* alms, double2* eo, hipStream_t s) {
  const int64_t eo_stride = (int64_t)P->g.npairs * (P->g.mmax + 1) * 2;
  for (int c0 = 0; c0 < nrhs;) {
    const int nr = pick_nr(nrhs - c0);
    const double2* a = alms + (int64_t)c0 * P->g.nalm;
    double2* e = eo + (int64_t)c0 * eo_stride;
    hipError_t err = nr == 8 ? synth_pass<8>(P, a, e, s)
                   : nr == 4 ? synth_pass<4>(P, a, e, s)
                   : nr == 2 ? synth_pass<2>(P, a, e, s)
                             : synth_pass<1>(P, a, e, s);
    if (err != hipSuccess) return err;
    c0 += nr;
  }
  return hipSuccess;
}

hipError_t launch_legendre_adjoint(const crsht_plan* P, int nrhs, const double2* geo, double2* out, int mode,
                                   const double2* pin, const double* sinv, const double* bk, double* partial,
                                   bool square, hipStream_t s) {
  if (square) return adj_pass<1>(P, nullptr, nullptr, reinterpret_cast<double*>(out), MODE_DIAG, nullptr, sinv,
                                 bk, nullptr, s);
  const int64_t geo_stride = (int64_t)P->g.npairs * (P->g.mmax + 1) * 2;
  const int nr_cap = adj_max_nr(adj_rpt(P));
  for (int c0 = 0; c0 < nrhs;) {
    int nr = pick_nr(nrhs - c0);
    if (nr > nr_cap) nr = nr_cap;
    const double2* gi = geo + (int64_t)c0 * geo_stride;
    double2* oo = out + (int64_t)c0 * P->g.nalm;
    const double2* pi = pin ? pin + (int64_t)c0 * P->g.nalm : nullptr;
    double* pa = partial ? partial + (int64_t)c0 * 4 * P->w.npart : nullptr;
    hipError_t err = nr == 8 ? adj_pass<8>(P, gi, oo, nullptr, mode, pi, sinv, bk, pa, s)
                   : nr == 4 ? adj_pass<4>(P, gi, oo, nullptr, mode, pi, sinv, bk, pa, s)
                   : nr == 2 ? adj_pass<2>(P, gi, oo, nullptr, mode, pi, sinv, bk, pa, s)
                             : adj_pass<1>(P, gi, oo, nullptr, mode, pi, sinv, bk, pa, s);
    if (err != hipSuccess) return err;
    c0 += nr;
  }
  return hipSuccess;
}

}  // namespace crsht
