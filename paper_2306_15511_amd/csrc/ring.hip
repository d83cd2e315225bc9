// Azimuthal step of the transforms: one block per (ring pair, column).
//
// Synthesis (map of one ring from its Legendre sums F(m), m = 0..mmax):
//   map_j = sum_{m=-mmax}^{mmax} F(m) e^{i m (phi0 + 2 pi j / n)},  F(-m) = conj F(m),
// i.e. fold F(m) e^{i m phi0} onto the n frequencies k = m mod n (Hermitian
// spectrum) and take a length-n inverse DFT. The north and south rings of a
// pair share n and phi0, so both real maps come from one complex transform of
// c_N + i c_S.
// Adjoint (the transpose, no 1/n): G(m) = e^{-i m phi0} X(m mod n) with X the
// forward DFT of the ring's pixels; again one complex transform of x_N + i x_S
// serves both rings and X_N, X_S are separated by Hermitian symmetry.
// Fused operator pass: synthesis, multiply by N^-1 per pixel (paper App. A
// N^-1 is diagonal in pixels), adjoint, with the map kept in LDS.
//
// DFT lengths n = 4i that are not powers of two use Bluestein's chirp-z
// algorithm: X_k = c_k sum_j (x_j c_j) conj(c_{k-j}), c_j = exp(-i pi j^2/n),
// computed as a cyclic convolution of power-of-two length L >= 2n - 1 with the
// FFT of the conjugate chirp precomputed per ring. All FFTs are radix-2 in LDS.
#include "internal.h"

namespace crsht {
namespace {

constexpr int kRingBlock = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 add2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 sub2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ unsigned bitrev(unsigned x, int bits) { return bits ? (__brev(x) >> (32 - bits)) : 0u; }
__device__ __forceinline__ int ilog2(int n) { return 31 - __clz(n); }

// e^{i m phi0} with phi0 = pi / den (den = 0 means phi0 = 0); m reduced
// exactly modulo 2 den before the trigonometric call.
__device__ __forceinline__ double2 phase(int m, int den) {
  if (den == 0) return make_double2(1.0, 0.0);
  const int r = m % (2 * den);
  double s, c;
  sincospi((double)r / (double)den, &s, &c);
  return make_double2(c, s);
}

// twiddle W_{2h}^j = exp(sign 2 pi i j / (2h)) from the table exp(-2 pi i q / fmax)
__device__ __forceinline__ double2 twid(const double2* __restrict__ tw, int fmax, int j, int h2, bool inverse) {
  const double2 w = tw[j * (fmax / h2)];
  return inverse ? conj2(w) : w;
}

// Decimation in time: bit-reversed input, natural-order output.
__device__ void fft_dit(double2* buf, int L, const double2* __restrict__ tw, int fmax, bool inverse) {
  for (int h = 1; h < L; h <<= 1) {
    __syncthreads();
    for (int b = threadIdx.x; b < L / 2; b += blockDim.x) {
      const int j = b & (h - 1);
      const int i0 = ((b - j) << 1) + j, i1 = i0 + h;
      const double2 t = cmul(twid(tw, fmax, j, 2 * h, inverse), buf[i1]);
      const double2 u = buf[i0];
      buf[i0] = add2(u, t);
      buf[i1] = sub2(u, t);
    }
  }
  __syncthreads();
}

// Decimation in frequency: natural-order input, bit-reversed output.
__device__ void fft_dif(double2* buf, int L, const double2* __restrict__ tw, int fmax, bool inverse) {
  for (int h = L >> 1; h >= 1; h >>= 1) {
    __syncthreads();
    for (int b = threadIdx.x; b < L / 2; b += blockDim.x) {
      const int j = b & (h - 1);
      const int i0 = ((b - j) << 1) + j, i1 = i0 + h;
      const double2 u = buf[i0], v = buf[i1];
      buf[i0] = add2(u, v);
      buf[i1] = cmul(sub2(u, v), twid(tw, fmax, j, 2 * h, inverse));
    }
  }
  __syncthreads();
}

struct PairInfo {
  int n, L, bits, den;
  int64_t fn, fs;
  bool equator, blue;
  const double2* chirp;
  const double2* kern;
};

__device__ __forceinline__ PairInfo pair_info(const Tables& T, int p, int nside) {
  PairInfo q;
  q.n = T.pair_nphi[p];
  q.L = T.pair_fft_len[p];
  q.bits = ilog2(q.L);
  q.fn = T.pair_first_n[p];
  q.fs = T.pair_first_s[p];
  q.equator = (q.fn == q.fs);
  q.blue = (q.L != q.n);
  const int i = p + 1;
  // phi0 = pi/(4i) in the polar caps, 0 or pi/(4 nside) in the belt
  if (i < nside) q.den = 4 * i;
  else q.den = ((i + nside) & 1) ? 0 : 4 * nside;
  q.chirp = q.blue ? T.bs_chirp + T.pair_bs_off[p] : nullptr;
  q.kern = q.blue ? T.bs_kern + T.pair_bk_off[p] : nullptr;
  return q;
}

// Hermitian spectrum h_k = c_N[k] + i c_S[k], k < n, from the Legendre sums.
__device__ __forceinline__ double2 spectrum(const double2* __restrict__ eo, int mmax, int n, int den, bool equator,
                                            int k) {
  double2 cn = make_double2(0.0, 0.0), cs = make_double2(0.0, 0.0);
  for (int m = k; m <= mmax; m += n) {
    const double2 E = eo[2 * m], O = eo[2 * m + 1];
    double2 fn = add2(E, O), fs = sub2(E, O);
    if (m == 0) {
      fn.y = 0.0;
      fs.y = 0.0;
    }
    const double2 ph = phase(m, den);
    cn = add2(cn, cmul(fn, ph));
    cs = add2(cs, cmul(fs, ph));
  }
  for (int m = (k == 0 ? n : n - k); m <= mmax; m += n) {
    const double2 E = eo[2 * m], O = eo[2 * m + 1];
    const double2 ph = phase(m, den);
    cn = add2(cn, conj2(cmul(add2(E, O), ph)));
    cs = add2(cs, conj2(cmul(sub2(E, O), ph)));
  }
  if (equator) cs = make_double2(0.0, 0.0);
  return make_double2(cn.x - cs.y, cn.y + cs.x);
}

// Inverse DFT of the spectrum into buf. Afterwards Z_j (map_N + i map_S) is
// at zpos(j): j for power-of-two rings, bitrev(j) for Bluestein rings, where
// it is stored conjugated and without the final chirp (see zval()).
__device__ void ring_inverse(double2* buf, const PairInfo& q, const double2* __restrict__ eo, int mmax,
                             const double2* __restrict__ tw, int fmax) {
  if (!q.blue) {
    for (int k = threadIdx.x; k < q.n; k += blockDim.x)
      buf[bitrev(k, q.bits)] = spectrum(eo, mmax, q.n, q.den, q.equator, k);
    fft_dit(buf, q.L, tw, fmax, true);
  } else {
    // IDFT(h) = conj(DFT(conj h)); DFT by chirp-z
    for (int j = threadIdx.x; j < q.L; j += blockDim.x) {
      double2 v = make_double2(0.0, 0.0);
      if (j < q.n) v = cmul(conj2(spectrum(eo, mmax, q.n, q.den, q.equator, j)), q.chirp[j]);
      buf[bitrev(j, q.bits)] = v;
    }
    fft_dit(buf, q.L, tw, fmax, false);
    for (int j = threadIdx.x; j < q.L; j += blockDim.x) buf[j] = cmul(buf[j], q.kern[j]);
    fft_dif(buf, q.L, tw, fmax, true);
  }
}

__device__ __forceinline__ int zpos(const PairInfo& q, int j) { return q.blue ? (int)bitrev(j, q.bits) : j; }
__device__ __forceinline__ double2 zval(const PairInfo& q, const double2* buf, int j) {
  const double2 v = buf[zpos(q, j)];
  return q.blue ? conj2(cmul(v, q.chirp[j])) : v;
}

// Forward DFT of z_j (already placed by the caller: for power-of-two rings at
// natural positions, for Bluestein rings as z_j c_j at bitrev(j) with zeros
// elsewhere). Afterwards X_k is at bitrev(k) (Bluestein: times chirp, xval()).
__device__ void ring_forward(double2* buf, const PairInfo& q, const double2* __restrict__ tw, int fmax) {
  if (!q.blue) {
    fft_dif(buf, q.L, tw, fmax, false);
  } else {
    fft_dit(buf, q.L, tw, fmax, false);
    for (int j = threadIdx.x; j < q.L; j += blockDim.x) buf[j] = cmul(buf[j], q.kern[j]);
    fft_dif(buf, q.L, tw, fmax, true);
  }
}

__device__ __forceinline__ double2 xval(const PairInfo& q, const double2* buf, int k) {
  const double2 v = buf[bitrev(k, q.bits)];
  return q.blue ? cmul(v, q.chirp[k]) : v;
}

// G_E = G_N + G_S and G_O = G_N - G_S for m = 0..mmax.
__device__ void write_geo(double2* __restrict__ geo, const double2* buf, const PairInfo& q, int mmax) {
  for (int m = threadIdx.x; m <= mmax; m += blockDim.x) {
    const int k = m % q.n;
    const int kn = (q.n - k) % q.n;
    const double2 X = xval(q, buf, k), Xm = conj2(xval(q, buf, kn));
    // X_N = (X + conj X(-k))/2, X_S = (X - conj X(-k))/(2i)
    const double2 XN = make_double2(0.5 * (X.x + Xm.x), 0.5 * (X.y + Xm.y));
    const double2 XS = make_double2(0.5 * (X.y - Xm.y), -0.5 * (X.x - Xm.x));
    const double2 ph = conj2(phase(m, q.den));
    const double2 GN = cmul(XN, ph);
    const double2 GS = q.equator ? make_double2(0.0, 0.0) : cmul(XS, ph);
    geo[2 * m] = add2(GN, GS);
    geo[2 * m + 1] = sub2(GN, GS);
  }
}

template <int MODE>
__global__ __launch_bounds__(kRingBlock) void k_ring(Tables T, int nside, int mmax, int fmax,
                                                     const double2* __restrict__ eo, int64_t eo_stride,
                                                     double* __restrict__ map, int64_t map_stride,
                                                     const double* __restrict__ ninv, double2* __restrict__ geo,
                                                     int64_t geo_stride) {
  extern __shared__ double2 buf[];
  const int p = blockIdx.x, c = blockIdx.y;
  const PairInfo q = pair_info(T, p, nside);
  const double2* __restrict__ eop = eo + c * eo_stride + (size_t)p * (mmax + 1) * 2;
  double2* __restrict__ geop = geo + c * geo_stride + (size_t)p * (mmax + 1) * 2;
  double* __restrict__ mp = map + c * map_stride;

  if (MODE == RING_SYNTH || MODE == RING_FUSED) ring_inverse(buf, q, eop, mmax, T.twiddle, fmax);

  if (MODE == RING_SYNTH) {
    for (int j = threadIdx.x; j < q.n; j += blockDim.x) {
      const double2 Z = zval(q, buf, j);
      mp[q.fn + j] = Z.x;
      if (!q.equator) mp[q.fs + j] = Z.y;
    }
    return;
  }

  if (MODE == RING_FUSED) {
    // z_j = Re Z_j ninv_N + i Im Z_j ninv_S, placed for the forward transform
    if (!q.blue) {
      for (int j = threadIdx.x; j < q.n; j += blockDim.x) {
        const double2 Z = buf[j];
        buf[j] = make_double2(Z.x * ninv[q.fn + j], q.equator ? 0.0 : Z.y * ninv[q.fs + j]);
      }
    } else {
      for (int j = threadIdx.x; j < q.L; j += blockDim.x) {
        const int pos = bitrev(j, q.bits);
        double2 v = make_double2(0.0, 0.0);
        if (j < q.n) {
          const double2 Z = conj2(cmul(buf[pos], q.chirp[j]));
          v = cmul(make_double2(Z.x * ninv[q.fn + j], q.equator ? 0.0 : Z.y * ninv[q.fs + j]), q.chirp[j]);
        }
        buf[pos] = v;
      }
    }
  } else {  // RING_ADJOINT: load the pixels
    if (!q.blue) {
      for (int j = threadIdx.x; j < q.n; j += blockDim.x)
        buf[j] = make_double2(mp[q.fn + j], q.equator ? 0.0 : mp[q.fs + j]);
    } else {
      for (int j = threadIdx.x; j < q.L; j += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (j < q.n) v = cmul(make_double2(mp[q.fn + j], q.equator ? 0.0 : mp[q.fs + j]), q.chirp[j]);
        buf[bitrev(j, q.bits)] = v;
      }
    }
  }
  ring_forward(buf, q, T.twiddle, fmax);
  write_geo(geop, buf, q, mmax);
}

}  // namespace

size_t ring_lds_bytes(const crsht_plan* P) { return (size_t)P->g.fft_max * sizeof(double2); }

hipError_t launch_ring(const crsht_plan* P, int nrhs, RingMode mode, const double2* eo, double* map,
                       const double* ninv, double2* geo, hipStream_t s) {
  const Geometry& g = P->g;
  const int64_t eo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  const size_t lds = ring_lds_bytes(P);
  dim3 grid(g.npairs, nrhs);
#define CRSHT_RING(MD)                                                                                   \
  do {                                                                                                   \
    if (lds > 65536)                                                                                     \
      (void)hipFuncSetAttribute((const void*)k_ring<MD>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    hipLaunchKernelGGL(k_ring<MD>, grid, dim3(kRingBlock), lds, s, P->t, g.nside, g.mmax, g.fft_max, eo,    \
                       eo_stride, map, (int64_t)g.npix, ninv, geo, eo_stride);                           \
  } while (0)
  timing_begin(P, 2, s);
  if (mode == RING_SYNTH)
    CRSHT_RING(RING_SYNTH);
  else if (mode == RING_ADJOINT)
    CRSHT_RING(RING_ADJOINT);
  else
    CRSHT_RING(RING_FUSED);
  timing_end(P, 2, s);
#undef CRSHT_RING
  return hipGetLastError();
}

}  // namespace crsht
