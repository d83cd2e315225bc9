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
// Fused operator pass: synthesis, multiply by N^-1 per pixel (N^-1 is
// diagonal in pixels), adjoint, with the map kept in LDS.
//
// DFT lengths n = 4i that are not powers of two use Bluestein's chirp-z
// algorithm: X_k = c_k sum_j (x_j c_j) conj(c_{k-j}), c_j = exp(-i pi j^2/n),
// a cyclic convolution of power-of-two length L >= 2n - 1 with the FFT of the
// conjugate chirp precomputed per ring. Power-of-two FFTs are in-place
// Stockham passes of radix 16 (8, 4, 2 for the last): each thread loads R
// points from LDS into registers, applies the inter-pass twiddles, does an
// R-point DFT in registers and writes back; natural order in and out.
#include "internal.h"

namespace crsht {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 add2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 sub2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ int ilog2(int n) { return 31 - __clz(n); }

// exp(-2 pi i q / 16), q = 0..15
__device__ __forceinline__ double2 root16(int q) {
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, r2 = 0.70710678118654752440;
  switch (q & 15) {
    case 0: return make_double2(1.0, 0.0);
    case 1: return make_double2(c1, -s1);
    case 2: return make_double2(r2, -r2);
    case 3: return make_double2(s1, -c1);
    case 4: return make_double2(0.0, -1.0);
    case 5: return make_double2(-s1, -c1);
    case 6: return make_double2(-r2, -r2);
    case 7: return make_double2(-c1, -s1);
    case 8: return make_double2(-1.0, 0.0);
    case 9: return make_double2(-c1, s1);
    case 10: return make_double2(-r2, r2);
    case 11: return make_double2(-s1, c1);
    case 12: return make_double2(0.0, 1.0);
    case 13: return make_double2(s1, c1);
    case 14: return make_double2(r2, r2);
    default: return make_double2(c1, s1);
  }
}

// multiply by exp(-2 pi i q/16) (conjugate root if inv), q a compile-time constant after unrolling
__device__ __forceinline__ double2 mul_root(double2 a, int q, bool inv) {
  q &= 15;
  if (q == 0) return a;
  if (q == 8) return make_double2(-a.x, -a.y);
  if (q == 4) return inv ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
  if (q == 12) return inv ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
  const double2 w = root16(q);
  return cmul(a, inv ? conj2(w) : w);
}

__host__ __device__ constexpr int brev_c(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

// R-point DFT in registers (natural order in and out), R = 2, 4, 8, 16
template <int R>
__device__ __forceinline__ void dft_reg(double2 (&v)[R], bool inv) {
  constexpr int B = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
  double2 t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) t[brev_c(i, B)] = v[i];
#pragma unroll
  for (int h = 1; h < R; h <<= 1) {
#pragma unroll
    for (int g = 0; g < R; g += 2 * h) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const double2 a = t[g + j];
        const double2 b = mul_root(t[g + j + h], j * (16 / (2 * h)), inv);
        t[g + j] = add2(a, b);
        t[g + j + h] = sub2(a, b);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = t[i];
}

// one in-place Stockham pass of radix R over N points with stride Ns
// (Govindaraju et al. 2008 formulation). tw: exp(-2 pi i q / fmax), q < fmax.
// Every thread handles up to J = 16 / R butterflies, so any N <= 16 blockDim
// fits; all inputs are read into registers before the barrier that precedes
// the writes, which makes the pass in place.
template <int R>
__device__ __forceinline__ void stockham_pass(double2* x, int N, int Ns, const double2* __restrict__ tw, int fmax,
                                              bool inv) {
  constexpr int J = 16 / R;
  const int nt = N / R;
  double2 v[J][R];
#pragma unroll
  for (int u = 0; u < J; ++u) {
    const int j = threadIdx.x + u * blockDim.x;
    if (j < nt) {
      const int k = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[u][r] = x[j + r * nt];
      if (Ns > 1) {
        const int step = k * (fmax / (Ns * R));
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const double2 w = tw[r * step];
          v[u][r] = cmul(v[u][r], inv ? conj2(w) : w);
        }
      }
      dft_reg<R>(v[u], inv);
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < J; ++u) {
    const int j = threadIdx.x + u * blockDim.x;
    if (j < nt) {
      const int k = j % Ns;
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) x[base + r * Ns] = v[u][r];
    }
  }
  __syncthreads();
}

// length-N (power of two, N <= 16 blockDim) DFT in place, natural order
__device__ void fft_pow2(double2* x, int N, const double2* __restrict__ tw, int fmax, bool inv) {
  __syncthreads();
  int b = ilog2(N);
  int Ns = 1;
  while (b >= 4) {
    stockham_pass<16>(x, N, Ns, tw, fmax, inv);
    Ns *= 16;
    b -= 4;
  }
  if (b == 3) stockham_pass<8>(x, N, Ns, tw, fmax, inv);
  else if (b == 2) stockham_pass<4>(x, N, Ns, tw, fmax, inv);
  else if (b == 1) stockham_pass<2>(x, N, Ns, tw, fmax, inv);
}

struct PairInfo {
  int n, L, den;
  int64_t fn, fs;
  bool equator, blue;
  const double2* chirp;
  const double2* kern;
};

__device__ __forceinline__ PairInfo pair_info(const Tables& T, int p, int nside) {
  PairInfo q;
  q.n = T.pair_nphi[p];
  q.L = T.pair_fft_len[p];
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

// e^{i m phi0} with phi0 = pi / den (den = 0 means phi0 = 0); m reduced
// exactly modulo 2 den before the trigonometric call.
__device__ __forceinline__ double2 phase(int m, int den) {
  if (den == 0) return make_double2(1.0, 0.0);
  const int r = m % (2 * den);
  double s, c;
  sincospi((double)r / (double)den, &s, &c);
  return make_double2(c, s);
}

// Hermitian spectrum h = c_N + i c_S of a ring pair into buf[0..n).
// For 0 <= k <= n/2 let A = sum_{m = k mod n} F'(m) and
// B = sum_{m = -k mod n, m >= 1} F'(m), F' = F e^{i m phi0} (F(0) real):
// c_k = A + conj B and c_{n-k} = B + conj A, so every F(m) is read once.
// When n/2 + 1 < blockDim the alias sums of one k are split over S threads
// (alias indices s, s + S, ...) whose partial sums are combined in a fixed
// order through LDS (scratch, at least blockDim x 8 doubles); the result is
// the same sum regrouped. Bluestein rings store conj(h_k) c_k (chirp) instead.
// alias sums of frequency k over the aliases s, s + S, s + 2S, ...
__device__ __forceinline__ void alias_sums(const double2* __restrict__ eo, int mmax, int n, int den, int k, int s,
                                           int S, double2& aN, double2& aS, double2& bN, double2& bS) {
  aN = make_double2(0.0, 0.0);
  aS = aN;
  bN = aN;
  bS = aN;
  for (int m = k + s * n; m <= mmax; m += S * n) {
    const double2 E = eo[2 * m], O = eo[2 * m + 1];
    double2 fn = add2(E, O), fs = sub2(E, O);
    if (m == 0) {
      fn.y = 0.0;
      fs.y = 0.0;
    }
    const double2 ph = phase(m, den);
    aN = add2(aN, cmul(fn, ph));
    aS = add2(aS, cmul(fs, ph));
  }
  if (k > 0 && 2 * k != n) {
    for (int m = n - k + s * n; m <= mmax; m += S * n) {
      const double2 E = eo[2 * m], O = eo[2 * m + 1];
      const double2 ph = phase(m, den);
      bN = add2(bN, cmul(add2(E, O), ph));
      bS = add2(bS, cmul(sub2(E, O), ph));
    }
  }
}

// h_k and h_{n-k} from the complete alias sums of k, stored in buf
__device__ __forceinline__ void store_spectrum(double2* buf, const PairInfo& q, const double2* __restrict__ eo, int k,
                                               double2 aN, double2 aS, double2 bN, double2 bS) {
  const int n = q.n;
  if (k == 0 || 2 * k == n) {
    // k = 0: B = A without the m = 0 term; k = n/2: the two alias sets coincide
    bN = aN;
    bS = aS;
    if (k == 0) {
      const double2 E = eo[0], O = eo[1];
      bN.x -= E.x + O.x;
      bS.x -= E.x - O.x;
    }
  }
  double2 cn = add2(aN, conj2(bN)), cs = add2(aS, conj2(bS));
  double2 cnn = add2(bN, conj2(aN)), csn = add2(bS, conj2(aS));
  if (q.equator) cs = csn = make_double2(0.0, 0.0);
  double2 hk = make_double2(cn.x - cs.y, cn.y + cs.x);
  double2 hnk = make_double2(cnn.x - csn.y, cnn.y + csn.x);
  if (q.blue) {
    hk = cmul(conj2(hk), q.chirp[k]);
    if (k > 0) hnk = cmul(conj2(hnk), q.chirp[n - k]);
  }
  buf[k] = hk;
  if (k > 0) buf[n - k] = hnk;   // k = n/2 writes the same value twice
}

__device__ void spectrum(double2* buf, double* scratch, const PairInfo& q, const double2* __restrict__ eo,
                         int mmax) {
  const int n = q.n, nk = n / 2 + 1;
  const int S = (int)blockDim.x / nk;
  double2 aN, aS, bN, bS;
  if (S <= 1) {
    for (int k = threadIdx.x; k < nk; k += blockDim.x) {
      alias_sums(eo, mmax, n, q.den, k, 0, 1, aN, aS, bN, bS);
      store_spectrum(buf, q, eo, k, aN, aS, bN, bS);
    }
    return;
  }
  const int t = threadIdx.x;
  const int k = t / S, s = t % S;
  if (k < nk) alias_sums(eo, mmax, n, q.den, k, s, S, aN, aS, bN, bS);
  else aN = aS = bN = bS = make_double2(0.0, 0.0);
  // combine the S partial sums of each k in order of s
  double* sc = scratch + (size_t)t * 8;
  sc[0] = aN.x; sc[1] = aN.y; sc[2] = aS.x; sc[3] = aS.y;
  sc[4] = bN.x; sc[5] = bN.y; sc[6] = bS.x; sc[7] = bS.y;
  __syncthreads();
  if (k < nk && s == 0) {
    for (int u = 1; u < S; ++u) {
      const double* o = scratch + (size_t)(t + u) * 8;
      aN.x += o[0]; aN.y += o[1]; aS.x += o[2]; aS.y += o[3];
      bN.x += o[4]; bN.y += o[5]; bS.x += o[6]; bS.y += o[7];
    }
    store_spectrum(buf, q, eo, k, aN, aS, bN, bS);
  }
}

// Z_j = map_N[j] + i map_S[j] for j < n, left in buf[0..n) (natural order)
__device__ void ring_inverse(double2* buf, double* scratch, const PairInfo& q, const double2* __restrict__ eo,
                             int mmax, const double2* __restrict__ tw, int fmax) {
  spectrum(buf, scratch, q, eo, mmax);
  if (!q.blue) {
    fft_pow2(buf, q.n, tw, fmax, true);
  } else {
    // IDFT(h) = conj(DFT(conj h)); DFT by chirp-z
    for (int j = q.n + threadIdx.x; j < q.L; j += blockDim.x) buf[j] = make_double2(0.0, 0.0);
    fft_pow2(buf, q.L, tw, fmax, false);
    for (int j = threadIdx.x; j < q.L; j += blockDim.x) buf[j] = cmul(buf[j], q.kern[j]);
    fft_pow2(buf, q.L, tw, fmax, true);
    for (int j = threadIdx.x; j < q.n; j += blockDim.x) buf[j] = conj2(cmul(buf[j], q.chirp[j]));
    __syncthreads();
  }
}

// forward DFT of z_j (buf[0..n), natural order) in place; X_k in buf[k]
__device__ void ring_forward(double2* buf, const PairInfo& q, const double2* __restrict__ tw, int fmax) {
  if (!q.blue) {
    fft_pow2(buf, q.n, tw, fmax, false);
  } else {
    for (int j = threadIdx.x; j < q.L; j += blockDim.x)
      buf[j] = j < q.n ? cmul(buf[j], q.chirp[j]) : make_double2(0.0, 0.0);
    fft_pow2(buf, q.L, tw, fmax, false);
    for (int j = threadIdx.x; j < q.L; j += blockDim.x) buf[j] = cmul(buf[j], q.kern[j]);
    fft_pow2(buf, q.L, tw, fmax, true);
    for (int j = threadIdx.x; j < q.n; j += blockDim.x) buf[j] = cmul(buf[j], q.chirp[j]);
    __syncthreads();
  }
}

// G_E = G_N + G_S and G_O = G_N - G_S for m = 0..mmax.
__device__ void write_geo(double2* __restrict__ geo, const double2* buf, const PairInfo& q, int mmax) {
  for (int m = threadIdx.x; m <= mmax; m += blockDim.x) {
    const int k = m % q.n;
    const int kn = (q.n - k) % q.n;
    const double2 X = buf[k], Xm = conj2(buf[kn]);
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
__global__ __launch_bounds__(1024) void k_ring(Tables T, int nside, int mmax, int fmax,
                                              const double2* __restrict__ eo, int64_t eo_stride,
                                              double* __restrict__ map, int64_t map_stride,
                                              const double* __restrict__ ninv, double2* __restrict__ geo,
                                              int64_t geo_stride) {
  extern __shared__ double2 buf[];
  // spectrum scratch (blockDim x 8 doubles) after the FFT buffer
  double* scratch = reinterpret_cast<double*>(buf + fmax);
  const int p = blockIdx.x, c = blockIdx.y;
  const PairInfo q = pair_info(T, p, nside);
  const double2* __restrict__ eop = eo + c * eo_stride + (size_t)p * (mmax + 1) * 2;
  double2* __restrict__ geop = geo + c * geo_stride + (size_t)p * (mmax + 1) * 2;
  double* __restrict__ mp = map + c * map_stride;

  if (MODE == RING_SYNTH || MODE == RING_FUSED) ring_inverse(buf, scratch, q, eop, mmax, T.twiddle, fmax);

  if (MODE == RING_SYNTH) {
    for (int j = threadIdx.x; j < q.n; j += blockDim.x) {
      const double2 Z = buf[j];
      mp[q.fn + j] = Z.x;
      if (!q.equator) mp[q.fs + j] = Z.y;
    }
    return;
  }

  if (MODE == RING_FUSED) {
    for (int j = threadIdx.x; j < q.n; j += blockDim.x) {
      const double2 Z = buf[j];
      buf[j] = make_double2(Z.x * ninv[q.fn + j], q.equator ? 0.0 : Z.y * ninv[q.fs + j]);
    }
  } else {  // RING_ADJOINT: load the pixels
    for (int j = threadIdx.x; j < q.n; j += blockDim.x)
      buf[j] = make_double2(mp[q.fn + j], q.equator ? 0.0 : mp[q.fs + j]);
  }
  ring_forward(buf, q, T.twiddle, fmax);
  write_geo(geop, buf, q, mmax);
}

}  // namespace

// threads per ring block: fft_pow2 needs N <= 16 blockDim for every N <= fft_max
int ring_block(const crsht_plan* P) {
  int t = P->g.fft_max / 16;
  if (t < 64) t = 64;
  return t;
}
size_t ring_lds_bytes(const crsht_plan* P) {
  return (size_t)P->g.fft_max * sizeof(double2) + (size_t)ring_block(P) * 8 * sizeof(double);
}

hipError_t launch_ring(const crsht_plan* P, int nrhs, RingMode mode, const double2* eo, double* map,
                       const double* ninv, double2* geo, hipStream_t s) {
  const Geometry& g = P->g;
  const int64_t eo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  const size_t lds = ring_lds_bytes(P);
  dim3 grid(g.npairs, nrhs);
  const int bt = ring_block(P);
#define CRSHT_RING(MD)                                                                                   \
  do {                                                                                                   \
    if (lds > 65536)                                                                                     \
      (void)hipFuncSetAttribute((const void*)k_ring<MD>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    hipLaunchKernelGGL(k_ring<MD>, grid, dim3(bt), lds, s, P->t, g.nside, g.mmax, g.fft_max, eo,           \
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
