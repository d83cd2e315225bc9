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
// On every HEALPix ring n phi0 is pi (or phi0 = 0), so e^{i (m + n) phi0} =
// sigma e^{i m phi0} with sigma = -1 (or +1): all aliases m = k + s n of one
// frequency share the phase e^{i k phi0} up to the sign sigma^s, and one
// sincospi per frequency serves every alias.
//
// DFT lengths n = 4i that are not powers of two use Bluestein's chirp-z
// algorithm: X_k = c_k sum_j (x_j c_j) conj(c_{k-j}), c_j = exp(-i pi j^2/n),
// a cyclic convolution of power-of-two length L >= 2n - 1 with the FFT of the
// conjugate chirp precomputed per ring. Power-of-two FFTs are in-place
// Stockham passes of radix 16 (8, 4, 2 for the last): each thread loads R
// points from LDS into registers, applies the inter-pass twiddles (one table
// load, the other powers by multiplication), does an R-point DFT in registers
// and writes back; natural order in and out. LDS arrays are padded by one
// element every 16 so that the strided writes of a pass spread over the banks.
//
// Ring pairs are launched by classes of FFT length (LDS and block size sized
// to the class) and the (pair, column) blocks of one pair are kept on one XCD
// so that N^-1 and the Bluestein tables of the ring are shared in its L2.
// The kernels are instantiated for double (FP64 path) and float (the
// azimuthal step of the mixed-precision path); maps and N^-1 stay FP64.
#include "internal.h"

namespace crsht {
namespace {

template <class V> struct RealOf;
template <> struct RealOf<double2> { using T = double; };
template <> struct RealOf<float2> { using T = float; };
template <class V> using Re = typename RealOf<V>::T;

__device__ __forceinline__ double fmr(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmr(float a, float b, float c) { return fmaf(a, b, c); }

template <class V> __device__ __forceinline__ V mk(Re<V> x, Re<V> y) {
  V v;
  v.x = x;
  v.y = y;
  return v;
}
template <class V> __device__ __forceinline__ V zero() { return mk<V>(Re<V>(0), Re<V>(0)); }
template <class V> __device__ __forceinline__ V cmul(V a, V b) {
  return mk<V>(fmr(a.x, b.x, -a.y * b.y), fmr(a.x, b.y, a.y * b.x));
}
template <class V> __device__ __forceinline__ V conj2(V a) { return mk<V>(a.x, -a.y); }
template <class V> __device__ __forceinline__ V add2(V a, V b) { return mk<V>(a.x + b.x, a.y + b.y); }
template <class V> __device__ __forceinline__ V sub2(V a, V b) { return mk<V>(a.x - b.x, a.y - b.y); }
template <class V> __device__ __forceinline__ V scl(Re<V> s, V a) { return mk<V>(s * a.x, s * a.y); }

__device__ __forceinline__ int ilog2(int n) { return 31 - __clz(n); }
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// LDS-only barrier: waits for this wavefront's LDS operations, not for its
// global loads in flight (prefetched operands stay in flight across it)
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// exp(-2 pi i q / 16), q = 0..15
template <class V> __device__ __forceinline__ V root16(int q) {
  using R = Re<V>;
  constexpr R c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173), r2 = R(0.70710678118654752440);
  switch (q & 15) {
    case 0: return mk<V>(R(1), R(0));
    case 1: return mk<V>(c1, -s1);
    case 2: return mk<V>(r2, -r2);
    case 3: return mk<V>(s1, -c1);
    case 4: return mk<V>(R(0), R(-1));
    case 5: return mk<V>(-s1, -c1);
    case 6: return mk<V>(-r2, -r2);
    case 7: return mk<V>(-c1, -s1);
    case 8: return mk<V>(R(-1), R(0));
    case 9: return mk<V>(-c1, s1);
    case 10: return mk<V>(-r2, r2);
    case 11: return mk<V>(-s1, c1);
    case 12: return mk<V>(R(0), R(1));
    case 13: return mk<V>(s1, c1);
    case 14: return mk<V>(r2, r2);
    default: return mk<V>(c1, s1);
  }
}

// multiply by exp(-2 pi i q/16) (conjugate root if inv), q a compile-time constant after unrolling
template <class V> __device__ __forceinline__ V mul_root(V a, int q, bool inv) {
  q &= 15;
  if (q == 0) return a;
  if (q == 8) return mk<V>(-a.x, -a.y);
  if (q == 4) return inv ? mk<V>(-a.y, a.x) : mk<V>(a.y, -a.x);
  if (q == 12) return inv ? mk<V>(a.y, -a.x) : mk<V>(-a.y, a.x);
  const V w = root16<V>(q);
  return cmul(a, inv ? conj2(w) : w);
}

__host__ __device__ constexpr int brev_c(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

// R-point DFT in registers (natural order in and out), R = 2, 4, 8, 16
template <int R, class V>
__device__ __forceinline__ void dft_reg(V (&v)[R], bool inv) {
  constexpr int B = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
  V t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) t[brev_c(i, B)] = v[i];
#pragma unroll
  for (int h = 1; h < R; h <<= 1) {
#pragma unroll
    for (int g = 0; g < R; g += 2 * h) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const V a = t[g + j];
        const V b = mul_root(t[g + j + h], j * (16 / (2 * h)), inv);
        t[g + j] = add2(a, b);
        t[g + j + h] = sub2(a, b);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = t[i];
}

// one in-place Stockham pass of radix R over N = 2^lN points with stride
// Ns = 2^lNs (Govindaraju et al. 2008 formulation). tw: exp(-2 pi i q / fmax),
// q < fmax = 2^lf. Blocks have at least N/8 threads, so a thread handles at
// most J = 8/R butterflies; all inputs are read into registers before the
// barrier that precedes the writes, which makes the pass in place. The
// twiddles w^r of a butterfly come from one table load w and products (at
// most six roundings). All lengths are powers of two, so the index
// arithmetic is shifts and masks, and the padded LDS offsets of a
// butterfly's R points are one padded base plus multiples of a padded
// stride (exact when the stride is 1 or a multiple of 16).
template <int R, class V>
__device__ __forceinline__ void stockham_pass(V* x, int lN, int lNs, const V* __restrict__ tw, int lf, bool inv) {
  constexpr int J = R >= 8 ? 1 : 8 / R;
  constexpr int lR = R == 16 ? 4 : R == 8 ? 3 : R == 4 ? 2 : 1;
  const int nt = 1 << (lN - lR);
  const int Ns = 1 << lNs;
  const bool in_strided = nt >= 16;                  // pad(j + r nt) = pad(j) + r (nt + nt / 16)
  const int in_stride = nt + (nt >> 4);
  const int out_stride = Ns == 1 ? 1 : Ns + (Ns >> 4);   // Ns = 1 or a multiple of 16
  V v[J][R];
  // twiddle loads first, for every u and without per-lane conditions (a
  // load under one is waited for at once), so their latency overlaps the
  // LDS reads
  V wl[J];
  if (lNs > 0) {
#pragma unroll
    for (int u = 0; u < J; ++u) wl[u] = tw[((threadIdx.x + u * blockDim.x) & (Ns - 1)) << (lf - lNs - lR)];
  }
#pragma unroll
  for (int u = 0; u < J; ++u) {
    const int j = threadIdx.x + u * blockDim.x;
    if (j < nt) {
      if (in_strided) {
        const int pj = pad(j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = x[pj + r * in_stride];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = x[pad(j + r * nt)];
      }
      if (lNs > 0) {
        V w1 = wl[u];
        if (inv) w1.y = -w1.y;
        const V w2 = cmul(w1, w1);
        const V w3 = cmul(w2, w1);
        const V w4 = cmul(w2, w2);
        V anc = w4;   // w^(r - r % 4) for the current group of four
#pragma unroll
        for (int r = 1; r < R; ++r) {
          if (r % 4 == 0 && r > 4) anc = cmul(anc, w4);
          const V lo = (r % 4 == 1) ? w1 : (r % 4 == 2) ? w2 : w3;
          const V wr = (r % 4 == 0) ? anc : (r < 4) ? lo : cmul(anc, lo);
          v[u][r] = cmul(v[u][r], wr);
        }
      }
      dft_reg<R>(v[u], inv);
    }
  }
  lds_barrier();
#pragma unroll
  for (int u = 0; u < J; ++u) {
    const int j = threadIdx.x + u * blockDim.x;
    if (j < nt) {
      const int k = j & (Ns - 1);
      const int pb = pad(((j >> lNs) << (lNs + lR)) + k);
#pragma unroll
      for (int r = 0; r < R; ++r) x[pb + r * out_stride] = v[u][r];
    }
  }
  lds_barrier();
}

// length-N (power of two, N <= 8 blockDim) DFT in place, natural order;
// fmax = 2^lf entries in the twiddle table
template <class V>
__device__ __forceinline__ void fft_pow2(V* x, int N, const V* __restrict__ tw, int lf, bool inv) {
  lds_barrier();
  const int lN = ilog2(N);
  int b = lN;
  int lNs = 0;
  while (b >= 4) {
    stockham_pass<16>(x, lN, lNs, tw, lf, inv);
    lNs += 4;
    b -= 4;
  }
  if (b == 3) stockham_pass<8>(x, lN, lNs, tw, lf, inv);
  else if (b == 2) stockham_pass<4>(x, lN, lNs, tw, lf, inv);
  else if (b == 1) stockham_pass<2>(x, lN, lNs, tw, lf, inv);
}

template <class V>
struct PairInfo {
  int n, L, den;
  int64_t fn, fs;
  bool equator, blue;
  Re<V> sigma;        // e^{i n phi0}
  const V* chirp;
  const V* kern;
};

template <class V>
__device__ __forceinline__ PairInfo<V> pair_info(const Tables& T, int p, int nside, const V* chirp, const V* kern) {
  PairInfo<V> q;
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
  q.sigma = q.den == 0 ? Re<V>(1) : Re<V>(-1);
  q.chirp = q.blue ? chirp + T.pair_bs_off[p] : nullptr;
  q.kern = q.blue ? kern + T.pair_bk_off[p] : nullptr;
  return q;
}

// e^{i k phi0} with phi0 = pi / den (den = 0 means phi0 = 0), for 0 <= k < n:
// on every ring den = n (polar caps) or den = n = 4 nside (belt), so k / den
// already lies in [0, 2) and needs no reduction before the trigonometric call.
__device__ __forceinline__ double2 phase_of(double2*, int k, int den) {
  if (den == 0) return make_double2(1.0, 0.0);
  double s, c;
  sincospi((double)k / (double)den, &s, &c);
  return make_double2(c, s);
}
__device__ __forceinline__ float2 phase_of(float2*, int k, int den) {
  if (den == 0) return make_float2(1.0f, 0.0f);
  float s, c;
  sincospif((float)k / (float)den, &s, &c);
  return make_float2(c, s);
}
template <class V> __device__ __forceinline__ V phase(int k, int den) { return phase_of((V*)nullptr, k, den); }


template <class V> __device__ __forceinline__ Re<V> sign_pow(Re<V> sigma, int e) {
  return (sigma < Re<V>(0) && (e & 1)) ? Re<V>(-1) : Re<V>(1);
}

// h_k and h_{n-k} of the Hermitian spectrum h = c_N + i c_S from the
// phased alias sums of k: A = sum_{m = k mod n, m >= 0} F'(m) and
// B = sum_{m = -k mod n, m >= 1} F'(m), F' = F e^{i m phi0} (F(0) real), so
// that c_k = A + conj B and c_{n-k} = B + conj A. e0, o0: E and O of m = 0
// (used for k = 0). Bluestein rings store conj(h_k) c_k (chirp) instead.
template <class V>
__device__ __forceinline__ void store_spectrum(V* buf, const PairInfo<V>& q, int k, V aN, V aS, V bN, V bS, V e0,
                                               V o0, V chk, V chnk) {
  const int n = q.n;
  if (k == 0 || 2 * k == n) {
    // k = 0: B = A without the m = 0 term; k = n/2: the two alias sets coincide
    bN = aN;
    bS = aS;
    if (k == 0) {
      bN.x -= e0.x + o0.x;
      bS.x -= e0.x - o0.x;
    }
  }
  V cn = add2(aN, conj2(bN)), cs = add2(aS, conj2(bS));
  V cnn = add2(bN, conj2(aN)), csn = add2(bS, conj2(aS));
  if (q.equator) cs = csn = zero<V>();
  V hk = mk<V>(cn.x - cs.y, cn.y + cs.x);
  V hnk = mk<V>(cnn.x - csn.y, cnn.y + csn.x);
  if (q.blue) {
    hk = cmul(conj2(hk), chk);
    if (k > 0) hnk = cmul(conj2(hnk), chnk);
  }
  buf[pad(k)] = hk;
  if (k > 0) buf[pad(n - k)] = hnk;   // k = n/2 writes the same value twice
}

// further aliases m = first + s n (s = 1, 2, ...) of one set, signed sigma^s
template <class V>
__device__ __forceinline__ void more_aliases(const V* __restrict__ eo, int mmax, int n, Re<V> sigma, int first, V& sN,
                                             V& sS) {
  Re<V> sg = sigma;
  for (int m = first + n; m <= mmax; m += n) {
    const V E = eo[2 * m], O = eo[2 * m + 1];
    sN = add2(sN, scl(sg, add2(E, O)));
    sS = add2(sS, scl(sg, sub2(E, O)));
    sg *= sigma;
  }
}

template <class V>
__device__ void spectrum(V* buf, Re<V>* scratch, const PairInfo<V>& q, const V* __restrict__ eo, int mmax) {
  const int n = q.n, nk = n / 2 + 1;
  const int B = blockDim.x;
  const int S = B / nk;
  const V e0 = eo[0], o0 = eo[1];
  if (S <= 1) {
    // frequencies k = t + u B, two at a time: the first alias of both sets
    // (and the chirp) of both is loaded before any use
    constexpr int U = 2;
    for (int k0 = threadIdx.x; k0 < nk; k0 += U * B) {
    V ea[U], oa[U], eb[U], ob[U], ca[U], cb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * B;
      ea[u] = oa[u] = eb[u] = ob[u] = ca[u] = cb[u] = zero<V>();
      if (k < nk) {
        if (k <= mmax) {
          ea[u] = eo[2 * k];
          oa[u] = eo[2 * k + 1];
        }
        const int mb = n - k;
        if (k > 0 && 2 * k != n && mb <= mmax) {
          eb[u] = eo[2 * mb];
          ob[u] = eo[2 * mb + 1];
        }
        if (q.blue) {
          ca[u] = q.chirp[k];
          if (k > 0) cb[u] = q.chirp[n - k];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * B;
      if (k < nk) {
        V aN = add2(ea[u], oa[u]), aS = sub2(ea[u], oa[u]);
        if (k == 0) aN.y = aS.y = Re<V>(0);
        if (k <= mmax) more_aliases(eo, mmax, n, q.sigma, k, aN, aS);
        V bN = zero<V>(), bS = zero<V>();
        if (k > 0 && 2 * k != n && n - k <= mmax) {
          V tN = add2(eb[u], ob[u]), tS = sub2(eb[u], ob[u]);
          more_aliases(eo, mmax, n, q.sigma, n - k, tN, tS);
          bN = scl(q.sigma, tN);
          bS = scl(q.sigma, tS);
        }
        const V ph = phase<V>(k, q.den);
        aN = cmul(aN, ph);
        aS = cmul(aS, ph);
        bN = cmul(bN, conj2(ph));
        bS = cmul(bS, conj2(ph));
        store_spectrum(buf, q, k, aN, aS, bN, bS, e0, o0, ca[u], cb[u]);
      }
    }
    }
    return;
  }
  // small rings: the alias sums of one k are split over S threads (aliases
  // s, s + S, ... of each set) and combined in a fixed order through LDS
  const int t = threadIdx.x;
  const int k = t / S, s = t % S;
  V aN = zero<V>(), aS = zero<V>(), bN = zero<V>(), bS = zero<V>();
  if (k < nk) {
    for (int j = s, m = k + s * n; m <= mmax; j += S, m += S * n) {
      const V E = eo[2 * m], O = eo[2 * m + 1];
      V fn = add2(E, O), fs = sub2(E, O);
      if (m == 0) fn.y = fs.y = Re<V>(0);
      const Re<V> sg = sign_pow<V>(q.sigma, j);
      aN = add2(aN, scl(sg, fn));
      aS = add2(aS, scl(sg, fs));
    }
    if (k > 0 && 2 * k != n) {
      for (int j = s, m = n - k + s * n; m <= mmax; j += S, m += S * n) {
        const V E = eo[2 * m], O = eo[2 * m + 1];
        const Re<V> sg = sign_pow<V>(q.sigma, j + 1);
        bN = add2(bN, scl(sg, add2(E, O)));
        bS = add2(bS, scl(sg, sub2(E, O)));
      }
    }
  }
  Re<V>* sc = scratch + (size_t)t * 8;
  sc[0] = aN.x; sc[1] = aN.y; sc[2] = aS.x; sc[3] = aS.y;
  sc[4] = bN.x; sc[5] = bN.y; sc[6] = bS.x; sc[7] = bS.y;
  lds_barrier();
  if (k < nk && s == 0) {
    for (int u = 1; u < S; ++u) {
      const Re<V>* o = scratch + (size_t)(t + u) * 8;
      aN.x += o[0]; aN.y += o[1]; aS.x += o[2]; aS.y += o[3];
      bN.x += o[4]; bN.y += o[5]; bS.x += o[6]; bS.y += o[7];
    }
    const V ph = phase<V>(k, q.den);
    aN = cmul(aN, ph);
    aS = cmul(aS, ph);
    bN = cmul(bN, conj2(ph));
    bS = cmul(bS, conj2(ph));
    const V ck = q.blue ? q.chirp[k] : zero<V>();
    const V cnk = (q.blue && k > 0) ? q.chirp[n - k] : zero<V>();
    store_spectrum(buf, q, k, aN, aS, bN, bS, e0, o0, ck, cnk);
  }
  lds_barrier();   // scratch is read before anything else is written there
}

// multiply buf[0..L) by the ring's Bluestein kernel (loads issued first)
template <class V>
__device__ __forceinline__ void kern_mul(V* buf, const PairInfo<V>& q) {
  constexpr int U = 8;   // L <= 8 blockDim
  V kv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = threadIdx.x + u * blockDim.x;
    kv[u] = j < q.L ? q.kern[j] : zero<V>();
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = threadIdx.x + u * blockDim.x;
    if (j < q.L) buf[pad(j)] = cmul(buf[pad(j)], kv[u]);
  }
}

// Z_j = map_N[j] + i map_S[j] for j < n, left in buf[0..n) (natural order)
template <class V>
__device__ void ring_inverse(V* buf, Re<V>* scratch, const PairInfo<V>& q, const V* __restrict__ eo, int mmax,
                             const V* __restrict__ tw, int lf) {
  spectrum(buf, scratch, q, eo, mmax);
  if (!q.blue) {
    fft_pow2(buf, q.n, tw, lf, true);
  } else {
    // IDFT(h) = conj(DFT(conj h)); DFT by chirp-z
    for (int j = q.n + threadIdx.x; j < q.L; j += blockDim.x) buf[pad(j)] = zero<V>();
    fft_pow2(buf, q.L, tw, lf, false);
    kern_mul(buf, q);
    fft_pow2(buf, q.L, tw, lf, true);
    for (int j = threadIdx.x; j < q.n; j += blockDim.x) buf[pad(j)] = conj2(cmul(buf[pad(j)], q.chirp[j]));
    lds_barrier();
  }
}

// forward DFT of z_j (buf[0..n), natural order) in place; X_k in buf[k],
// except that Bluestein rings leave X_k / c_k (the final chirp factor is
// applied where the spectrum is read, in write_geo)
template <class V>
__device__ void ring_forward(V* buf, const PairInfo<V>& q, const V* __restrict__ tw, int lf) {
  if (!q.blue) {
    fft_pow2(buf, q.n, tw, lf, false);
  } else {
    for (int j = threadIdx.x; j < q.L; j += blockDim.x)
      buf[pad(j)] = j < q.n ? cmul(buf[pad(j)], q.chirp[j]) : zero<V>();
    fft_pow2(buf, q.L, tw, lf, false);
    kern_mul(buf, q);
    fft_pow2(buf, q.L, tw, lf, true);
  }
}

// G_E = G_N + G_S and G_O = G_N - G_S for m = 0..mmax, by frequency k = m mod n
template <class V>
__device__ void write_geo(V* __restrict__ geo, const V* buf, const PairInfo<V>& q, int mmax) {
  const int n = q.n;
  const int kmax = n < mmax + 1 ? n : mmax + 1;
  for (int k = threadIdx.x; k < kmax; k += blockDim.x) {
    const int kn = (n - k) % n;
    V X = buf[pad(k)], Xm = buf[pad(kn)];
    if (q.blue) {
      X = cmul(X, q.chirp[k]);
      Xm = cmul(Xm, q.chirp[kn]);
    }
    Xm = conj2(Xm);
    const Re<V> h = Re<V>(0.5);
    // X_N = (X + conj X(-k))/2, X_S = (X - conj X(-k))/(2i)
    const V XN = mk<V>(h * (X.x + Xm.x), h * (X.y + Xm.y));
    const V XS = mk<V>(h * (X.y - Xm.y), -h * (X.x - Xm.x));
    const V ph = conj2(phase<V>(k, q.den));
    const V GN = cmul(XN, ph);
    const V GS = q.equator ? zero<V>() : cmul(XS, ph);
    V gE = add2(GN, GS), gO = sub2(GN, GS);
    for (int m = k; m <= mmax; m += n) {
      geo[2 * m] = gE;
      geo[2 * m + 1] = gO;
      gE = scl(q.sigma, gE);
      gO = scl(q.sigma, gO);
    }
  }
}

template <class V, int MODE, int NT>
__global__ __launch_bounds__(NT) void k_ring(Tables T, int nside, int mmax, int fmax, const int* __restrict__ pairs,
                                              int npc, int nrhs, int Lc, const V* __restrict__ tw,
                                              const V* __restrict__ chirp, const V* __restrict__ kern,
                                              const V* __restrict__ eo, int64_t eo_stride, double* __restrict__ map,
                                              int64_t map_stride, const double* __restrict__ ninv,
                                              V* __restrict__ geo, int64_t geo_stride, RingCols rc,
                                              const int* __restrict__ pred) {
  if (pred && *pred) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  V* buf = reinterpret_cast<V*>(lds_raw);
  // spectrum scratch of small rings (blockDim x 8 reals) in the upper half
  Re<V>* scratch = reinterpret_cast<Re<V>*>(buf + pad(Lc / 2));
  // blocks b, b + 8, ... run on one XCD: give them consecutive (pair, column) items
  const int b = blockIdx.x;
  const int g = (b & 7) * (int)(gridDim.x >> 3) + (b >> 3);
  if (g >= npc * nrhs) return;
  const int p = pairs[g / nrhs], c = g % nrhs;
  const PairInfo<V> q = pair_info<V>(T, p, nside, chirp, kern);
  const int lf = ilog2(fmax);   // the twiddle table has fmax = 2^lf entries
  // logical column c = component kc of group gq (T+Q+U plans: 3 maps per group)
  const int gq = c / rc.group, kc = c % rc.group;
  const V* __restrict__ eop = eo + ((int64_t)gq * rc.eo_cols + kc) * eo_stride + (size_t)p * (mmax + 1) * 2;
  V* __restrict__ geop = geo + ((int64_t)gq * rc.geo_cols + kc) * geo_stride + (size_t)p * (mmax + 1) * 2;
  double* __restrict__ mp = map + c * map_stride;
  if (ninv) ninv += kc * rc.ninv_stride;

  // m above the pair's last live m: no Legendre sums to fold, no G written
  const int mtop = rc.mtop ? min(mmax, rc.mtop[p]) : mmax;
  if (MODE == RING_FUSED) {
    ring_inverse(buf, scratch, q, eop, mtop, tw, lf);
    // N^-1 of the ring (n <= 8 blockDim): all loads issued before the
    // products, without per-lane conditions (indices past the ring read its
    // first pixel; the values are not used)
    constexpr int U = 8;
    double wn[U], ws[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = threadIdx.x + u * blockDim.x;
      const int jj = j < q.n ? j : 0;
      wn[u] = ninv[q.fn + jj];
      ws[u] = ninv[(q.equator ? q.fn : q.fs) + jj];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = threadIdx.x + u * blockDim.x;
      if (j < q.n) {
        const V Z = buf[pad(j)];
        buf[pad(j)] = mk<V>(Z.x * (Re<V>)wn[u], q.equator ? Re<V>(0) : Z.y * (Re<V>)ws[u]);
      }
    }
  } else if (MODE == RING_SYNTH) {
    ring_inverse(buf, scratch, q, eop, mmax, tw, lf);
    for (int j = threadIdx.x; j < q.n; j += blockDim.x) {
      const V Z = buf[pad(j)];
      mp[q.fn + j] = (double)Z.x;
      if (!q.equator) mp[q.fs + j] = (double)Z.y;
    }
    return;
  } else {  // RING_ADJOINT: load the pixels
    for (int j = threadIdx.x; j < q.n; j += blockDim.x)
      buf[pad(j)] = mk<V>((Re<V>)mp[q.fn + j], q.equator ? Re<V>(0) : (Re<V>)mp[q.fs + j]);
  }
  ring_forward(buf, q, tw, lf);
  lds_barrier();
  write_geo(geop, buf, q, mtop);
}

// threads of a class of FFT length Lc with Lc / div points per thread
// (the kernels need at least Lc / 8 threads)
int ring_threads(int Lc, int div = 8) {
  const int t = Lc / (div < 8 ? div : 8);
  return t < 64 ? 64 : t > 1024 ? 1024 : t;
}

template <class V>
size_t ring_lds(int Lc) {
  return (size_t)(Lc + Lc / 16) * sizeof(V);
}

template <class V, int MODE>
hipError_t ring_launch(const crsht_plan* P, int nrhs, const V* eo, double* map, const double* ninv, V* geo,
                       const V* tw, const V* chirp, const V* kern, RingCols cols, hipStream_t s) {
  const Geometry& g = P->g;
  const int64_t stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  // the classes are independent (disjoint ring pairs): class 0 runs on the
  // caller's stream, class k > 0 on auxiliary stream (k - 1) mod kAux,
  // forked from and joined back to it (parallel branches when captured), so
  // that the short launches of the small-ring classes overlap the large ones
  const int ncls = (int)P->ring_cls.size();
  const int naux = ncls - 1 < crsht_plan::kAux ? ncls - 1 : crsht_plan::kAux;
  hipError_t e;
  if ((e = aux_fork(P, naux, s)) != hipSuccess) return e;
  for (int k = 0; k < ncls; ++k) {
    const RingClass& rc = P->ring_cls[k];
    const size_t lds = ring_lds<V>(rc.L);
    const int nt = ring_class_threads(P, k);
    const int64_t items = (int64_t)rc.count * nrhs;
    const unsigned nb = (unsigned)((items + 7) / 8 * 8);
    hipStream_t q = aux_q(P, k, s);
#define CRSHT_RING_LAUNCH(NT)                                                                                   \
  do {                                                                                                          \
    hipLaunchKernelGGL((k_ring<V, MODE, NT>), dim3(nb), dim3(nt), lds, q, P->t, g.nside, g.mmax, g.fft_max,      \
                       P->t.ring_pairs + rc.off, rc.count, nrhs, rc.L, tw, chirp, kern, eo, stride, map,         \
                       (int64_t)g.npix, ninv, geo, stride, cols, P->pred);                                      \
  } while (0)
    if (nt <= 512)
      CRSHT_RING_LAUNCH(512);
    else
      CRSHT_RING_LAUNCH(1024);
#undef CRSHT_RING_LAUNCH
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return aux_join(P, naux, s);
}

template <class V>
hipError_t ring_mode(const crsht_plan* P, int nrhs, RingMode mode, const V* eo, double* map, const double* ninv,
                     V* geo, const V* tw, const V* chirp, const V* kern, RingCols cols, hipStream_t s) {
  if (mode == RING_SYNTH) return ring_launch<V, RING_SYNTH>(P, nrhs, eo, map, ninv, geo, tw, chirp, kern, cols, s);
  if (mode == RING_ADJOINT)
    return ring_launch<V, RING_ADJOINT>(P, nrhs, eo, map, ninv, geo, tw, chirp, kern, cols, s);
  return ring_launch<V, RING_FUSED>(P, nrhs, eo, map, ninv, geo, tw, chirp, kern, cols, s);
}

// dynamic LDS above 64 KiB must be allowed per kernel before launches
template <class V, int MODE>
hipError_t ring_allow_lds(const crsht_plan* P) {
  for (const RingClass& rc : P->ring_cls) {
    const size_t lds = ring_lds<V>(rc.L);
    if (lds <= 65536) continue;
    // either instantiation may serve the class (tuned threads per workgroup)
    for (const void* f : {(const void*)k_ring<V, MODE, 512>, (const void*)k_ring<V, MODE, 1024>}) {
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace

// Classes above 512 hold rings of exactly their FFT length L (n > L/4), so
// with L/4 threads the spectrum still takes its one-thread-per-frequency path
// (the small-ring path with scratch of blockDim x 8 reals needs blockDim <=
// L/8): only those classes may take L/4 threads.
int ring_class_threads(const crsht_plan* P, int k) {
  const int L = P->ring_cls[k].L;
  const int div = (k < kMaxRingClasses && L >= 1024 && P->tune.ring_div[k] == 4) ? 4 : 8;
  return ring_threads(L, div);
}

hipError_t ring_prepare(const crsht_plan* P) {
  hipError_t e;
  if ((e = ring_allow_lds<float2, RING_SYNTH>(P)) != hipSuccess) return e;
  if ((e = ring_allow_lds<float2, RING_ADJOINT>(P)) != hipSuccess) return e;
  if ((e = ring_allow_lds<float2, RING_FUSED>(P)) != hipSuccess) return e;
  if ((e = ring_allow_lds<double2, RING_SYNTH>(P)) != hipSuccess) return e;
  if ((e = ring_allow_lds<double2, RING_ADJOINT>(P)) != hipSuccess) return e;
  return ring_allow_lds<double2, RING_FUSED>(P);
}

// classes of ring pairs by FFT length: pairs with L <= 512 share one class,
// every larger power of two has its own
void ring_classes(const std::vector<int>& fft_len, std::vector<RingClass>& cls, std::vector<int>& pairs) {
  cls.clear();
  pairs.clear();
  int Lmax = 512;
  for (int L : fft_len) Lmax = L > Lmax ? L : Lmax;
  for (int Lc = 512; Lc <= Lmax; Lc *= 2) {
    RingClass rc;
    rc.L = Lc;
    rc.off = (int)pairs.size();
    for (int p = 0; p < (int)fft_len.size(); ++p) {
      const int L = fft_len[p];
      if ((Lc == 512 && L <= 512) || (Lc > 512 && L == Lc)) pairs.push_back(p);
    }
    rc.count = (int)pairs.size() - rc.off;
    if (rc.count > 0) cls.push_back(rc);
  }
}

size_t ring_lds_bytes(const crsht_plan* P, bool f32) {
  size_t mx = 0;
  for (const RingClass& rc : P->ring_cls) {
    const size_t b = f32 ? ring_lds<float2>(rc.L) : ring_lds<double2>(rc.L);
    mx = b > mx ? b : mx;
  }
  return mx;
}

hipError_t aux_fork(const crsht_plan* P, int n, hipStream_t s) {
  if (n <= 0 || P->aux_off) return hipSuccess;
  hipError_t e = hipEventRecord(P->aux_fork_ev, s);
  for (int a = 0; a < n && e == hipSuccess; ++a) e = hipStreamWaitEvent(P->aux_stream[a], P->aux_fork_ev, 0);
  return e;
}

hipError_t aux_join(const crsht_plan* P, int n, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (P->aux_off) return e;
  for (int a = 0; a < n && e == hipSuccess; ++a) {
    e = hipEventRecord(P->aux_join_ev[a], P->aux_stream[a]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, P->aux_join_ev[a], 0);
  }
  return e;
}

hipStream_t aux_q(const crsht_plan* P, int k, hipStream_t s) {
  return (k == 0 || P->aux_off) ? s : P->aux_stream[(k - 1) % crsht_plan::kAux];
}

hipError_t launch_ring(const crsht_plan* P, int nrhs, RingMode mode, const void* eo, double* map,
                       const double* ninv, void* geo, bool f32, hipStream_t s, RingCols cols) {
  // timed: the fused operator passes, FP32 (id 2) and FP64 (id 6) apart
  const int tid = mode == RING_FUSED ? (f32 ? 2 : 6) : -1;
  timing_begin(P, tid, s);
  hipError_t e;
  if (f32 && mode == RING_FUSED && P->ncomp == 1) cols.mtop = P->t.pair_mtop;
  if (f32)
    e = ring_mode<float2>(P, nrhs, mode, (const float2*)eo, map, ninv, (float2*)geo, P->t.twiddle32, P->t.bs_chirp32,
                          P->t.bs_kern32, cols, s);
  else
    e = ring_mode<double2>(P, nrhs, mode, (const double2*)eo, map, ninv, (double2*)geo, P->t.twiddle, P->t.bs_chirp,
                           P->t.bs_kern, cols, s);
  timing_end(P, tid, s);
  return e;
}

}  // namespace crsht
