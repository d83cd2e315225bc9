// Spin-2 (polarisation) part of the transforms of T+Q+U plans, built around
// the scalar Legendre kernels.
//
// Convention (HEALPix / COSMO): Q +- iU = sum (+-2 a_lm)(+-2 Y_lm) with
// +-2 a = -(a_E +- i a_B) and +-2Y_lm = (W_lm +- X_lm) e^{i m phi}, where, with
// c = cos(theta), s = sin(theta), F_lm = sqrt((2l+1)/(2l-1) (l^2 - m^2)) and
// N_l = sqrt((l-1) l (l+1) (l+2)) (l >= 2),
//   W_lm = ( -2 ((l - m^2)/s^2 + l(l-1)/2) lambda_l + 2 c F_lm / s^2 lambda_{l-1} ) / N_l
//   X_lm = -2 m / s^2 ( (l-1) c lambda_l - F_lm lambda_{l-1} ) / N_l
// (the spin-raising operators applied twice to Y_lm). The per-ring spectra
// of Q and U are G_Q = -sum_l (a_E W + i a_B X) and G_U = -sum_l (a_B W - i a_E X).
//
// Every l-sum is a scalar Legendre sum sum_l lambda_l q_l of a derived
// coefficient array, with the ring-dependent factors 1/s^2, c/s^2 applied
// afterwards:
//   sum_l a W = -2/s^2 (T1 - m^2 T0) + 2 c/s^2 T3 - (T2 - T1),
//   sum_l a X = -2 m c/s^2 (T1 - T0) + 2 m/s^2 T3,
// T0 = sum lambda_l a_l/N_l, T1 = sum lambda_l l a_l/N_l, T2 = sum lambda_l l^2 a_l/N_l,
// T3 = sum lambda_l F_{l+1} a_{l+1}/N_{l+1}. The synthesis of one T+Q+U column
// is therefore: coefficient preparation (9 scalar columns: T, T0..T3 of E,
// T0..T3 of B), the scalar Legendre synthesis of those 9 columns, and a
// per-(ring pair, m) combination into the Q and U spectra. The transpose
// weights the azimuthal adjoints G^_Q, G^_U by 1/s^2 and c/s^2 per ring,
// takes 7 scalar Legendre adjoints (T, Q, U, Q/s^2, Q c/s^2, U/s^2, U c/s^2)
// and combines per (l, m):
//   sum_r W G^ = ( -2 (l - m^2) R1(l) - l (l-1) R0(l) + 2 F_lm R2(l-1) ) / N_l
//   sum_r X G^ = ( -2 m (l-1) R2(l) + 2 m F_lm R1(l-1) ) / N_l
//   a_E = -W G^_Q - i X G^_U,   a_B = i X G^_Q - W G^_U.
// Legendre sums are kept in the (E, O) = (north + south, north - south) form
// of the scalar kernels; a factor odd in z (c) swaps E and O.
#include "internal.h"
#include "devutil.h"

namespace crsht {
namespace {

constexpr int kVecT = 256;

__device__ __forceinline__ double ninv_l(int l) {
  return l < 2 ? 0.0 : 1.0 / sqrt(((double)l - 1.0) * l * (l + 1.0) * (l + 2.0));
}
__device__ __forceinline__ double fcoef(int l, int m) {
  return sqrt((2.0 * l + 1.0) / (2.0 * l - 1.0) * ((double)l * l - (double)m * m));
}
__device__ __forceinline__ double2 sc2(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 ad2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 sb2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 mul_i(double2 a) { return make_double2(-a.y, a.x); }

__device__ __forceinline__ double2 ld2(const double2* p) { return *p; }
__device__ __forceinline__ double2 ld2(const float2* p) { const float2 v = *p; return make_double2(v.x, v.y); }
__device__ __forceinline__ void st2(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void st2(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

// 9 scalar coefficient columns per T+Q+U column: kappa f a_T, then for E and B
// kappa f a / N_l x (1, l, l^2) and kappa_l F_{l+1} f_{l+1} a_{l+1} / N_{l+1}.
// alm: [nrhs][3][nalm]; out: [nrhs][9][nalm]; f (per element) may be null.
__global__ void k_pol_prep_synth(int64_t nalm, int nrhs, const int* __restrict__ idx_l,
                                 const int* __restrict__ idx_m, const double* __restrict__ kappa,
                                 const double* __restrict__ f, const double2* __restrict__ alm,
                                 double2* __restrict__ out, const int* __restrict__ pred) {
  if (pred && *pred) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const int l = idx_l[i], m = idx_m[i];
  const double kap = kappa[i];
  const double fi = f ? f[i] : 1.0;
  const bool next = (i + 1 < nalm) && idx_m[i + 1] == m;   // (l+1, m) is the next element
  const double q = kap * fi * ninv_l(l);
  const double q3 = next ? kap * fcoef(l + 1, m) * (f ? f[i + 1] : 1.0) * ninv_l(l + 1) : 0.0;
  for (int c = 0; c < nrhs; ++c) {
    const double2* a = alm + (int64_t)c * 3 * nalm;
    double2* o = out + (int64_t)c * 9 * nalm;
    o[i] = sc2(kap * fi, a[i]);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double2 v = a[(1 + k) * nalm + i];
      double2* ok = o + (1 + 4 * k) * nalm;
      ok[0 * nalm + i] = sc2(q, v);
      ok[1 * nalm + i] = sc2(q * l, v);
      ok[2 * nalm + i] = sc2(q * l * l, v);
      ok[3 * nalm + i] = next ? sc2(q3, a[(1 + k) * nalm + i + 1]) : make_double2(0.0, 0.0);
    }
  }
}

// Q and U spectra (E/O form) of column group c from its 8 polarisation sums,
// written over group columns 1 (Q) and 2 (U). eo: [groups][9][pairs][mmax+1][2].
template <class V>
__global__ void k_pol_combine_synth(int npairs, int mmax, int nrhs, const double* __restrict__ pair_z, V* eo,
                                    int64_t col_stride, const int* __restrict__ pred) {
  if (pred && *pred) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)npairs * (mmax + 1)) return;
  const int p = (int)(t / (mmax + 1)), m = (int)(t % (mmax + 1));
  const double z = pair_z[p];
  const double is2 = 1.0 / ((1.0 - z) * (1.0 + z));
  const double mm = (double)m;
  for (int c = 0; c < nrhs; ++c) {
    V* g = eo + (int64_t)c * 9 * col_stride + t * 2;
    double2 E[8], O[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      E[k] = ld2(g + (1 + k) * col_stride);
      O[k] = ld2(g + (1 + k) * col_stride + 1);
    }
    double2 gq[2], gu[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const double cz = side ? -z : z;
      double2 W[2], X[2];
#pragma unroll
      for (int comp = 0; comp < 2; ++comp) {
        double2 T[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) T[k] = side ? sb2(E[4 * comp + k], O[4 * comp + k]) : ad2(E[4 * comp + k], O[4 * comp + k]);
        W[comp] = sb2(ad2(sc2(-2.0 * is2, sb2(T[1], sc2(mm * mm, T[0]))), sc2(2.0 * cz * is2, T[3])), sb2(T[2], T[1]));
        X[comp] = ad2(sc2(-2.0 * mm * cz * is2, sb2(T[1], T[0])), sc2(2.0 * mm * is2, T[3]));
      }
      // G_Q = -(W_E + i X_B), G_U = -(W_B - i X_E)
      gq[side] = sc2(-1.0, ad2(W[0], mul_i(X[1])));
      gu[side] = sc2(-1.0, sb2(W[1], mul_i(X[0])));
    }
    st2(g + 1 * col_stride, sc2(0.5, ad2(gq[0], gq[1])));
    st2(g + 1 * col_stride + 1, sc2(0.5, sb2(gq[0], gq[1])));
    st2(g + 2 * col_stride, sc2(0.5, ad2(gu[0], gu[1])));
    st2(g + 2 * col_stride + 1, sc2(0.5, sb2(gu[0], gu[1])));
  }
}

// Ring-weighted copies of the azimuthal adjoints of Q and U (group columns 1,
// 2) into group columns 3..6: Q/s^2, Q c/s^2, U/s^2, U c/s^2 (E/O form; the odd
// factor c swaps E and O). geo: [groups][7][pairs][mmax+1][2].
template <class V>
__global__ void k_pol_pre_adjoint(int npairs, int mmax, int nrhs, const double* __restrict__ pair_z, V* geo,
                                  int64_t col_stride, const int* __restrict__ pred) {
  if (pred && *pred) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)npairs * (mmax + 1)) return;
  const int p = (int)(t / (mmax + 1));
  const double z = pair_z[p];
  const double is2 = 1.0 / ((1.0 - z) * (1.0 + z)), cs2 = z * is2;
  for (int c = 0; c < nrhs; ++c) {
    V* g = geo + (int64_t)c * 7 * col_stride + t * 2;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double2 e = ld2(g + (1 + k) * col_stride), o = ld2(g + (1 + k) * col_stride + 1);
      V* d = g + (3 + 2 * k) * col_stride;
      st2(d, sc2(is2, e));
      st2(d + 1, sc2(is2, o));
      st2(d + col_stride, sc2(cs2, o));
      st2(d + col_stride + 1, sc2(cs2, e));
    }
  }
}

// a = f * (T, E, B) from the 7 raw Legendre adjoints of each group (raw:
// [nrhs][7][nalm], sums of mu = lambda / kappa); out: [nrhs][3][nalm].
__global__ void k_pol_combine_adjoint(int64_t nalm, int nrhs, const int* __restrict__ idx_l,
                                      const int* __restrict__ idx_m, const double* __restrict__ kappa,
                                      const double* __restrict__ f, const double2* __restrict__ raw,
                                      double2* __restrict__ out, const int* __restrict__ pred) {
  if (pred && *pred) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const int l = idx_l[i], m = idx_m[i];
  const double kap = kappa[i];
  const bool prev = l > m;                                   // (l-1, m) is the previous element
  const double kap1 = prev ? kappa[i - 1] : 0.0;
  const double fi = f ? f[i] : 1.0;
  const double n = ninv_l(l), F = prev ? fcoef(l, m) : 0.0, mm = (double)m;
  for (int c = 0; c < nrhs; ++c) {
    const double2* r = raw + (int64_t)c * 7 * nalm;
    double2* o = out + (int64_t)c * 3 * nalm;
    o[i] = sc2(fi * kap, r[i]);
    if (l < 2) {
      o[nalm + i] = make_double2(0.0, 0.0);
      o[2 * nalm + i] = make_double2(0.0, 0.0);
      continue;
    }
    double2 Ws[2], Xs[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {                           // k = 0: Q, 1: U
      const double2 R0 = sc2(kap, r[(1 + k) * nalm + i]);
      const double2 R1 = sc2(kap, r[(3 + 2 * k) * nalm + i]);
      const double2 R2 = sc2(kap, r[(4 + 2 * k) * nalm + i]);
      const double2 R1m = prev ? sc2(kap1, r[(3 + 2 * k) * nalm + i - 1]) : make_double2(0.0, 0.0);
      const double2 R2m = prev ? sc2(kap1, r[(4 + 2 * k) * nalm + i - 1]) : make_double2(0.0, 0.0);
      Ws[k] = sc2(n, ad2(sb2(sc2(-2.0 * (l - mm * mm), R1), sc2((double)l * (l - 1.0), R0)), sc2(2.0 * F, R2m)));
      Xs[k] = sc2(n * mm, ad2(sc2(-2.0 * (l - 1.0), R2), sc2(2.0 * F, R1m)));
    }
    // a_E = -W Q^ - i X U^,  a_B = i X Q^ - W U^
    const double2 aE = sb2(sc2(-1.0, Ws[0]), mul_i(Xs[1]));
    const double2 aB = sb2(mul_i(Xs[0]), Ws[1]);
    o[nalm + i] = sc2(fi, aE);
    o[2 * nalm + i] = sc2(fi, aB);
  }
}

// per-l spectra blocks: sblk[l] = (S^-1: TT, TE, EE, BB, S^-1/2: TT, TE, EE, BB)
__device__ __forceinline__ void block3(const double* s, double2 t, double2 e, double2 b, double2& ot, double2& oe,
                                       double2& ob) {
  ot = ad2(sc2(s[0], t), sc2(s[1], e));
  oe = ad2(sc2(s[1], t), sc2(s[2], e));
  ob = sc2(s[3], b);
}

// q = camp[c].x S^-1 p + dterm (3x3 blocks per l; S^-1 term omitted when sblk
// is null) per column c; partial <p, q> per block
__global__ void k_cg_q_tqu(int64_t nalm, const int* __restrict__ idx_l, const int* __restrict__ idx_m,
                           const double* __restrict__ sblk, const double2* __restrict__ camp,
                           const double2* __restrict__ p, const double2* __restrict__ dterm, double2* __restrict__ q,
                           double* __restrict__ partial, int npart, const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ double sh[kVecT];
  const int c = blockIdx.y;
  const double qa = camp[c].x;
  const int64_t base = (int64_t)c * 3 * nalm;
  double pq = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x) {
    const int m = idx_m[i];
    const double* s = sblk ? sblk + 8 * idx_l[i] : nullptr;
    const double2 pt = p[base + i], pe = p[base + nalm + i], pb = p[base + 2 * nalm + i];
    double2 qt = dterm[base + i], qe = dterm[base + nalm + i], qb = dterm[base + 2 * nalm + i];
    if (sblk) {
      double2 st, se, sb;
      block3(s, pt, pe, pb, st, se, sb);
      qt = ad2(qt, sc2(qa, st));
      qe = ad2(qe, sc2(qa, se));
      qb = ad2(qb, sc2(qa, sb));
    }
    q[base + i] = qt;
    q[base + nalm + i] = qe;
    q[base + 2 * nalm + i] = qb;
    pq += wdot(m, pt, qt) + wdot(m, pe, qe) + wdot(m, pb, qb);
  }
  pq = block_sum(pq, sh);
  if (threadIdx.x == 0) partial[(size_t)c * npart * 4 + blockIdx.x] = pq;
}

// partial of a^T S^-1 a (3x3 blocks per l, real-field product) per block
__global__ void k_alm_wquad_tqu(int64_t nalm, const int* __restrict__ idx_l, const int* __restrict__ idx_m,
                                const double* __restrict__ sblk, const double2* __restrict__ a,
                                double* __restrict__ partial) {
  __shared__ double sh[kVecT];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x) {
    const int m = idx_m[i];
    const double2 t = a[i], e = a[nalm + i], b = a[2 * nalm + i];
    double2 ot, oe, ob;
    block3(sblk + 8 * idx_l[i], t, e, b, ot, oe, ob);
    acc += wdot(m, t, ot) + wdot(m, e, oe) + wdot(m, b, ob);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// out = dterm + camp[c].y S^-1/2 w0 per column c (either term may be null),
// Im of m = 0 set to 0
__global__ void k_rhs_finish_tqu(int64_t nalm, int nrhs, const int* __restrict__ idx_l, const int* __restrict__ idx_m,
                                 const double* __restrict__ sblk, const double2* __restrict__ camp,
                                 const double2* __restrict__ dterm, const double2* __restrict__ w0,
                                 double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const bool m0 = idx_m[i] == 0;
  const double* s = sblk + 8 * idx_l[i] + 4;
  for (int c = 0; c < nrhs; ++c) {
    const int64_t base = (int64_t)c * 3 * nalm;
    double2 v[3] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    if (dterm)
      for (int k = 0; k < 3; ++k) v[k] = dterm[base + k * nalm + i];
    if (w0) {
      double2 a, b, d;
      block3(s, w0[base + i], w0[base + nalm + i], w0[base + 2 * nalm + i], a, b, d);
      const double qh = camp[c].y;
      v[0] = ad2(v[0], sc2(qh, a));
      v[1] = ad2(v[1], sc2(qh, b));
      v[2] = ad2(v[2], sc2(qh, d));
    }
    for (int k = 0; k < 3; ++k) {
      if (m0) v[k].y = 0.0;
      out[base + k * nalm + i] = v[k];
    }
  }
}

// Jacobi diagonal [3][nalm]: (S^-1)_kk + bk^2 raw_k (raw_T with the T ring
// weights, raw_P with the polarisation ones), 1 on modes not kept
__global__ void k_diag_tqu(int64_t nalm, const int* __restrict__ idx_l, const double* __restrict__ sblk,
                           const double* __restrict__ bk, const double* __restrict__ keep,
                           const double2* __restrict__ rawt, const double2* __restrict__ rawp,
                           double* __restrict__ diag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const double* s = sblk + 8 * idx_l[i];
  const double b2 = bk[i] * bk[i];
  const bool kp = keep[i] > 0.0;
  diag[i] = kp ? fma(b2, rawt[i].x, s[0]) : 1.0;
  diag[nalm + i] = kp ? fma(b2, rawp[i].x, s[2]) : 1.0;
  diag[2 * nalm + i] = kp ? fma(b2, rawp[i].x, s[3]) : 1.0;
}

// per-element arrays from the per-l blocks (perl rows: 2 = b_l, 3 = keep)
__global__ void k_expand_tqu(int64_t nalm, int lmax, const int* __restrict__ idx_l, const double* __restrict__ kappa,
                             const double* __restrict__ sblk, const double* __restrict__ perl,
                             double* __restrict__ sinv, double* __restrict__ sinvhalf, double* __restrict__ bk,
                             double* __restrict__ bl_keep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const int l = idx_l[i];
  const double keep = perl[3 * (lmax + 1) + l];
  const double b = keep * perl[2 * (lmax + 1) + l];
  const double* s = sblk + 8 * l;
  sinv[i] = keep * s[0];
  sinv[nalm + i] = keep * s[2];
  sinv[2 * nalm + i] = keep * s[3];
  sinvhalf[i] = keep * s[4];
  sinvhalf[nalm + i] = keep * s[6];
  sinvhalf[2 * nalm + i] = keep * s[7];
  const double bkv = b * kappa[i];
  bk[i] = bkv;
  bk[nalm + i] = bkv;
  bk[2 * nalm + i] = bkv;
  bl_keep[i] = b;
}

int nblk(int64_t n) { return (int)((n + kVecT - 1) / kVecT); }


// ---- polar rings of the mixed path: ring pairs [0, npol), whose Q and U
// divide cancelling Legendre sums by sin^2 theta, are summed in FP64 in
// buffers of npol pairs per column (pol64: [nrhs][ncol][npol][mmax+1][2])
// next to the float2 buffers of all pairs ([nrhs][ncol][npairs][mmax+1][2]).
// T, Q, U spectra (group columns 0..2) of the polar pairs: FP64 -> float2
__global__ void k_polar_spectra_to_f32(int npol, int mmax, int nrhs, const double2* __restrict__ pol64,
                                       int64_t col64, float2* __restrict__ eo, int64_t col32,
                                       const int* __restrict__ pred) {
  if (pred && *pred) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (pair, m, E/O) entry of a column
  const int64_t n = (int64_t)npol * (mmax + 1) * 2;
  if (t >= n) return;
  for (int c = 0; c < nrhs; ++c)
    for (int k = 0; k < 3; ++k) {
      const double2 v = pol64[((int64_t)c * 9 + k) * col64 + t];
      eo[((int64_t)c * 9 + k) * col32 + t] = make_float2((float)v.x, (float)v.y);
    }
}

// azimuthal adjoints T, Q, U (group columns 0..2) of the polar pairs:
// float2 -> FP64, and those float2 entries set to 0 (the weighted copies that
// the pre-adjoint step then derives from them are 0 as well)
__global__ void k_polar_geo_to_f64(int npol, int mmax, int nrhs, float2* __restrict__ geo, int64_t col32,
                                   double2* __restrict__ pol64, int64_t col64, const int* __restrict__ pred) {
  if (pred && *pred) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)npol * (mmax + 1) * 2;
  if (t >= n) return;
  for (int c = 0; c < nrhs; ++c) {
    for (int k = 0; k < 3; ++k) {
      float2* gk = geo + ((int64_t)c * 7 + k) * col32 + t;
      const float2 v = *gk;
      pol64[((int64_t)c * 7 + k) * col64 + t] = make_double2((double)v.x, (double)v.y);
      *gk = make_float2(0.f, 0.f);
    }
  }
}

}  // namespace

hipError_t launch_pol_prep_synth(const crsht_plan* P, int nrhs, const double2* alm, const double* f, double2* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_pol_prep_synth, dim3(nblk(P->g.nalm)), dim3(kVecT), 0, s, P->g.nalm, nrhs, P->t.idx_l,
                     P->t.idx_m, P->t.rec_kappa, f, alm, out, P->pred);
  return hipGetLastError();
}

hipError_t launch_pol_combine_synth(const crsht_plan* P, int nrhs, void* eo, bool f32, hipStream_t s, int npairs) {
  const Geometry& g = P->g;
  const int np = npairs < 0 ? g.npairs : npairs;
  const int64_t n = (int64_t)np * (g.mmax + 1);
  const int64_t cs = n * 2;
  if (n == 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_pol_combine_synth<float2>, dim3(nblk(n)), dim3(kVecT), 0, s, np, g.mmax, nrhs,
                       P->t.pair_z, (float2*)eo, cs, P->pred);
  else
    hipLaunchKernelGGL(k_pol_combine_synth<double2>, dim3(nblk(n)), dim3(kVecT), 0, s, np, g.mmax, nrhs,
                       P->t.pair_z, (double2*)eo, cs, P->pred);
  return hipGetLastError();
}

hipError_t launch_pol_pre_adjoint(const crsht_plan* P, int nrhs, void* geo, bool f32, hipStream_t s, int npairs) {
  const Geometry& g = P->g;
  const int np = npairs < 0 ? g.npairs : npairs;
  const int64_t n = (int64_t)np * (g.mmax + 1);
  const int64_t cs = n * 2;
  if (n == 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_pol_pre_adjoint<float2>, dim3(nblk(n)), dim3(kVecT), 0, s, np, g.mmax, nrhs,
                       P->t.pair_z, (float2*)geo, cs, P->pred);
  else
    hipLaunchKernelGGL(k_pol_pre_adjoint<double2>, dim3(nblk(n)), dim3(kVecT), 0, s, np, g.mmax, nrhs,
                       P->t.pair_z, (double2*)geo, cs, P->pred);
  return hipGetLastError();
}

hipError_t launch_pol_combine_adjoint(const crsht_plan* P, int nrhs, const double2* raw, const double* f,
                                      double2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pol_combine_adjoint, dim3(nblk(P->g.nalm)), dim3(kVecT), 0, s, P->g.nalm, nrhs, P->t.idx_l,
                     P->t.idx_m, P->t.rec_kappa, f, raw, out, P->pred);
  return hipGetLastError();
}

hipError_t launch_expand_tqu(const crsht_plan* P, const double* perl, hipStream_t s) {
  hipLaunchKernelGGL(k_expand_tqu, dim3(nblk(P->g.nalm)), dim3(kVecT), 0, s, P->g.nalm, P->g.lmax, P->t.idx_l,
                     P->t.rec_kappa, P->w.sblk, perl, P->w.sinv, P->w.sinvhalf, P->w.bk, P->w.bl_keep);
  return hipGetLastError();
}

hipError_t launch_alm_wquad_tqu(const crsht_plan* P, const double2* a, double* partial, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_alm_wquad_tqu, dim3(nb), dim3(kVecT), 0, s, P->g.nalm, P->t.idx_l, P->t.idx_m, P->w.sblk, a,
                     partial);
  return hipGetLastError();
}

hipError_t launch_cg_q_tqu(const crsht_plan* P, int nrhs, const double2* p, const double2* dterm, double2* q,
                           hipStream_t s, bool prior) {
  const int nb = vec_reduce_blocks(P);
  hipLaunchKernelGGL(k_cg_q_tqu, dim3(nb, nrhs), dim3(kVecT), 0, s, P->g.nalm, P->t.idx_l, P->t.idx_m,
                     prior ? P->w.sblk : nullptr, P->w.camp, p, dterm, q, P->w.partial, P->w.npart, P->pred);
  return hipGetLastError();
}

hipError_t launch_rhs_finish_tqu(const crsht_plan* P, int nrhs, const double2* dterm, const double2* w0,
                                 double2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_rhs_finish_tqu, dim3(nblk(P->g.nalm)), dim3(kVecT), 0, s, P->g.nalm, nrhs, P->t.idx_l,
                     P->t.idx_m, P->w.sblk, P->w.camp, dterm, w0, out);
  return hipGetLastError();
}

hipError_t launch_diag_tqu(const crsht_plan* P, const double2* rawt, const double2* rawp, double* diag,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_diag_tqu, dim3(nblk(P->g.nalm)), dim3(kVecT), 0, s, P->g.nalm, P->t.idx_l, P->w.sblk,
                     P->w.bk, P->w.sinv, rawt, rawp, diag);
  return hipGetLastError();
}


hipError_t launch_polar_spectra_to_f32(const crsht_plan* P, int nrhs, const double2* pol64, float2* eo,
                                       hipStream_t s) {
  const Geometry& g = P->g;
  const int npol = P->npol;
  const int64_t n = (int64_t)npol * (g.mmax + 1) * 2;
  const int64_t col64 = n, col32 = (int64_t)g.npairs * (g.mmax + 1) * 2;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_polar_spectra_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, npol, g.mmax, nrhs,
                     pol64, col64, eo, col32, P->pred);
  return hipGetLastError();
}

hipError_t launch_polar_geo_to_f64(const crsht_plan* P, int nrhs, float2* geo, double2* pol64, hipStream_t s) {
  const Geometry& g = P->g;
  const int npol = P->npol;
  const int64_t n = (int64_t)npol * (g.mmax + 1) * 2;
  const int64_t col64 = n, col32 = (int64_t)g.npairs * (g.mmax + 1) * 2;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_polar_geo_to_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, npol, g.mmax, nrhs, geo,
                     col32, pol64, col64, P->pred);
  return hipGetLastError();
}
}  // namespace crsht
