// Elementwise and reduction kernels on a_lm vectors and maps: problem set-up,
// right-hand-side assembly, the vector part of preconditioned conjugate
// gradients (Shewchuk 1994, PCG with a diagonal preconditioner), and FP64
// reductions in a fixed order (block partial sums, then one block summing the
// partials), so results are run-to-run reproducible.
#include "internal.h"
#include "devutil.h"

namespace crsht {
namespace {

constexpr int kVecBlock = 256;


// per-index problem arrays from per-l arrays:
// sinv = keep/C_l, sinvhalf = keep/sqrt(C_l), bk = keep b_l kappa_lm
__global__ void k_expand(int64_t nalm, const int* __restrict__ idx_l, const double* __restrict__ kappa,
                         const double* __restrict__ perl, int lmax, double* __restrict__ sinv,
                         double* __restrict__ sinvhalf, double* __restrict__ bk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const int l = idx_l[i];
  const double keep = perl[3 * (lmax + 1) + l];
  sinv[i] = perl[l];
  sinvhalf[i] = perl[(lmax + 1) + l];
  bk[i] = keep * perl[2 * (lmax + 1) + l] * kappa[i];
}

// out = f * in per column (in and out may be the same array)
__global__ void k_scale(int64_t nalm, int nrhs, const double2* in, const double* __restrict__ f, double2* out,
                        const int* __restrict__ pred) {
  if (pred && *pred) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const double s = f[i];
  for (int c = 0; c < nrhs; ++c) {
    const double2 v = in[c * nalm + i];
    out[c * nalm + i] = make_double2(s * v.x, s * v.y);
  }
}

// out = fac_l[l] * in per coefficient (one column)
__global__ void k_scale_l(int64_t nalm, const int* __restrict__ idx_l, const double* __restrict__ fac_l,
                          const double2* __restrict__ in, double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const double f = fac_l[idx_l[i]];
  const double2 v = in[i];
  out[i] = make_double2(f * v.x, f * v.y);
}

__global__ void k_ring_weights(int npairs, const int* __restrict__ nphi, const int64_t* __restrict__ fn,
                               const int64_t* __restrict__ fs, const double* __restrict__ ninv,
                               const double* __restrict__ ninv2, double scale, double* __restrict__ w) {
  __shared__ double sh[kVecBlock];
  const int p = blockIdx.x;
  const int n = nphi[p];
  const bool eq = fn[p] == fs[p];
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    acc += ninv[fn[p] + j];
    if (!eq) acc += ninv[fs[p] + j];
    if (ninv2) {
      acc += ninv2[fn[p] + j];
      if (!eq) acc += ninv2[fs[p] + j];
    }
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) w[p] = scale * acc;
}

// u = ninv * d + sqrt(ninv) * w1 (either may be absent); maps [nrhs][ncomp][npix],
// ninv [ncomp][npix]
__global__ void k_pix_rhs(int64_t npix, int nrhs, int ncomp, const double* __restrict__ ninv,
                          const double* __restrict__ d, const double* __restrict__ w1, double* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix) return;
  for (int k = 0; k < ncomp; ++k) {
    const double n = ninv[k * npix + i];
    const double sn = sqrt(n);
    for (int c = 0; c < nrhs; ++c) {
      const int64_t j = ((int64_t)c * ncomp + k) * npix + i;
      double v = 0.0;
      if (d) v = n * d[j];
      if (w1) v = fma(sn, w1[j], v);
      u[j] = v;
    }
  }
}

// out = bk * raw + sinvhalf * w0 (either may be absent; the S^-1/2 term of
// column c scaled by camp[c].y), raw = the unscaled adjoint Legendre sums of
// N^-1 d + N^-1/2 w1; Im of m = 0 forced to 0
__global__ void k_rhs_finish(int64_t nalm, int nrhs, const int* __restrict__ idx_m, const double* __restrict__ bk,
                             const double* __restrict__ sinvhalf, const double2* __restrict__ camp,
                             const double2* __restrict__ raw, const double2* __restrict__ w0,
                             double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const double sh = sinvhalf[i], b = bk[i];
  const bool m0 = idx_m[i] == 0;
  for (int c = 0; c < nrhs; ++c) {
    double2 v = raw ? raw[c * nalm + i] : make_double2(0.0, 0.0);
    v.x *= b;
    v.y *= b;
    if (w0) {
      const double2 w = w0[c * nalm + i];
      const double shc = sh * camp[c].y;
      v.x = fma(shc, w.x, v.x);
      v.y = fma(shc, w.y, v.y);
    }
    if (m0) v.y = 0.0;
    out[c * nalm + i] = v;
  }
}

// out = x on kept modes (sinv > 0), 0 elsewhere, Im of m = 0 set to 0
__global__ void k_project(int64_t nalm, int nrhs, const int* __restrict__ idx_m, const double* __restrict__ sinv,
                          const double2* __restrict__ x, double2* __restrict__ out, const int* __restrict__ pred) {
  if (pred && *pred) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const bool keep = sinv[i] > 0.0;
  const bool m0 = idx_m[i] == 0;
  for (int c = 0; c < nrhs; ++c) {
    double2 v = keep ? x[c * nalm + i] : make_double2(0.0, 0.0);
    if (m0) v.y = 0.0;
    out[c * nalm + i] = v;
  }
}

// map = a - b (for analysis corrections), and map *= s
__global__ void k_map_axpby(int64_t n, double a, const double* __restrict__ x, double b,
                            const double* __restrict__ y, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

__global__ void k_alm_axpby(int64_t n, double a, const double2* __restrict__ x, double b,
                            const double2* __restrict__ y, double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 u = x[i];
  double2 v = make_double2(a * u.x, a * u.y);
  if (y) {
    const double2 w = y[i];
    v.x = fma(b, w.x, v.x);
    v.y = fma(b, w.y, v.y);
  }
  out[i] = v;
}

// ---------------------------------------------------------------- PCG pieces
// weighted dot partials of one column: w_m (a.x c.x + a.y c.y)

// start: x = 0 (or given), r = b - A x0 computed by caller in r, z = r / D,
// p = z, pt = bk * p; partial sums of <r,z>, <r,r>, <b,b>. Z: the stored
// type of z (float2 only with zgiven)
template <typename Z>
__global__ void k_cg_start(int64_t nalm, const int* __restrict__ idx_m, const double* __restrict__ diag,
                           const double* __restrict__ bk, const double2* __restrict__ b,
                           const double2* __restrict__ r, Z* __restrict__ z, double2* __restrict__ p,
                           double2* __restrict__ pt, double* __restrict__ partial, int npart,
                           const double* __restrict__ scal, int zgiven, const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ double sh[kVecBlock];
  const int c = blockIdx.y;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x) {
      const int64_t ci = c * nalm + i;
      const int m = idx_m[i];
      const double2 rv = r[ci];
      double2 zv;
      if (zgiven) {
        zv = zload(z + ci);
      } else {
        const double dinv = 1.0 / diag[i];
        zv = zstore(z + ci, make_double2(rv.x * dinv, rv.y * dinv));
      }
      p[ci] = zv;
      pt[ci] = make_double2(bk[i] * zv.x, bk[i] * zv.y);
      rz += wdot(m, rv, zv);
      rr += wdot(m, rv, rv);
      bb += wdot(m, b[ci], b[ci]);
    }
  }
  rz = block_sum(rz, sh);
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    double* pa = partial + (size_t)c * npart * 4;
    pa[blockIdx.x] = rz;
    pa[npart + blockIdx.x] = rr;
    pa[2 * npart + blockIdx.x] = bb;
  }
}

// sums partial[c][slot-row][0..nb) into scal; what = 0: start, 1: alpha, 2: beta,
// 3: residual replacement
// (kScalBlock threads: the per-task and per-tile partials of the block
// preconditioner and the fused adjoint number several thousand per column)
constexpr int kScalBlock = 1024;
__global__ __launch_bounds__(kScalBlock) void k_cg_scalars(int what, int nb, const double* __restrict__ partial,
                                                           int npart, double* __restrict__ scal, double tol,
                                                           int restart, const double* __restrict__ part0, int n0,
                                                           const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ double sh[kScalBlock];
  const int c = blockIdx.x;
  const double* pa = partial + (size_t)c * npart * 4;
  double* sc = scal + c * kScalSlots;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    if (!part0) s0 += pa[i];
    if (what != 1) {
      s1 += pa[npart + i];
      s2 += pa[2 * npart + i];
    }
  }
  if (part0)
    for (int i = threadIdx.x; i < n0; i += blockDim.x) s0 += part0[(size_t)c * n0 + i];
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x != 0) return;
  if (what == 0) {  // after k_cg_start: fresh start, or restart of the columns not done
    if (restart && sc[S_DONE] != 0.0) return;
    sc[S_RZ] = s0;
    sc[S_RR] = s1;
    if (!restart) {
      sc[S_BB] = s2;
      sc[S_ITERS] = 0.0;
      sc[S_BREAK] = 0.0;
      sc[S_XA] = 0.0;
    }
    const double bb = sc[S_BB];
    sc[S_REL] = bb > 0.0 ? sqrt(s1 / bb) : 0.0;
    sc[S_DONE] = (bb == 0.0) ? 1.0 : 0.0;
  } else if (what == 1) {  // alpha = <r,z>/<p,Ap>
    if (sc[S_DONE] != 0.0) return;
    sc[S_PQ] = s0;
    if (!(s0 > 0.0) || !isfinite(s0) || !isfinite(sc[S_RZ])) {
      sc[S_BREAK] = 1.0;
      sc[S_DONE] = 1.0;
      sc[S_ALPHA] = 0.0;
    } else {
      sc[S_ALPHA] = sc[S_RZ] / s0;
    }
  } else if (what == 3) {  // residual replaced after the update: beta from the new <r,z>
    if (sc[S_DONE] != 0.0) return;
    sc[S_BETA] = sc[S_RESTART] != 0.0 ? 0.0 : s0 / sc[S_RZ_PREV];
    sc[S_RZ] = s0;
    sc[S_RR] = s1;
    sc[S_REL] = sc[S_BB] > 0.0 ? sqrt(s1 / sc[S_BB]) : 0.0;
  } else {  // beta after the update
    if (sc[S_DONE] != 0.0) return;
    const double rznew = s0, rr = s1;
    sc[S_ITERS] += 1.0;
    sc[S_RZ_PREV] = sc[S_RZ];
    sc[S_BETA] = rznew / sc[S_RZ];
    sc[S_RZ] = rznew;
    sc[S_RR] = rr;
    sc[S_REL] = sqrt(rr / sc[S_BB]);
    if (!isfinite(rr)) {
      sc[S_BREAK] = 1.0;
      sc[S_DONE] = 1.0;
    } else if (sc[S_REL] <= tol) {
      sc[S_DONE] = 1.0;
    }
  }
}

// x += alpha p; r -= alpha q; z = r / D; partial <r,z>, <r,r>. Q: the
// vector type of q (float2 in the mixed-precision T iteration)
// With defer (FP32 q of the mixed T iteration) x and p are not touched: the
// column's alpha (0 if it is done) is left in scal[S_XA] for the next
// direction update, which reads that p anyway.
template <typename Q>
__global__ void k_cg_update(int64_t nalm, const int* __restrict__ idx_m, const double* __restrict__ diag,
                            const double* __restrict__ bk, double2* __restrict__ x, double2* __restrict__ r,
                            double2* __restrict__ z, const double2* __restrict__ p, const Q* __restrict__ q,
                            double* __restrict__ partial, int npart, double* __restrict__ scal, int noz, int defer,
                            const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ double sh[kVecBlock];
  const int c = blockIdx.y;
  double* sc = scal + c * kScalSlots;
  const bool skip = sc[S_DONE] != 0.0;
  const double a = sc[S_ALPHA];
  if (defer && blockIdx.x == 0 && threadIdx.x == 0) sc[S_XA] = skip ? 0.0 : a;
  double rz = 0.0, rr = 0.0;
  if (!skip) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x) {
      const int64_t ci = c * nalm + i;
      const int m = idx_m[i];
      const Q qq = q[ci];
      const double2 qv = make_double2((double)qq.x, (double)qq.y);
      double2 rv = r[ci];
      if (!defer) {
        const double2 pv = p[ci];
        double2 xv = x[ci];
        xv.x = fma(a, pv.x, xv.x);
        xv.y = fma(a, pv.y, xv.y);
        x[ci] = xv;
      }
      rv.x = fma(-a, qv.x, rv.x);
      rv.y = fma(-a, qv.y, rv.y);
      r[ci] = rv;
      if (!noz) {
        const double dinv = 1.0 / diag[i];
        const double2 zv = make_double2(rv.x * dinv, rv.y * dinv);
        z[ci] = zv;
        rz += wdot(m, rv, zv);
      }
      rr += wdot(m, rv, rv);
    }
  }
  rz = block_sum(rz, sh);
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    double* pa = partial + (size_t)c * npart * 4;
    pa[blockIdx.x] = rz;
    pa[npart + blockIdx.x] = rr;
  }
}

// residual replacement: z = r / D; partial <r,z>, <r,r> (p untouched)
__global__ void k_cg_replace(int64_t nalm, const int* __restrict__ idx_m, const double* __restrict__ diag,
                             const double2* __restrict__ r, double2* __restrict__ z, double* __restrict__ partial,
                             int npart, const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ double sh[kVecBlock];
  const int c = blockIdx.y;
  double rz = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ci = c * nalm + i;
    const int m = idx_m[i];
    const double2 rv = r[ci];
    const double dinv = 1.0 / diag[i];
    const double2 zv = make_double2(rv.x * dinv, rv.y * dinv);
    z[ci] = zv;
    rz += wdot(m, rv, zv);
    rr += wdot(m, rv, rv);
  }
  rz = block_sum(rz, sh);
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    double* pa = partial + (size_t)c * npart * 4;
    pa[blockIdx.x] = rz;
    pa[npart + blockIdx.x] = rr;
  }
}

// p = z + beta p; pt = bk p
__global__ void k_cg_pupdate(int64_t nalm, const double* __restrict__ bk, const double2* __restrict__ z,
                             double2* __restrict__ p, double2* __restrict__ pt, const double* __restrict__ scal,
                             const int* __restrict__ pred) {
  if (pred && *pred) return;
  const int c = blockIdx.y;
  const double* sc = scal + c * kScalSlots;
  if (sc[S_DONE] != 0.0) return;
  const double beta = sc[S_BETA];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ci = c * nalm + i;
    const double2 zv = z[ci];
    double2 pv = p[ci];
    pv.x = fma(beta, pv.x, zv.x);
    pv.y = fma(beta, pv.y, zv.y);
    p[ci] = pv;
    pt[ci] = make_double2(bk[i] * pv.x, bk[i] * pv.y);
  }
}

// q = camp[c].x sinv * p + bk * raw for column c; partial <p, q>
__global__ void k_cg_q(int64_t nalm, const int* __restrict__ idx_m, const double* __restrict__ sinv,
                       const double2* __restrict__ camp, const double* __restrict__ bk,
                       const double2* __restrict__ p, const double2* __restrict__ raw, double2* __restrict__ q,
                       double* __restrict__ partial, int npart, const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ double sh[kVecBlock];
  const int c = blockIdx.y;
  const double qa = camp[c].x;
  double pq = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ci = c * nalm + i;
    const double si = sinv ? qa * sinv[i] : 0.0, b = bk[i];
    const double2 pv = p[ci], rv = raw[ci];
    const double2 qv = make_double2(fma(si, pv.x, b * rv.x), fma(si, pv.y, b * rv.y));
    q[ci] = qv;
    pq += wdot(idx_m[i], pv, qv);
  }
  pq = block_sum(pq, sh);
  if (threadIdx.x == 0) partial[(size_t)c * npart * 4 + blockIdx.x] = pq;
}

__global__ void k_diag(int64_t nalm, const double* __restrict__ sinv, const double* __restrict__ bk,
                       const double2* __restrict__ raw, double* __restrict__ diag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const double si = sinv[i], b = bk[i];
  diag[i] = si > 0.0 ? fma(b * b, raw[i].x, si) : 1.0;
}

// r = b - Ax; partial <r,r> into row 1 (row 0: <r,r> as well)
__global__ void k_residual(int64_t nalm, const int* __restrict__ idx_m, const double2* __restrict__ b,
                           const double2* __restrict__ ax, double2* __restrict__ r, double* __restrict__ partial,
                           int npart, const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ double sh[kVecBlock];
  const int c = blockIdx.y;
  double rr = 0.0, bb = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ci = c * nalm + i;
    const int m = idx_m[i];
    const double2 bv = b[ci], av = ax[ci];
    const double2 rv = make_double2(bv.x - av.x, bv.y - av.y);
    r[ci] = rv;
    rr += wdot(m, rv, rv);
    bb += wdot(m, bv, bv);
  }
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    double* pa = partial + (size_t)c * npart * 4;
    pa[blockIdx.x] = rr;
    pa[npart + blockIdx.x] = bb;
    pa[2 * npart + blockIdx.x] = 0.0;
  }
}

// sum rows 0, 1, 2 of the partials of column c into scal[c][AUX0..AUX2]
__global__ void k_sum_rows(int nb, const double* __restrict__ partial, int npart, double* __restrict__ scal,
                           const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ double sh[kVecBlock];
  const int c = blockIdx.x;
  const double* pa = partial + (size_t)c * npart * 4;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    s0 += pa[i];
    s1 += pa[npart + i];
    s2 += pa[2 * npart + i];
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    scal[c * kScalSlots + S_AUX0] = s0;
    scal[c * kScalSlots + S_AUX1] = s1;
    scal[c * kScalSlots + S_AUX2] = s2;
  }
}

// sum_p ninv (a - b)^2 style pixel reductions: partial of sum w x^2 (w may be null -> 1)
__global__ void k_pix_wsq(int64_t npix, const double* __restrict__ w, const double* __restrict__ x,
                          const double* __restrict__ y, double* __restrict__ partial) {
  __shared__ double sh[kVecBlock];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = y ? x[i] - y[i] : x[i];
    acc = fma(w ? w[i] * v : v, v, acc);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// partial of w_m a^T (f a) (f per index)
__global__ void k_alm_wquad(int64_t nalm, const int* __restrict__ idx_m, const double* __restrict__ f,
                            const double2* __restrict__ a, double* __restrict__ partial) {
  __shared__ double sh[kVecBlock];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = a[i];
    acc += f[i] * wdot(idx_m[i], v, v);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

int nblocks(int64_t n) {
  int64_t b = (n + kVecBlock - 1) / kVecBlock;
  return (int)(b < 1 ? 1 : b);
}

// u = N^-1 (d - m) per column (data residual weighted by the inverse noise);
// maps [nrhs][ncomp][npix], ninv [ncomp][npix]
__global__ void k_pix_wres(int64_t npix, int nrhs, int ncomp, const double* __restrict__ ninv,
                           const double* __restrict__ d, const double* m, double* u) {   // u may alias m
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix) return;
  for (int k = 0; k < ncomp; ++k) {
    const double n = ninv[k * npix + i];
    for (int c = 0; c < nrhs; ++c) {
      const int64_t j = ((int64_t)c * ncomp + k) * npix + i;
      u[j] = n * (d[j] - m[j]);
    }
  }
}

// real-field weights of the synthesis gradient: x 2 for m > 0, Im of m = 0 set to 0
__global__ void k_mweight(int64_t nalm, int nrhs, const int* __restrict__ idx_m, double2* a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nalm) return;
  const bool m0 = idx_m[i] == 0;
  for (int c = 0; c < nrhs; ++c) {
    double2 v = a[c * nalm + i];
    if (m0) v.y = 0.0;
    else v = make_double2(2.0 * v.x, 2.0 * v.y);
    a[c * nalm + i] = v;
  }
}

// Per multipole bin k = blockIdx.x (l in [edges[k], edges[k+1])), slice
// blockIdx.y of the m values: partial sums of
//   t1 = <a^, S^-1_k a^>,  t2 = <lambda, S^-1/2_k w0>,  t3 = <lambda, S^-1_k f^>
// in the real-field inner product. The elements of (l, m) for one m are
// contiguous in l, so each m contributes a coalesced run.
__global__ void k_bin_terms(int mmax, const int64_t* __restrict__ mstart, const int* __restrict__ edges,
                            const double* __restrict__ sinv, const double* __restrict__ sinvhalf,
                            const double2* __restrict__ ahat, const double2* __restrict__ fhat,
                            const double2* __restrict__ lam, const double2* __restrict__ w0,
                            double* __restrict__ partial, int mode) {
  __shared__ double sh[kVecBlock];
  const int k = blockIdx.x, sl = blockIdx.y, S = gridDim.y;
  const int l0 = edges[k], l1 = edges[k + 1];
  double t1 = 0.0, t2 = 0.0, t3 = 0.0;
  const int mtop = min(mmax, l1 - 1);
  for (int m = sl; m <= mtop; m += S) {
    const int lo = max(l0, m);
    const int64_t base = mstart[m] - m;
    for (int l = lo + threadIdx.x; l < l1; l += blockDim.x) {
      const int64_t i = base + l;
      const double2 a = ahat[i], f = fhat[i], L = lam[i];
      const double si = sinv[i];
      t1 += si * wdot(m, a, a);
      t3 += (mode == 1 ? 1.0 : si) * wdot(m, L, f);
      if (w0) t2 += sinvhalf[i] * wdot(m, L, w0[i]);
    }
  }
  t1 = block_sum(t1, sh);
  t2 = block_sum(t2, sh);
  t3 = block_sum(t3, sh);
  if (threadIdx.x == 0) {
    double* o = partial + ((size_t)k * S + sl) * 3;
    o[0] = t1;
    o[1] = t2;
    o[2] = t3;
  }
}

// per-bin real-field dots of vectors of ncomp blocks of nalm coefficients
// (T+Q+U gradient): t1 = <x1, y1>_k, t2 = <x2, y2>_k (x2 or y2 null: 0),
// t3 = <x3, y3>_k over the coefficients of bin k of every block
__global__ void k_bin_dots3(int mmax, int64_t nalm, int ncomp, const int64_t* __restrict__ mstart,
                            const int* __restrict__ edges, const double2* __restrict__ x1,
                            const double2* __restrict__ y1, const double2* __restrict__ x2,
                            const double2* __restrict__ y2, const double2* __restrict__ x3,
                            const double2* __restrict__ y3, double* __restrict__ partial) {
  __shared__ double sh[kVecBlock];
  const int k = blockIdx.x, sl = blockIdx.y, S = gridDim.y;
  const int l0 = edges[k], l1 = edges[k + 1];
  double t1 = 0.0, t2 = 0.0, t3 = 0.0;
  const int mtop = min(mmax, l1 - 1);
  for (int m = sl; m <= mtop; m += S) {
    const int lo = max(l0, m);
    for (int c = 0; c < ncomp; ++c) {
      const int64_t base = c * nalm + mstart[m] - m;
      for (int l = lo + threadIdx.x; l < l1; l += blockDim.x) {
        const int64_t i = base + l;
        t1 += wdot(m, x1[i], y1[i]);
        if (x2 && y2) t2 += wdot(m, x2[i], y2[i]);
        t3 += wdot(m, x3[i], y3[i]);
      }
    }
  }
  t1 = block_sum(t1, sh);
  t2 = block_sum(t2, sh);
  t3 = block_sum(t3, sh);
  if (threadIdx.x == 0) {
    double* o = partial + ((size_t)k * S + sl) * 3;
    o[0] = t1;
    o[1] = t2;
    o[2] = t3;
  }
}

// d ln pi / d theta_k = t1/2 + t2/2 - t3 (mode 0: fixed w0, w1) or t1/2 - t3/2
// (mode 1: fixed whitened fluctuation, lam = M f); mode 2: t1 alone (the
// bin's a^T S^-1 a); slices summed in a fixed order
__global__ void k_bin_grad(int nbins, int S, const double* __restrict__ partial, double* __restrict__ grad,
                           int mode) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nbins) return;
  double t1 = 0.0, t2 = 0.0, t3 = 0.0;
  for (int sl = 0; sl < S; ++sl) {
    const double* o = partial + ((size_t)k * S + sl) * 3;
    t1 += o[0];
    t2 += o[1];
    t3 += o[2];
  }
  grad[k] = mode == 2 ? t1 : mode == 1 ? 0.5 * t1 - 0.5 * t3 : 0.5 * t1 + 0.5 * t2 - t3;
}

}  // namespace

int vec_reduce_blocks(const crsht_plan* P) {
  int64_t b = (vlen(P) + kVecBlock - 1) / kVecBlock;
  int cap = P->w.npart;
  if (cap > 1024) cap = 1024;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

hipError_t launch_expand(const crsht_plan* P, const double* perl, hipStream_t s) {
  hipLaunchKernelGGL(k_expand, dim3(nblocks(P->g.nalm)), dim3(kVecBlock), 0, s, P->g.nalm, P->t.idx_l,
                     P->t.rec_kappa, perl, P->g.lmax, P->w.sinv, P->w.sinvhalf, P->w.bk);
  return hipGetLastError();
}

hipError_t launch_scale_alm(const crsht_plan* P, int nrhs, const double2* in, const double* f, double2* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(nblocks(P->g.nalm)), dim3(kVecBlock), 0, s, P->g.nalm, nrhs, in, f, out, P->pred);
  return hipGetLastError();
}

hipError_t launch_ring_weights(const crsht_plan* P, const double* ninv, double* w, hipStream_t s,
                               const double* ninv2, double scale) {
  hipLaunchKernelGGL(k_ring_weights, dim3(P->g.npairs), dim3(kVecBlock), 0, s, P->g.npairs, P->t.pair_nphi,
                     P->t.pair_first_n, P->t.pair_first_s, ninv, ninv2, scale, w);
  return hipGetLastError();
}

hipError_t launch_pix_rhs(const crsht_plan* P, int nrhs, const double* ninv, const double* d, const double* w1,
                          double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_pix_rhs, dim3(nblocks(P->g.npix)), dim3(kVecBlock), 0, s, P->g.npix, nrhs, P->ncomp, ninv, d,
                     w1, u);
  return hipGetLastError();
}

hipError_t launch_rhs_finish(const crsht_plan* P, int nrhs, const double2* raw, const double2* w0, double2* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_rhs_finish, dim3(nblocks(P->g.nalm)), dim3(kVecBlock), 0, s, P->g.nalm, nrhs, P->t.idx_m,
                     P->w.bk, P->w.sinvhalf, P->w.camp, raw, w0, out);
  return hipGetLastError();
}

hipError_t launch_project(const crsht_plan* P, int nrhs, const double2* x, double2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_project, dim3(nblocks(vlen(P))), dim3(kVecBlock), 0, s, vlen(P), nrhs, P->t.idx_mv,
                     P->w.sinv, x, out, P->pred);
  return hipGetLastError();
}

hipError_t launch_map_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_map_axpby, dim3(nblocks(n)), dim3(kVecBlock), 0, s, n, a, x, b, y, out);
  return hipGetLastError();
}

hipError_t launch_alm_axpby(int64_t n, double a, const double2* x, double b, const double2* y, double2* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_alm_axpby, dim3(nblocks(n)), dim3(kVecBlock), 0, s, n, a, x, b, y, out);
  return hipGetLastError();
}

hipError_t launch_cg_start(const crsht_plan* P, int nrhs, const double2* b, const double2* r, double2* z,
                           double2* p, double2* pt, hipStream_t s, bool zgiven, bool z32) {
  const int nb = vec_reduce_blocks(P);
  if (z32 && zgiven)
    hipLaunchKernelGGL(k_cg_start<float2>, dim3(nb, nrhs), dim3(kVecBlock), 0, s, vlen(P), P->t.idx_mv, P->w.diag,
                       P->w.bk, b, r, reinterpret_cast<float2*>(z), p, pt, P->w.partial, P->w.npart, P->w.scal, 1,
                       P->pred);
  else
    hipLaunchKernelGGL(k_cg_start<double2>, dim3(nb, nrhs), dim3(kVecBlock), 0, s, vlen(P), P->t.idx_mv, P->w.diag,
                       P->w.bk, b, r, z, p, pt, P->w.partial, P->w.npart, P->w.scal, zgiven ? 1 : 0, P->pred);
  return hipGetLastError();
}

hipError_t launch_cg_scalars(const crsht_plan* P, int nrhs, int what, int nb, double tol, int restart,
                             hipStream_t s, const double* part0, int n0) {
  hipLaunchKernelGGL(k_cg_scalars, dim3(nrhs), dim3(kScalBlock), 0, s, what, nb, P->w.partial, P->w.npart,
                     P->w.scal, tol, restart, part0, n0, P->pred);
  return hipGetLastError();
}

hipError_t launch_cg_q(const crsht_plan* P, int nrhs, const double2* p, const double2* raw, double2* q,
                       hipStream_t s, bool prior) {
  const int nb = vec_reduce_blocks(P);
  hipLaunchKernelGGL(k_cg_q, dim3(nb, nrhs), dim3(kVecBlock), 0, s, P->g.nalm, P->t.idx_m,
                     prior ? P->w.sinv : nullptr, P->w.camp, P->w.bk, p, raw, q, P->w.partial, P->w.npart, P->pred);
  return hipGetLastError();
}

hipError_t launch_diag(const crsht_plan* P, const double2* raw, double* diag, hipStream_t s) {
  hipLaunchKernelGGL(k_diag, dim3(nblocks(P->g.nalm)), dim3(kVecBlock), 0, s, P->g.nalm, P->w.sinv, P->w.bk, raw,
                     diag);
  return hipGetLastError();
}

hipError_t launch_cg_update(const crsht_plan* P, int nrhs, double2* x, double2* r, double2* z, const double2* p,
                            const double2* q, hipStream_t s, bool noz, const float2* q32) {
  const int nb = vec_reduce_blocks(P);
  if (q32)
    hipLaunchKernelGGL(k_cg_update<float2>, dim3(nb, nrhs), dim3(kVecBlock), 0, s, vlen(P), P->t.idx_mv, P->w.diag,
                       P->w.bk, x, r, z, p, q32, P->w.partial, P->w.npart, P->w.scal, noz ? 1 : 0, 1, P->pred);
  else
    hipLaunchKernelGGL(k_cg_update<double2>, dim3(nb, nrhs), dim3(kVecBlock), 0, s, vlen(P), P->t.idx_mv, P->w.diag,
                       P->w.bk, x, r, z, p, q, P->w.partial, P->w.npart, P->w.scal, noz ? 1 : 0, 0, P->pred);
  return hipGetLastError();
}

// x += scal[S_XA] p per column
__global__ void k_x_flush(int64_t nalm, double2* __restrict__ x, const double2* __restrict__ p,
                          const double* __restrict__ scal, const int* __restrict__ pred) {
  if (pred && *pred) return;
  const int c = blockIdx.y;
  const double a = scal[c * kScalSlots + S_XA];
  if (a == 0.0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ci = c * nalm + i;
    const double2 pv = p[ci];
    double2 xv = x[ci];
    xv.x = fma(a, pv.x, xv.x);
    xv.y = fma(a, pv.y, xv.y);
    x[ci] = xv;
  }
}

__global__ void k_xa_clear(int nrhs, double* __restrict__ scal, const int* __restrict__ pred) {
  if (pred && *pred) return;
  for (int c = threadIdx.x; c < nrhs; c += blockDim.x) scal[c * kScalSlots + S_XA] = 0.0;
}

hipError_t launch_x_flush(const crsht_plan* P, int nrhs, hipStream_t s) {
  const int nb = vec_reduce_blocks(P);
  hipLaunchKernelGGL(k_x_flush, dim3(nb, nrhs), dim3(kVecBlock), 0, s, vlen(P), P->w.cg_x, P->w.cg_p, P->w.scal,
                     P->pred);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_xa_clear, dim3(1), dim3(1024), 0, s, nrhs, P->w.scal, P->pred);
  return hipGetLastError();
}

hipError_t launch_cg_replace(const crsht_plan* P, int nrhs, const double2* r, double2* z, hipStream_t s) {
  const int nb = vec_reduce_blocks(P);
  hipLaunchKernelGGL(k_cg_replace, dim3(nb, nrhs), dim3(kVecBlock), 0, s, vlen(P), P->t.idx_mv, P->w.diag, r, z,
                     P->w.partial, P->w.npart, P->pred);
  return hipGetLastError();
}

hipError_t launch_cg_pupdate(const crsht_plan* P, int nrhs, const double2* z, double2* p, double2* pt,
                             hipStream_t s) {
  const int nb = vec_reduce_blocks(P);
  hipLaunchKernelGGL(k_cg_pupdate, dim3(nb, nrhs), dim3(kVecBlock), 0, s, vlen(P), P->w.bk, z, p, pt,
                     P->w.scal, P->pred);
  return hipGetLastError();
}

hipError_t launch_residual(const crsht_plan* P, int nrhs, const double2* b, const double2* ax, double2* r,
                           hipStream_t s) {
  const int nb = vec_reduce_blocks(P);
  hipLaunchKernelGGL(k_residual, dim3(nb, nrhs), dim3(kVecBlock), 0, s, vlen(P), P->t.idx_mv, b, ax, r,
                     P->w.partial, P->w.npart, P->pred);
  return hipGetLastError();
}

hipError_t launch_sum_rows(const crsht_plan* P, int nrhs, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_rows, dim3(nrhs), dim3(kVecBlock), 0, s, nb, P->w.partial, P->w.npart, P->w.scal, P->pred);
  return hipGetLastError();
}

hipError_t launch_pix_wsq(const crsht_plan* P, const double* w, const double* x, const double* y, double* partial,
                          int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_pix_wsq, dim3(nb), dim3(kVecBlock), 0, s, P->g.npix, w, x, y, partial);
  return hipGetLastError();
}

hipError_t launch_alm_wquad(const crsht_plan* P, const double* f, const double2* a, double* partial, int nb,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_alm_wquad, dim3(nb), dim3(kVecBlock), 0, s, P->g.nalm, P->t.idx_m, f, a, partial);
  return hipGetLastError();
}

hipError_t launch_pix_wres(const crsht_plan* P, int nrhs, const double* ninv, const double* d, const double* m,
                           double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_pix_wres, dim3(nblocks(P->g.npix)), dim3(kVecBlock), 0, s, P->g.npix, nrhs, P->ncomp, ninv,
                     d, m, u);
  return hipGetLastError();
}

hipError_t launch_mweight(const crsht_plan* P, int nrhs, double2* a, hipStream_t s) {
  hipLaunchKernelGGL(k_mweight, dim3(nblocks(vlen(P))), dim3(kVecBlock), 0, s, vlen(P), nrhs, P->t.idx_mv, a);
  return hipGetLastError();
}

hipError_t launch_bin_grad(const crsht_plan* P, int nbins, const int* edges, const double2* ahat,
                           const double2* fhat, const double2* lam, const double2* w0, double* grad,
                           hipStream_t s, int mode) {
  hipLaunchKernelGGL(k_bin_terms, dim3(nbins, kBinSlices), dim3(kVecBlock), 0, s, P->g.mmax, P->t.mstart, edges,
                     P->w.sinv, P->w.sinvhalf, ahat, fhat, lam, w0, P->w.bin_part, mode);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bin_grad, dim3((nbins + 63) / 64), dim3(64), 0, s, nbins, kBinSlices, P->w.bin_part, grad,
                     mode);
  return hipGetLastError();
}

hipError_t launch_bin_grad_dots(const crsht_plan* P, int nbins, const int* edges, const double2* x1,
                                const double2* y1, const double2* x2, const double2* y2, const double2* x3,
                                const double2* y3, double* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_bin_dots3, dim3(nbins, kBinSlices), dim3(kVecBlock), 0, s, P->g.mmax, P->g.nalm, P->ncomp,
                     P->t.mstart, edges, x1, y1, x2, y2, x3, y3, P->w.bin_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bin_grad, dim3((nbins + 63) / 64), dim3(64), 0, s, nbins, kBinSlices, P->w.bin_part, grad, 0);
  return hipGetLastError();
}

hipError_t launch_scale_per_l(const crsht_plan* P, const double2* in, const double* fac_l, double2* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_scale_l, dim3(nblocks(P->g.nalm)), dim3(kVecBlock), 0, s, P->g.nalm, P->t.idx_l, fac_l, in,
                     out);
  return hipGetLastError();
}

}  // namespace crsht
