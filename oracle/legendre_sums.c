/*
 * Legendre sums of the spherical-harmonic transforms on iso-latitude rings,
 * in plain C.
 *
 * TEST INFRASTRUCTURE ONLY (part of the oracle): loaded by oracle/clegendre.py
 * for the tests, the smoke check and the CPU baseline of the benchmark. It
 * shares no code with the HIP library.
 *
 * The same definitions as oracle/legendre.py and oracle/sht.py, written as
 * plain loops so that the transforms of the largest workloads (Nside 512 and
 * 1024) finish in seconds on the host:
 *
 *   lambda_lm(z) = Delta_lm P_lm(z), Delta_lm = (-1)^m sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
 *   (paper, App. A), evaluated by the textbook three-term recurrence
 *     lambda_mm     = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1},  lambda_00 = 1/sqrt(4 pi)
 *     lambda_{m+1,m} = sqrt(2m+3) z lambda_mm
 *     lambda_lm     = a_lm (z lambda_{l-1,m} - b_lm lambda_{l-2,m}),
 *     a_lm = sqrt((4 l^2 - 1)/(l^2 - m^2)),  b_lm = sqrt(((l-1)^2 - m^2)/(4 (l-1)^2 - 1)).
 *
 * sin^m(theta) underflows double precision near the poles at large m, so
 * the values are carried as f * 2^E: lambda_mm with its exponent taken out by
 * frexp after every factor, then the l-recurrence on mantissas that share one
 * exponent E, which is raised by 100 (and both carried mantissas scaled by
 * 2^-100, exactly) whenever a mantissa exceeds 2^100. A value is rounded to
 * double only when it is used; below the double range it is 0.
 *
 *   synthesis:  F[m][r]   = sum_{l=m}^{lmax} lambda_lm(z_r) a_lm
 *   transpose:  out_lm    = sum_r lambda_lm(z_r) G[m][r]      (lambda^2 with `square`)
 *
 * Complex numbers are interleaved (re, im) doubles; a_lm is m-major
 * (element (l, m) at mstart(m) + l - m, mstart(m) = m (lmax+1) - m (m-1)/2);
 * F and G are [mmax+1][nring]. The m values are independent and are shared
 * among OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define RESCALE_BITS 100
#define PI_VALUE 3.14159265358979323846

static int64_t mstart(int lmax, int m) { return (int64_t)m * (lmax + 1) - (int64_t)m * (m - 1) / 2; }

/* recurrence coefficients of one m: a[l], b[l] for l = m+2 .. lmax */
static void coefficients(int lmax, int m, double *a, double *b) {
  for (int l = m + 2; l <= lmax; ++l) {
    const double L = l, M = m, L1 = l - 1.0;
    a[l] = sqrt((4.0 * L * L - 1.0) / (L * L - M * M));
    b[l] = sqrt((L1 * L1 - M * M) / (4.0 * L1 * L1 - 1.0));
  }
}

/* lambda_mm(z) as mantissa and exponent */
static void lambda_mm(int m, double sin_theta, double *f, int64_t *e) {
  int ex = 0;
  double v = frexp(1.0 / sqrt(4.0 * PI_VALUE), &ex);
  int64_t E = ex;
  for (int k = 1; k <= m; ++k) {
    v = -sqrt((2.0 * k + 1.0) / (2.0 * k)) * sin_theta * v;
    if (v == 0.0) { E = INT64_MIN / 2; break; }   /* sin_theta == 0 */
    v = frexp(v, &ex);
    E += ex;
  }
  *f = v;
  *e = E;
}

static double to_double(double f, int64_t e) {
  if (e < -2200) return 0.0;
  return ldexp(f, (int)e);
}

/* Walks l = m .. lmax for one (m, z), running BODY with l and lam =
 * lambda_lm(z) rounded to double at every step. */
#define WALK_L(lmax, m, z, st, a, b, BODY)                                      \
  do {                                                                          \
    double f0_, f1_;                                                            \
    int64_t E_;                                                                 \
    lambda_mm((m), (st), &f1_, &E_);                                            \
    { const int l = (m); const double lam = to_double(f1_, E_); BODY; }         \
    if ((m) + 1 <= (lmax)) {                                                    \
      f0_ = f1_;                                                                \
      f1_ = sqrt(2.0 * (m) + 3.0) * (z) * f0_;                                  \
      { const int l = (m) + 1; const double lam = to_double(f1_, E_); BODY; }   \
    }                                                                           \
    for (int l_ = (m) + 2; l_ <= (lmax); ++l_) {                                \
      const double fn_ = (a)[l_] * ((z) * f1_ - (b)[l_] * f0_);                 \
      f0_ = f1_;                                                                \
      f1_ = fn_;                                                                \
      if (fabs(f1_) > 0x1p100) {                                                \
        f1_ = ldexp(f1_, -RESCALE_BITS);                                        \
        f0_ = ldexp(f0_, -RESCALE_BITS);                                        \
        E_ += RESCALE_BITS;                                                     \
      }                                                                         \
      { const int l = l_; const double lam = to_double(f1_, E_); BODY; }        \
    }                                                                           \
  } while (0)

/* F[m][r] = sum_l lambda_lm(z_r) alm[l, m] */
void oc_legendre_synth(int lmax, int mmax, int nring, const double *z, const double *sin_theta, const double *alm,
                       double *F) {
#pragma omp parallel
  {
    double *a = (double *)malloc((size_t)(lmax + 2) * sizeof(double));
    double *b = (double *)malloc((size_t)(lmax + 2) * sizeof(double));
#pragma omp for schedule(dynamic, 1)
    for (int m = 0; m <= mmax; ++m) {
      coefficients(lmax, m, a, b);
      const double *am = alm + 2 * mstart(lmax, m);
      for (int r = 0; r < nring; ++r) {
        double sre = 0.0, sim = 0.0;
        WALK_L(lmax, m, z[r], sin_theta[r], a, b, {
          sre += lam * am[2 * (l - m)];
          sim += lam * am[2 * (l - m) + 1];
        });
        F[2 * ((int64_t)m * nring + r)] = sre;
        F[2 * ((int64_t)m * nring + r) + 1] = sim;
      }
    }
    free(a);
    free(b);
  }
}

/* out[l, m] = sum_r lambda_lm(z_r) G[m][r] (lambda^2 if square) */
void oc_legendre_adjoint(int lmax, int mmax, int nring, const double *z, const double *sin_theta, const double *G,
                         int square, double *out) {
#pragma omp parallel
  {
    double *a = (double *)malloc((size_t)(lmax + 2) * sizeof(double));
    double *b = (double *)malloc((size_t)(lmax + 2) * sizeof(double));
#pragma omp for schedule(dynamic, 1)
    for (int m = 0; m <= mmax; ++m) {
      coefficients(lmax, m, a, b);
      double *om = out + 2 * mstart(lmax, m);
      for (int l = m; l <= lmax; ++l) om[2 * (l - m)] = om[2 * (l - m) + 1] = 0.0;
      for (int r = 0; r < nring; ++r) {
        const double gre = G[2 * ((int64_t)m * nring + r)], gim = G[2 * ((int64_t)m * nring + r) + 1];
        WALK_L(lmax, m, z[r], sin_theta[r], a, b, {
          const double w = square ? lam * lam : lam;
          om[2 * (l - m)] += w * gre;
          om[2 * (l - m) + 1] += w * gim;
        });
      }
    }
    free(a);
    free(b);
  }
}

/* lambda_lm(z_k) for one m: out[(l - m) * nz + k], l = m .. lmax */
void oc_lambda_m(int lmax, int m, int nz, const double *z, const double *sin_theta, double *out) {
  double *a = (double *)malloc((size_t)(lmax + 2) * sizeof(double));
  double *b = (double *)malloc((size_t)(lmax + 2) * sizeof(double));
  coefficients(lmax, m, a, b);
  for (int k = 0; k < nz; ++k) {
    WALK_L(lmax, m, z[k], sin_theta[k], a, b, { out[(int64_t)(l - m) * nz + k] = lam; });
  }
  free(a);
  free(b);
}
