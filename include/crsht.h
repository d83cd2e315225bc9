/*
 * crsht -- constrained-realization solves and spherical-harmonic transforms on
 * HEALPix, for AMD Instinct MI355X (gfx950).
 *
 * The library solves the constrained-realization (CR) system of Eskilt et al.
 * 2023 (arXiv:2306.15511), Sect. 2.2.1, eq. (mapmakingeq):
 *
 *     (S^-1 + B Y^T N^-1 Y B) s = B Y^T N^-1 d + S^-1/2 w0 + B Y^T N^-1/2 w1
 *
 * with S = diag(C_l) the signal covariance, B = diag(b_l) the beam, Y the
 * spherical-harmonic synthesis onto HEALPix pixels (RING order), Y^T its exact
 * transpose, N^-1 the per-pixel inverse noise variance (0 = masked), d the
 * map and w0, w1 unit white-noise draws. The paper's "B" (beam and projection)
 * is Y B here. It also implements one joint C_l-amplitude / sky Metropolis
 * move (Sect. 2.2.2, eq. acceptance-rate and the algorithm that follows it).
 *
 * Conventions
 *   - a_lm of a real field: m >= 0 only, m-major (for m = 0..mmax, l = m..lmax),
 *     complex interleaved float64: element (l, m) of column c is at
 *     alm[2*(c*nalm + mstart(m) + l - m) + {0: Re, 1: Im}],
 *     mstart(m) = m*(lmax+1) - m*(m-1)/2, nalm = mstart(mmax+1).
 *     Im a_l0 is ignored on input and written as 0.
 *   - Y_lm = Delta_lm P_lm(cos theta) e^{i m phi} with one overall (-1)^m
 *     (paper App. A); (Y a)_p = sum_l [a_l0 lambda_l0 + 2 Re sum_{m>0} a_lm Y_lm(p)].
 *   - (Y^T x)_lm = sum_p x_p Y*_lm(p): the plain transpose, no quadrature weight.
 *     It is the adjoint of Y under <a,c> = sum_l a_l0 c_l0 + 2 sum_{m>0} Re(a_lm c*_lm).
 *   - Maps: float64 [nrhs][npix], HEALPix RING order (Gorski et al. 2005).
 *   - Column c of a batched call is array slice c; columns are independent.
 *   - Plans with ncomp = 3 (temperature and polarisation, the T, E, B spectra
 *     and the 3x3 covariance blocks of Sect. 2.2.2): a column holds three
 *     coefficient blocks (a_T, a_E, a_B), alm [nrhs][3][nalm], and three maps
 *     (T, Q, U), map [nrhs][3][npix]; everything documented below as [nalm]
 *     or [npix] per column is [3][nalm] or [3][npix] for such plans. Q and U
 *     follow the HEALPix / COSMO convention: Q +- iU = sum (+-2 a_lm)(+-2 Y_lm)
 *     with +-2 a_lm = -(a_E +- i a_B) and +-2 Y_lm the spin-raised scalar
 *     harmonics (Goldberg et al. 1967) divided by sqrt((l-1) l (l+1) (l+2)).
 *
 * Memory and streams
 *   - Pointers documented as "device" are caller-owned device memory on the
 *     plan's device; the library never frees or keeps them past the call.
 *     Pointers documented as "host" are host memory.
 *   - A plan owns its tables and workspace (allocated at creation, sized for
 *     nrhs_max columns); calls allocate nothing.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). Transforms,
 *     cr_apply and cr_solve_async are asynchronous on it (cr_solve_async writes
 *     its statistics to device memory). cr_solve, cr_lnpi, joint_cl_step and
 *     the other chain moves synchronise `stream` (they read convergence
 *     scalars back); their outputs are complete when they return.
 *   - Calls allocate no device memory: plans own their workspace, staging
 *     and streams; cr_block_precond_build (a set-up call, once per noise
 *     model) allocates the preconditioner's storage.
 *   - A plan is not thread-safe: concurrent calls need distinct plans.
 *
 * Errors: functions return CR_OK (0) or a negative code detected before or
 * while enqueueing work; numerical outcomes go to cr_stats.status.
 */
#ifndef CRSHT_H
#define CRSHT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CR_OK = 0,
  CR_EINVAL = -1,    /* invalid argument (sizes, NULL pointers, bad spectra) */
  CR_ENOMEM = -2,    /* device allocation failed at plan creation */
  CR_EDEVICE = -3,   /* a HIP runtime call or kernel launch failed */
  CR_ENOTSUP = -4,   /* valid but not supported by this library */
  CR_ESCRATCH = -5,  /* sht_synth_noalloc: the call needs more than its static scratch */
  CR_NOCONV = 1,     /* maxiter reached; the last iterate is written */
  CR_BREAKDOWN = 2   /* <p, A p> <= 0 or non-finite; output undefined */
};

typedef struct crsht_plan crsht_plan;

/* Arithmetic of the transforms.
 * CR_F64: float64 throughout (FP64 matrix cores for two or more columns,
 *   vector ALU for one).
 * CR_MIXED (bf16x3): the lambda_lm recurrence stays float64; recurrence
 *   values and a_lm / ring coefficients are rounded to float and split into
 *   bf16 hi + lo parts, and each product is formed as hi*hi + hi*lo + lo*hi on
 *   the matrix cores with float32 accumulation (relative error about 5e-6 per
 *   transform); the ring FFTs run in float32; CG vectors, dot products and
 *   scalars stay float64. In cr_solve it is the inner operator of float64
 *   iterative refinement. T+Q+U plans: Q and U come from Legendre sums that
 *   cancel near the poles and are divided by sin^2(theta), so the ring pairs
 *   with sin^2(theta) < 0.01 take float64 Legendre sums (the rounding of the
 *   others is amplified by at most 100).
 * CR_BF16X6: user-visible transforms (sht_synth, sht_synth_adjoint,
 *   sht_synth_grad, cr_apply) to about 1e-7: the same kernels with three bf16
 *   parts per operand (hi, mid, lo; the float value to 2^-24) and the six
 *   products of total order <= 2, float32 accumulation and float32 ring FFTs.
 *   Not a cr_solve precision (CR_EINVAL there). */
typedef enum { CR_F64 = 0, CR_MIXED = 1, CR_BF16X6 = 3 } cr_prec;

/* Preconditioner of cr_solve (cr_opts.precond). */
enum { CR_PC_JACOBI = 0, CR_PC_BLOCK = 1 };
/* cr_opts.terms */
enum { CR_SUM = 0, CR_SEPARATE = 4 };

/* Create a plan for HEALPix resolution nside (power of two not required,
 * 1 <= nside <= 1024; larger nside returns CR_ENOTSUP), band limit lmax >= 0 and mmax (<= lmax; pass -1 for
 * mmax = lmax), ncomp = 1 (temperature) or 3 (temperature and polarisation),
 * for up to nrhs_max >= 1 columns per call. Builds the ring table (Gorski et
 * al. 2005), the recurrence tables of lambda_lm (paper App. A normalisation)
 * and the per-ring FFT tables, and allocates the workspace on the current HIP
 * device (a ncomp = 3 plan holds 9 Legendre-sum columns per right-hand side).
 * Returns CR_EINVAL, CR_ENOTSUP or CR_ENOMEM on failure (*out set to NULL). */
int crsht_plan_create(int nside, int lmax, int mmax, int ncomp, int nrhs_max, crsht_plan **out);

/* Free a plan and everything it owns. NULL is allowed. */
void crsht_plan_destroy(crsht_plan *plan);

/* Static string describing a status code. */
const char *crsht_strerror(int status);

typedef struct {
  int nside, lmax, mmax, ncomp, nrhs_max, nrings;
  int64_t npix, nalm;
  int64_t workspace_bytes;   /* device memory owned by the plan */
  int64_t precond_bytes;     /* bytes of the n x n entries of the stored
                                block-preconditioner inverses, each read once
                                per cr_block_precond_apply (0 if none is built) */
  int precond_blocks, precond_half_blocks;   /* blocks stored, of which in FP16 */
  int64_t live_pair_m;       /* (ring pair, m) combinations at which the pair's
                                Legendre values are not all below the underflow
                                threshold, of npairs x (mmax + 1): the Legendre
                                sums the mixed-precision T operator's ring pass
                                reads and writes per column */
} crsht_info;

/* Fill *info (host). */
int crsht_plan_info(const crsht_plan *plan, crsht_info *info);

/* Pixel-centre coordinates z = cos(theta) and phi of every pixel, RING order,
 * written to host arrays of npix doubles each. */
int crsht_pixel_coords(const crsht_plan *plan, double *z_host, double *phi_host);

/* Synthesis Y (paper Sect. 2.1, a(n) = sum a_lm Y_lm(n)).
 * alm: device, [nrhs][nalm] complex; map: device, [nrhs][npix].
 * 1 <= nrhs <= nrhs_max. prec: CR_F64 or CR_MIXED. Asynchronous. */
int sht_synth(const crsht_plan *plan, int nrhs, const double *alm, double *map, cr_prec prec, void *stream);

/* Bytes of the file-scope device scratch of sht_synth_noalloc (one copy per
 * GPU the library runs on, held until the process ends). */
#define CRSHT_NOALLOC_SCRATCH_BYTES (96u << 20)

/* sht_synth without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Same arguments, kernels and result as sht_synth
 * (temperature plans only: CR_ENOTSUP for ncomp = 3). The transform's
 * intermediate buffers (the scaled a_lm and the Legendre sums) live in a
 * static device scratch of CRSHT_NOALLOC_SCRATCH_BYTES instead of the plan
 * workspace; the call allocates nothing (no hipMalloc, no library routine
 * that allocates). Needs CR_F64: nrhs (16 nalm + 32 npairs (mmax+1)) bytes
 * (nalm term rounded up to 256), CR_MIXED: nrhs 16 npairs (mmax+1) bytes,
 * else CR_ESCRATCH (Nside 512, lmax 1535: one FP64 or three mixed columns).
 * The plan's device must be current (CR_EINVAL otherwise) and kernel timing
 * off (CR_EINVAL). Every call on one GPU shares that GPU's scratch, which
 * keeps the last call's contents: calls that overlap on one GPU (different
 * streams or threads, any plans) race and must be serialised by the caller.
 * The scratch's device address is looked up once per device at plan
 * creation. Asynchronous. */
int sht_synth_noalloc(const crsht_plan *plan, int nrhs, const double *alm, double *map, cr_prec prec,
                      void *stream);

/* Adjoint synthesis Y^T (the transpose; paper App. A pixel sums).
 * map: device [nrhs][npix]; alm: device [nrhs][nalm] complex. Asynchronous. */
int sht_synth_adjoint(const crsht_plan *plan, int nrhs, const double *map, double *alm, cr_prec prec,
                      void *stream);

/* Analysis: alm = (4 pi / Npix) Y^T map, followed by n_iter >= 0 Jacobi
 * corrections alm += (4 pi / Npix) Y^T (map - Y alm) (App. A: the pixel sum as
 * Npix/(4 pi) times the sphere integral). FP64. Asynchronous. */
int sht_analysis(const crsht_plan *plan, int nrhs, const double *map, double *alm, int n_iter, void *stream);

/* The statement of the problem (paper Sect. 2.2.1, r = B a + n; App. A N^-1). */
typedef struct {
  const double *cl;    /* host, [lmax+1]: C_l (temperature). Modes with l < lmin are fixed to 0;
                          C_l must be > 0 and finite for lmin <= l <= lmax.
                          ncomp = 3: [4][lmax+1] = TT, EE, BB, TE; per l >= lmin the block
                          [[TT, TE], [TE, EE]] must be positive definite and BB > 0 (TB = EB = 0).
                          S^-1/2 is the symmetric principal root of the block inverse. */
  const double *bl;    /* host, [lmax+1]: beam transfer function b_l (finite), all components. */
  const double *ninv;  /* device, [npix]: inverse noise variance per pixel, >= 0, 0 = masked.
                          ncomp = 3: [3][npix] for T, Q, U (no Q-U noise correlation). */
  int lmin;            /* first constrained multipole, 0 <= lmin <= lmax (2 for C_0 = C_1 = 0);
                          ncomp = 3 requires lmin >= 2. */
  const double *amp;   /* host, [nrhs] or NULL: column c of cr_rhs, cr_apply, cr_solve and
                          cr_solve_batched solves with the spectrum amp[c] C_l (amp[c] > 0 and
                          finite; NULL = 1 for every column), e.g. the right-hand sides of several
                          chains at different amplitudes in one call. The preconditioners (Jacobi
                          and block) stay those of C_l. Every other call taking a cr_problem
                          requires NULL (CR_EINVAL otherwise). */
} cr_problem;

typedef struct {
  double tol;          /* target relative residual ||b - A s|| / ||b|| (real-field norm), > 0 */
  int maxiter;         /* maximum CG iterations (all refinement sweeps together), >= 1 */
  cr_prec prec;        /* CR_F64: plain PCG; CR_MIXED: PCG on the mixed operator with FP64 residual
                          replacement (iterative refinement that keeps the search directions) */
  double inner_tol;    /* CR_MIXED: the FP64 true residual replaces the recursive one each time the latter
                          has dropped by this factor (0 < inner_tol < 1, e.g. 1e-2); ignored for CR_F64 */
  int max_refine;      /* CR_MIXED: maximum number of FP64 residual replacements (0 = 1000) */
  int check_every;     /* iterations between host convergence checks (>= 1; 0 = 8) */
  int precond;         /* CR_PC_JACOBI (0): the Jacobi diagonal of cr_precond, rebuilt by every solve;
                          CR_PC_BLOCK (1): the per-m block preconditioner stored in the plan by
                          cr_block_precond_build (CR_EINVAL if none is built) */
  int use_graph;       /* 1: each block of check_every iterations is captured once as a HIP graph
                          (plan-owned, re-captured when nrhs, ninv, tol, precision or the block
                          length change) and replayed on `stream`; 0: every kernel is launched
                          directly. Results are identical either way. Ignored while kernel timing
                          is enabled. */
  int terms;           /* read by cr_solve only. CR_SUM (0): one solution per column for the sum of
                          the given terms; CR_SEPARATE: per column the mean field (d term, eq.
                          mean-field-map) and the fluctuation (w0 and w1 terms, eq. fluc-map) as
                          two solutions, solved together as 2 nrhs columns (needs 2 nrhs <=
                          nrhs_max, d and at least one of w0, w1 non-NULL, rhs NULL) */
} cr_opts;

typedef struct {
  int status;              /* CR_OK, CR_NOCONV or CR_BREAKDOWN */
  int iters;               /* CG iterations (inner iterations summed for CR_MIXED) */
  int refinements;         /* FP64 residual replacements (0 for CR_F64) */
  double rel_resid_true;   /* ||b - A s|| / ||b|| evaluated in FP64 at exit */
} cr_stats;

/* Jacobi preconditioner diagonal (the paper's "standard diagonal
 * preconditioner", Sect. 4): D_lm = 1/C_l + b_l^2 sum_r lambda_lm(z_r)^2 W_r,
 * W_r = sum of N^-1 over ring r. diag: device [nalm] float64 (1 where l < lmin).
 * ncomp = 3: diag [3][nalm] with the diagonal entries of the S^-1 blocks, W_r
 * of N_T^-1 for T and the mean of the Q and U ring sums for E and B (the
 * spin-0 lambda_lm stand in for the spin-2 functions: an approximation that
 * only needs to stay positive). Asynchronous. */
int cr_precond(const crsht_plan *plan, const cr_problem *prob, double *diag, void *stream);

/* Per-m block preconditioner (paper App. A; Sect. 4 names better
 * preconditioners as the main lever on the cost of the solve). For every m and
 * parity q of l - m, the dense matrix
 *   M_mq[l, l'] = delta_ll' / C_l + b_l b_l' sum_r lambda_lm(z_r) lambda_l'm(z_r) W_r,
 * l, l' = m + q, m + q + 2, ..., with W_r the ring sum of N^-1 averaged over
 * ring r and its mirror ring (exact m-blocks of the operator for a noise
 * model that depends on latitude only and is symmetric under z -> -z, as for
 * the paper's constant-latitude mask; an SPD preconditioner otherwise; rows
 * l < lmin are the identity) is formed in FP64, inverted by Cholesky
 * factorisation (rocBLAS SYRK for the Gram matrices, rocSOLVER potrf/potri
 * for the factorisation and inverse, on blocks padded to multiples of 32
 * with the identity) and stored full symmetric in the plan as
 * S C S, S = diag(M^-1)^1/2 (FP32), C with a unit diagonal in FP16 where a
 * Cholesky factorisation of fl16(C) - 2 ||fl16(C) - C||_F I succeeds (the
 * rounding then keeps C positive definite and moves the eigenvalues of the
 * preconditioned operator by less than a factor 2, in practice by a few per
 * cent), else in FP32 (low-m blocks of a masked sky); storage about
 * 2 (lmax + 1)^3 / 3 bytes, crsht_info.precond_bytes of it read per
 * application; allocated by this call, freed with the plan or by the next
 * build. Built once per noise model, beam and spectrum shape,
 * it stays valid when the spectrum is rescaled (joint_cl_step): PCG only
 * needs a fixed symmetric positive definite preconditioner.
 * ncomp = 3: three sets of blocks, one per component, three times the
 * storage. T as above with N_T^-1 and (S^-1)_TT; E and B with the spin-2
 * functions of the polarisation transforms,
 *   M^E_mq[l, l'] = (S^-1)_EE,l delta_ll' + b_l b_l' sum_r (W_lm W_l'm + X_lm X_l'm)(z_r) W_P,r,
 * M^B with (S^-1)_BB, W_P,r the mean of the Q and U ring sums (mirror
 * averaged). The T-E prior coupling and the E-B coupling are left out, so
 * the preconditioner is block diagonal per component (exact E-E and B-B
 * m-blocks when the Q and U noise are equal and depend on latitude only).
 * CR_EINVAL if a block is not positive definite (or lmin < 2 for ncomp = 3).
 * Blocks until done. */
int cr_block_precond_build(crsht_plan *plan, const cr_problem *prob, void *stream);

/* z = M^-1 r with the stored block preconditioner, per column (the real and
 * imaginary parts alike). r, z: device [nrhs][ncomp][nalm], distinct.
 * CR_EINVAL if none is built. Asynchronous. */
int cr_block_precond_apply(const crsht_plan *plan, int nrhs, const double *r, double *z, void *stream);

/* Unit Gaussian white draws for the random terms of eq. mapmakingeq on the
 * device: w0 (device [nrhs][ncomp][nalm]) gets white a_lm of a real field
 * (Re and Im of N(0, 1/2) for m > 0, real N(0, 1) for m = 0), w1 (device
 * [nrhs][ncomp][npix]) standard normal pixels; either may be NULL, not both.
 * Philox4x32-10 (Salmon et al. 2011) keyed by `seed`, with counter words
 * (element, column | purpose << 31, counter lo, counter hi): every value
 * depends only on (seed, counter, column, element), and w0 and w1 of one call
 * are independent. Two standard normals per generator block by the
 * Box-Muller transform of two 53-bit uniforms. Asynchronous. */
int cr_white(const crsht_plan *plan, int nrhs, uint64_t seed, uint64_t counter, double *w0, double *w1,
             void *stream);

/* Right-hand side of eq. mapmakingeq: b = B Y^T N^-1 d + S^-1/2 w0 + B Y^T N^-1/2 w1,
 * restricted to l >= lmin. d, w1: device maps [nrhs][npix]; w0: device alm
 * [nrhs][nalm]; any of the three may be NULL (term omitted). b: device
 * [nrhs][nalm]. Asynchronous. */
int cr_rhs(const crsht_plan *plan, const cr_problem *prob, int nrhs, const double *d, const double *w0,
           const double *w1, double *b, void *stream);

/* The operator alone: Ax = (S^-1 + B Y^T N^-1 Y B) x on l >= lmin (0 below).
 * x, Ax: device [nrhs][nalm]. Asynchronous. */
int cr_apply(const crsht_plan *plan, const cr_problem *prob, int nrhs, const double *x, double *Ax,
             cr_prec prec, void *stream);

/* Solve eq. mapmakingeq for nrhs independent columns by preconditioned
 * conjugate gradients (Shewchuk 1994) from s = 0. The right-hand side is
 * assembled as in cr_rhs from d, w0, w1 (NULL = omitted: d only gives the mean
 * field of eq. mean-field-map, w0 and w1 only the fluctuation of eq. fluc-map),
 * unless rhs is non-NULL (device [nrhs][nalm]), which is used as b directly.
 * s_out: device [nrhs][nalm]. stats: host, nrhs entries. With opts->terms =
 * CR_SEPARATE: s_out [nrhs][2][ncomp][nalm] (mean field, then fluctuation, of
 * each column; the sum is the CR_SUM solution up to the tolerance) and stats
 * 2 nrhs entries in the same order; cr_problem.amp[c] applies to both
 * solutions of column c.
 * With the environment variable CRSHT_PROGRESS = k > 0, every k-th host
 * convergence check prints the iteration count and the largest recursive
 * residual of the open columns to stderr (long solves).
 * Blocks until the solve has finished on `stream`. */
int cr_solve(const crsht_plan *plan, const cr_problem *prob, int nrhs, const double *d, const double *w0,
             const double *w1, const double *rhs, double *s_out, const cr_opts *opts, cr_stats *stats,
             void *stream);

/* The solve of cr_solve, stream-ordered: the whole solve (right-hand side,
 * PCG, FP64 residual replacements, final true residual) is enqueued on
 * `stream` and the call returns at once; nothing waits on the host. The
 * decisions the host loop of cr_solve takes from scalars it reads back (when
 * to replace the residual, restart a direction, stop a column or the solve)
 * are taken on the device by a small control kernel between sections whose
 * kernels return at once once the solve has stopped. With opts->use_graph
 * each block of check_every iterations is one replay of a captured graph.
 * ceil(maxiter / check_every) blocks are enqueued, so maxiter should be near
 * the expected count (blocks after convergence cost a few microseconds per
 * kernel; the iteration count may exceed maxiter by less than check_every).
 * CR_MIXED: the iterates of cr_solve; CR_F64: PCG with the FP64 operator whose
 * residual is replaced by the true one when a column claims convergence.
 * stats_dev: device memory for nrhs cr_stats, written by the last kernel of
 * the solve: valid after the stream has been synchronised (or any later work
 * on it). s_out: device [nrhs][nalm]. The per-call host data (spectra, beam,
 * amplitudes) is copied through pinned staging slots of the plan: more than
 * four calls enqueued ahead of the device wait for the oldest. Other
 * arguments and errors as cr_solve (errors are detected before enqueueing;
 * opts->terms must be CR_SUM). Consecutive calls on one plan must use one
 * stream (they share the plan
 * workspace); changing nrhs, tolerance, preconditioner or limits between
 * calls re-captures the graphs after synchronising the device once. */
int cr_solve_async(const crsht_plan *plan, const cr_problem *prob, int nrhs, const double *d, const double *w0,
                   const double *w1, const double *rhs, double *s_out, const cr_opts *opts, cr_stats *stats_dev,
                   void *stream);

/* Many independent problems at once (each with its own plan, so Nside, lmax
 * and the noise model may all differ): problem i solves eq. mapmakingeq for
 * one column with plans[i], probs[i], d[i], w0[i], w1[i] (device; any of the
 * three arrays of pointers, or an entry, may be NULL = term omitted) into
 * s_out[i] (device [nalm_i]); stats: host [nprob]. The plans must be
 * distinct (each solve uses its plan's workspace) and on the current device.
 * Every problem runs the device-driven solve of cr_solve_async on its plan's
 * own stream (created with the plan), forked from `stream` by an event and
 * joined back to it; its blocks of check_every iterations are replays of
 * the plan's captured graph. No host threads and no streams are created per
 * call: one host loop enqueues the next block of every problem that the
 * device has not yet flagged as finished, keeping two blocks per problem in
 * flight. All share `opts`. Returns the first error. Blocks until all are
 * done. */
int cr_solve_batched(const crsht_plan *const *plans, const cr_problem *probs, int nprob, const double *const *d,
                     const double *const *w0, const double *const *w1, double *const *s_out, const cr_opts *opts,
                     cr_stats *stats, void *stream);

/* ln pi of the joint move (Sect. 2.2.2, definition of pi(theta)) for the
 * amplitude-scaled spectrum C_l(q) = q cl:
 *   ln pi = -1/2 (d - Y B a)^T N^-1 (d - Y B a) - 1/2 a^T S(q)^-1 a - 1/2 f^T B Y^T N^-1 Y B f
 * d: device map; ahat, fhat: device alm [nalm]. Result to *lnpi (host).
 * T+Q+U plans: d [3][npix], ahat, fhat [3][nalm]; the chi^2 and fluctuation
 * terms summed over T, Q, U with their N^-1, the prior with the 3x3 blocks of
 * S(q)^-1. Blocks until done. */
int cr_lnpi(const crsht_plan *plan, const cr_problem *fid, double q, const double *d, const double *ahat,
            const double *fhat, double *lnpi, void *stream);

/* State of one amplitude chain (host struct, device arrays of nalm complex). */
typedef struct {
  double q;            /* current amplitude, C_l = q * fid.cl */
  double lnpi;         /* ln pi(q) of the current (ahat, fhat) */
  double *ahat;        /* device [nalm]: mean field at q */
  double *fhat;        /* device [nalm]: fluctuation at q */
} cr_chain;

/* Randomness of one move, drawn by the caller. */
typedef struct {
  double xi;           /* standard normal: proposal ln q' = ln q + sigma_lnq xi */
  double u;            /* uniform in (0,1): accept iff ln u < ln A */
  const double *w0;    /* device [nalm]: fresh w0 for the fluctuation solve on acceptance */
  const double *w1;    /* device [npix]: fresh w1 */
  double sigma_lnq;    /* proposal width in ln q (> 0) */
} cr_draws;

typedef struct {
  int accepted;
  double lnA;          /* ln of the acceptance ratio (FP64) */
  double q_new;        /* proposed amplitude */
  double lnpi_new;     /* ln pi at the proposal with the rescaled fluctuation */
  cr_stats mean_stats; /* mean-field solve */
  cr_stats fluct_stats;/* fluctuation solve (zeros if rejected) */
} cr_step_out;

/* One joint C_l-amplitude / sky move (paper Sect. 2.2.2, algorithm steps 2-4),
 * temperature and T+Q+U plans (all four spectra scaled by q; states of
 * [3][nalm] coefficients, maps [3][npix]):
 * propose q' = q exp(sigma xi); solve the mean field at q'; rescale the
 * fluctuation by sqrt(q'/q); ln A = ln pi(q') - ln pi(q) + ln(q'/q) (uniform
 * prior in q; Gaussian proposal in ln q); accept iff ln u < ln A, and only then
 * solve a fresh fluctuation with draws->w0, w1 and update *state (q, lnpi,
 * ahat, fhat in place). The mean-field solve starts from state->ahat (the
 * mean field at q; the solve runs on the correction to the same tolerance
 * relative to the right-hand side). Needs nrhs_max >= 1; uses the plan
 * workspace.
 * `out` is host. Blocks until done. */
int joint_cl_step(const crsht_plan *plan, const cr_problem *fid, const double *d, cr_chain *state,
                  const cr_draws *draws, const cr_opts *opts, cr_step_out *out, void *stream);

/* The joint move of joint_cl_step for nchains chains at once, sharing the
 * data d: the mean fields at every chain's proposal q'_c = q_c exp(sigma_lnq
 * xi[c]) are the columns of one solve (per-column amplitudes, each warm-started
 * from the chain's mean field; the solve runs to the strictest column's
 * correction tolerance), and the fresh fluctuations of the chains that accept
 * are the columns of a second solve from w0, w1 (solved for every chain when
 * any accepts; the columns of rejected chains are discarded). The decision of
 * chain c is ln u[c] < ln A_c with ln A as in joint_cl_step. states: host
 * [nchains], updated in place like joint_cl_step's state; xi, u: host
 * [nchains]; w0: device [nchains][nalm]; w1: device [nchains][npix] (either
 * may be NULL, not both); out: host [nchains]. nchains <= nrhs_max of the
 * plan; fid->amp must be NULL. Temperature plans only. Blocks until done. */
int joint_cl_step_batch(const crsht_plan *plan, const cr_problem *fid, const double *d, int nchains,
                        cr_chain *states, const double *xi, const double *u, double sigma_lnq, const double *w0,
                        const double *w1, const cr_opts *opts, cr_step_out *out, void *stream);

typedef struct {
  double q_new;        /* the drawn amplitude */
  double t;            /* s^T S_fid^-1 s of the sky the draw conditioned on */
  cr_stats mean_stats; /* mean-field solve at q_new */
  cr_stats fluct_stats;/* fluctuation solve at q_new */
} cr_gibbs_out;

/* One move of the standard two-block Gibbs sampler (paper Sect. 2.2.1,
 * standard CMB Gibbs sampling: amplitude given sky, then sky given
 * amplitude), for the one-parameter family C_l(q) = q C_l^fid with a uniform
 * prior in q — the baseline the joint move of joint_cl_step is compared with.
 * With s = ahat + fhat the chain's current sky and t = s^T S_fid^-1 s over
 * l >= lmin (real-field product), q | s is inverse gamma with shape
 * alpha = k/2 - 1, k = sum_{l=lmin}^{lmax} (2l + 1), and scale t/2; the caller
 * draws g ~ Gamma(alpha, 1) and the move sets q' = (t/2) / g. Then s | q':
 * the mean field (warm-started from state->ahat) and a fresh fluctuation from
 * w0, w1 (device; either may be NULL, not both), and ln pi of the new state.
 * *state is updated in place; `out` is host. Temperature plans (CR_ENOTSUP
 * for ncomp = 3). Blocks until done. */
int gibbs_cl_step(const crsht_plan *plan, const cr_problem *fid, const double *d, cr_chain *state, double g,
                  const double *w0, const double *w1, const cr_opts *opts, cr_gibbs_out *out, void *stream);

/* The Gibbs move of gibbs_cl_step for nchains chains at once: q'_c from
 * g[c] and chain c's sky, then one solve of 2 nchains columns: columns
 * 0..nchains-1 the mean fields (warm-started from the chains' mean fields),
 * columns nchains..2 nchains-1 the fluctuations from w0, w1, each column at
 * its chain's amplitude (the columns of the mean-field and fluctuation terms
 * of several chains, as in a multi-chain Gibbs sampler). states, g, out:
 * host [nchains]; w0: device [nchains][nalm], w1: device [nchains][npix]
 * (either may be NULL, not both). 2 nchains <= nrhs_max of the plan;
 * fid->amp must be NULL. Temperature plans only. Blocks until done. */
int gibbs_cl_step_batch(const crsht_plan *plan, const cr_problem *fid, const double *d, int nchains,
                        cr_chain *states, const double *g, const double *w0, const double *w1, const cr_opts *opts,
                        cr_gibbs_out *out, void *stream);

/* ln pi (Sect. 2.2.2, definition of pi(theta)) and its gradient in per-bin
 * log-amplitudes theta_k (C_l -> C_l^fid exp(theta_k) for edges[k] <= l <
 * edges[k+1]) at a fixed whitened fluctuation: the fluctuation f0, given at
 * theta0, is carried to theta as f = exp((theta - theta0)/2) f0 per bin (the
 * rescaling of the joint move), so that
 *   d ln pi / d theta_k = 1/2 a^T S^-1_k a - 1/2 f^T B Y^T N^-1 Y B f_k
 * with a the mean field at theta (it minimises chi^2 + a^T S^-1 a, so only the
 * explicit S^-1 is differentiated; no adjoint solve). The mean-field solve
 * starts from a0 (device [nalm], may be NULL) and its result goes to ahat
 * (device [nalm], may be NULL). theta0, theta: host [nbins]; f0: device
 * [nalm]; edges: host, nbins + 1 strictly increasing values in [0, lmax + 1];
 * grad: host [nbins]; *lnpi host; stats: host, one entry (the mean-field
 * solve). Temperature plans only. Blocks until done. */
int cr_lnpi_grad_fixed(const crsht_plan *plan, const cr_problem *fid, const double *d, int nbins, const int *edges,
                       const double *theta0, const double *theta, const double *f0, const double *a0,
                       const cr_opts *opts, double *lnpi, double *grad, double *ahat, cr_stats *stats, void *stream);

/* State of a chain over per-bin log-amplitudes (host struct, device vectors). */
typedef struct {
  int nbins;
  const int *edges;    /* host, nbins + 1 bin edges in l */
  double *theta;       /* host [nbins]: log-amplitudes, C_l = C_l^fid exp(theta_k) */
  double lnpi;         /* ln pi of the current state */
  double *ahat;        /* device [nalm]: mean field */
  double *fhat;        /* device [nalm]: fluctuation */
} cr_bin_chain;

/* Randomness and tuning of one HMC move, drawn by the caller. */
typedef struct {
  const double *p0;    /* host [nbins]: momentum, standard normal */
  double u;            /* uniform in (0,1): accept iff ln u < -(H_end - H_start) */
  const double *w0;    /* device [nalm]: fresh w0 for the fluctuation after the move */
  const double *w1;    /* device [npix]: fresh w1 */
  double eps;          /* leapfrog step in theta (> 0) */
  int nleap;           /* leapfrog steps (>= 1) */
} cr_hmc_draws;

typedef struct {
  int accepted;
  int status;          /* CR_OK, or the status of a mean-field solve that did not converge */
  double dH;           /* H_end - H_start */
  double lnpi_new;     /* ln pi at the end of the trajectory (rescaled fluctuation) */
  int solves;          /* mean-field solves of the trajectory (nleap + 1) */
  int iters;           /* their iterations, summed */
  cr_stats fluct_stats;/* fresh fluctuation solve */
} cr_hmc_out;

/* One Hamiltonian Monte Carlo move of the per-bin log-amplitudes (the
 * derivative-based sampler the paper's discussion points to, Sect. 4; the
 * same target as the joint move: ln pi at a fixed whitened fluctuation, with
 * a uniform prior in the amplitudes exp(theta_k), i.e. the potential
 * U = -ln pi - sum_k theta_k and unit masses). nleap leapfrog steps of size
 * eps from momentum p0, each with one warm-started mean-field solve and the
 * gradient of cr_lnpi_grad_fixed; accept iff ln u < -(H_end - H_start). Then,
 * accepted or not, a fresh fluctuation from w0, w1 at the amplitudes the move
 * ends on (a draw of the whitened fluctuation given the amplitudes, which
 * leaves the joint target invariant by itself) and ln pi of the new state;
 * *state is updated in place (theta and ahat kept on rejection). `out` host.
 * Temperature plans only. Blocks until done. */
int hmc_cl_step(const crsht_plan *plan, const cr_problem *fid, const double *d, cr_bin_chain *state,
                const cr_hmc_draws *draws, const cr_opts *opts, cr_hmc_out *out, void *stream);

/* The standard two-block Gibbs move (paper Sect. 2.2.1: amplitudes given the
 * sky, then the sky given the amplitudes) for per-bin amplitudes A_b =
 * exp(theta_b) of C_l = C_l^fid A_b on [edges[b], edges[b+1]) with uniform
 * priors in the A_b: with s = ahat + fhat and t_b = s^T S_fid^-1 s summed
 * over the bin (real-field product), A_b | s is inverse gamma with shape
 * k_b/2 - 1 (k_b = sum over the bin of 2l + 1) and scale t_b/2; the caller
 * draws g_b ~ Gamma(k_b/2 - 1, 1) (host [nbins]) and the move sets theta_b =
 * ln((t_b/2) / g_b). Then the mean field (warm-started from state->ahat) and
 * a fresh fluctuation from w0, w1 (device; either may be NULL, not both) at
 * the new spectrum, and ln pi of the new state; *state updated in place.
 * Bins must start at or above fid->lmin. t: host [nbins] or NULL (the t_b);
 * stats: host [2] (mean field, fluctuation). Temperature plans only. Blocks
 * until done. */
int gibbs_bins_step(const crsht_plan *plan, const cr_problem *fid, const double *d, cr_bin_chain *state,
                    const double *g, const double *w0, const double *w1, const cr_opts *opts, double *t,
                    cr_stats *stats, void *stream);

/* Gradient of the synthesis for reverse-mode differentiation of a real
 * function L of the map: alm_grad = w_m Y^T map_grad with w_0 = 1 (Im of m = 0
 * set to 0) and w_{m>0} = 2, i.e. dL/dRe a_lm + i dL/dIm a_lm for a complex
 * leaf that stores the m >= 0 half of a real field (the convention of
 * torch.autograd for complex tensors). map_grad: device [nrhs][npix];
 * alm_grad: device [nrhs][nalm]. prec as for sht_synth_adjoint. Asynchronous. */
int sht_synth_grad(const crsht_plan *plan, int nrhs, const double *map_grad, double *alm_grad, cr_prec prec,
                   void *stream);

/* Data term of the posterior (Sect. 2.2.1, r = B a + n):
 *   chi^2(a) = (d - Y B a)^T N^-1 (d - Y B a)
 * and its gradient in the real-field inner product <a,c> = sum_l a_l0 c_l0 +
 * 2 sum_{m>0} Re(a_lm c*_lm):  g = -2 B Y^T N^-1 (d - Y B a), on the modes the
 * problem keeps (l >= lmin; 0 elsewhere), so that d chi^2 = <g, da>.
 * d: device [nrhs][npix]; a, grad: device [nrhs][nalm]; chi2: host [nrhs] or
 * NULL (ncomp = 3: the sum over T, Q, U). FP64. Blocks until done. */
int cr_grad_chi2(const crsht_plan *plan, const cr_problem *prob, int nrhs, const double *d, const double *a,
                 double *grad, double *chi2, void *stream);

/* Derivative of L = ln pi (Sect. 2.2.2, definition of pi(theta)) at the
 * spectrum of `prob`, with respect to per-bin log-amplitudes theta_k of
 * C_l -> C_l exp(theta_k) for edges[k] <= l < edges[k+1] (k < nbins), at fixed
 * w0, w1:
 *   dL/dtheta_k = 1/2 a^T S^-1_k a + 1/2 lambda^T S^-1/2_k w0 - lambda^T S^-1_k f,
 * with a the mean field, f the fluctuation and lambda = A^-1 B Y^T N^-1 Y B f
 * (one adjoint solve); X_k is X restricted to bin k. Three solves with
 * `opts`; their statistics go to stats[0..2] (host; mean field, fluctuation,
 * adjoint). d: device map; w0: device alm [nalm] or NULL; w1: device map or
 * NULL; edges: host, nbins + 1 strictly increasing values in [0, lmax + 1];
 * grad: host [nbins]; *lnpi (host) receives L. Needs nrhs_max >= 1; uses the
 * plan workspace. T+Q+U plans (ncomp = 3): d, w1 hold [3][npix], w0 [3][nalm],
 * and bin k scales the whole 3x3 block (TT, TE, EE, BB) of each l in the bin,
 * so S^-1_k, S^-1/2_k are the blocks' inverse and inverse square root scaled
 * alike. Blocks until done. */
int cr_grad_lnpi(const crsht_plan *plan, const cr_problem *prob, const double *d, const double *w0,
                 const double *w1, int nbins, const int *edges, const cr_opts *opts, double *grad,
                 double *lnpi, cr_stats *stats, void *stream);

/* Tile shapes chosen at run time by the library's autotuner. Each plan
 * starts with the default shapes; crsht_autotune measures the candidates on
 * the plan's own workspace for nrhs columns in precision prec and keeps the
 * fastest (results do not depend on the shapes: the same arithmetic per
 * element, in the same order). The choices:
 *   ring_div[k]: the ring pass (azimuthal FFTs with N^-1 fused) of FFT-length
 *     class k runs fft_len[k] / ring_div[k] threads per workgroup (8 or 4;
 *     4 only for classes of length >= 1024),
 *   f64_synth_cols, f64_adj_cols: complex columns per launch of the FP64
 *     matrix-core Legendre synthesis and adjoint (2, 4 or 8).
 * With the environment variable CRSHT_TUNE_CACHE naming a file, the choices
 * are looked up there first, keyed by device architecture, nside, lmax,
 * mmax, ncomp, nrhs and precision, and new measurements are appended.
 * Captured iteration graphs of the plan are dropped when its shapes change.
 * Synchronises the device. */
typedef struct {
  int nclasses;            /* ring FFT-length classes of the plan */
  int fft_len[8];          /* their lengths */
  int ring_div[8];         /* points per thread divisor per class (8 or 4) */
  int f64_synth_cols;      /* 2, 4 or 8 */
  int f64_adj_cols;        /* 2, 4 or 8 */
  int from_cache;          /* crsht_autotune: 1 = read from CRSHT_TUNE_CACHE, 0 = measured */
  double ms_default;       /* crsht_autotune (measured): the tuned kernels with the default shapes */
  double ms_tuned;         /* ... with the chosen shapes */
} crsht_tuning;
int crsht_autotune(crsht_plan *plan, int nrhs, cr_prec prec, crsht_tuning *out, void *stream);
/* the plan's current shapes */
int crsht_get_tuning(const crsht_plan *plan, crsht_tuning *out);
/* set shapes explicitly (validated as above; CR_EINVAL otherwise) */
int crsht_set_tuning(crsht_plan *plan, const crsht_tuning *in);

/* Per-kernel timing for measurement (not needed for computation).
 * crsht_timing_enable(plan, 1) synchronises the device, clears the counters
 * and makes the library bracket every launch of the tracked kernels with a
 * pair of HIP events on the launch stream; 0 turns it off. Tracked kernels:
 * 0 = FP64 Legendre synthesis, 1 = FP64 Legendre adjoint (incl. the
 * preconditioner diagonal pass), 2 = fused ring pass (azimuthal FFTs with
 * N^-1, FP32: the mixed operator), 3 = bf16x3 MFMA Legendre synthesis,
 * 4 = bf16x3 MFMA Legendre adjoint (bf16x6 launches are not tracked),
 * 5 = block preconditioner application,
 * 6 = fused ring pass in FP64 (the FP64 operator). Ring passes of a lone
 * synthesis or adjoint are not tracked.
 * crsht_timing_read waits for the recorded events and returns the summed
 * duration (milliseconds) and the number of launches since enabling. */
int crsht_timing_enable(const crsht_plan *plan, int on);
int crsht_timing_read(const crsht_plan *plan, int kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* CRSHT_H */
