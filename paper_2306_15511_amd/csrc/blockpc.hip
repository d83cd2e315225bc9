// Per-m block preconditioner (paper App. A; the better preconditioner that
// Sect. 4 names as the main lever on the cost of the solve).
//
// For a noise model that depends on latitude only, N^-1 in harmonic space is
// diagonal in m and S^-1 + B Y^T N^-1 Y B is one dense (l, l') matrix per m.
// For a general noise model the same matrices built from the ring sums of
// N^-1 (averaged over each ring and its mirror, so that blocks couple only
// l - l' even) form a symmetric positive definite preconditioner:
//   M_mq[i, j] = delta_ij / C_l + b_l b_l' sum_p lambda_lm(z_p) lambda_l'm(z_p) W_p,
// l = m + q + 2 i, l' = m + q + 2 j (q = parity of l - m), W_p = ring sum of
// N^-1 over both rings of pair p (the same ring weights as the Jacobi
// diagonal, whose entries are the diagonal of these blocks). Rows with
// l < lmin are the identity.
//
// T+Q+U plans hold three sets of blocks. T: as above with N_T^-1 and the TT
// entry of S^-1. E and B share one Gram matrix built from the spin-2
// functions W_lm, X_lm (the transforms' convention) and the mean of the Q and
// U ring sums W_P,p:
//   M^E_mq[i, j] = (S^-1)_EE,l delta_ij + b_l b_l' sum_p (W_lm W_l'm + X_lm X_l'm)(z_p) W_P,p,
// M^B with (S^-1)_BB. For Q and U noise equal and depending on latitude only
// these are the E-E and B-B m-blocks of the operator; the couplings left out
// are T-E (prior) and E-B (l - l' odd), so the preconditioner stays block
// diagonal per component, symmetric and positive definite.
//
// Set-up (once per noise model, beam and spectrum shape): the blocks are
// grouped into buckets of equal padded size; per bucket the FP64 factor
// L = [b_l lambda_lm(z_p) sqrt(W_p)] (T), or [b_l W_lm sqrt(W_P,p) | b_l X_lm
// sqrt(W_P,p)] (E and B, twice as many columns), is written by a recurrence
// kernel, the Gram matrix L L^T is formed with rocBLAS SYRK, the prior
// diagonal added, and the inverse computed with rocSOLVER (Cholesky, then
// inverse from the factor); the inverses are stored Jacobi-scaled, full
// symmetric, per block in FP16 (in MFMA operand tiles, see k_pc_half) where
// that provably keeps them positive definite, else in FP32 (see k_pc_store).
// Application (every PCG iteration): z_b = M_b^-1 r_b for the real and
// imaginary parts of every column and every block of every component on the
// matrix cores (FP16 products for FP16 blocks, FP32 for the others, FP32
// accumulation), one workgroup per 128 rows of both parity blocks of one m
// (one wavefront each).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "devutil.h"

namespace crsht {
namespace {

constexpr int kStartGroup = 16;   // start-table group of the Legendre recurrence
constexpr int kPcWaves = 2;       // wavefronts per application workgroup
constexpr int kPcRows = 128;     // rows of each parity block per application workgroup
constexpr int kPcCols = 16;       // right-hand sides per application pass
constexpr int kPcJ = 64;          // r rows staged per LDS tile
constexpr int kPad = 32;          // bucket granularity of the padded block size

// leading dimension (floats) of a stored inverse of n rows: 16-byte aligned rows
__host__ __device__ __forceinline__ int pc_ld(int n) { return (n + 3) & ~3; }

// L[i][p] = b_l kappa_lm mu_lm(z_p) sqrt(W_p) for the rows l = m + q + 2 i of
// block blk (0 for l < lmin); the recurrence and its start state are those of
// the transform kernels. L: [bucket block][npad][npairs], zeroed beforehand.
__global__ __launch_bounds__(256) void k_pc_lambda(int lmax, int npairs, int lmin, const double* __restrict__ pair_z,
                                                   const double* __restrict__ alpha,
                                                   const double* __restrict__ kappa, const int* __restrict__ lst_g,
                                                   const double2* __restrict__ lst_s,
                                                   const int64_t* __restrict__ mstart,
                                                   const double* __restrict__ ring_w, const double* __restrict__ bl,
                                                   const int* __restrict__ blocks, const int* __restrict__ bm,
                                                   const int* __restrict__ bq, int npad, double* __restrict__ L) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int blk = blocks[blockIdx.y];
  const int m = bm[blk], q = bq[blk];
  double* __restrict__ Lb = L + (size_t)blockIdx.y * npad * npairs;
  const double w = sqrt(ring_w[p]);
  const size_t o = (size_t)m * npairs + p;
  const int gs = lst_g[o];
  const double2 s0 = lst_s[o];
  const double z = pair_z[p];
  const int64_t base = mstart[m];
  const int nsteps = lmax - m + 1;
  double v0 = 0.0, v1 = 0.0;
  for (int st = 0; st < nsteps; ++st) {
    if (st % kStartGroup == 0 && st / kStartGroup == gs) {
      v0 = s0.x;
      v1 = s0.y;
    }
    const double mu = fma(alpha[base + st] * z, v1, -v0);
    v0 = v1;
    v1 = mu;
    if (st >= q && ((st - q) & 1) == 0) {
      const int l = m + st;
      if (l >= lmin) Lb[(size_t)((st - q) >> 1) * npairs + p] = bl[l] * kappa[base + st] * mu * w;
    }
  }
}

// E/B factor of the same blocks: L[i][p] = b_l W_lm(z_p) sqrt(W_p) and
// L[i][npairs + p] = b_l X_lm(z_p) sqrt(W_p), l = m + q + 2 i >= lmin, with
//   W_lm = (-2 ((l - m^2)/s^2 + l (l - 1)/2) lambda_l + 2 z F_lm / s^2 lambda_{l-1}) / N_l,
//   X_lm = -2 m / s^2 ((l - 1) z lambda_l - F_lm lambda_{l-1}) / N_l,
// F_lm = sqrt((2l+1)/(2l-1) (l^2 - m^2)), N_l = sqrt((l-1) l (l+1) (l+2)),
// s^2 = 1 - z^2, lambda_l = kappa_lm mu_lm from the scalar recurrence. Under
// z -> -z, W_lm and X_lm change sign with opposite parities, so within one
// block the products W W' and X X' are even and the pair sum of the ring
// weights serves both rings. L: [bucket block][npad][2 npairs], zeroed.
__global__ __launch_bounds__(256) void k_pc_spin(int lmax, int npairs, int lmin, const double* __restrict__ pair_z,
                                                 const double* __restrict__ alpha,
                                                 const double* __restrict__ kappa, const int* __restrict__ lst_g,
                                                 const double2* __restrict__ lst_s,
                                                 const int64_t* __restrict__ mstart,
                                                 const double* __restrict__ ring_w, const double* __restrict__ bl,
                                                 const int* __restrict__ blocks, const int* __restrict__ bm,
                                                 const int* __restrict__ bq, int npad, double* __restrict__ L) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int blk = blocks[blockIdx.y];
  const int m = bm[blk], q = bq[blk];
  double* __restrict__ Lb = L + (size_t)blockIdx.y * npad * 2 * npairs;
  const double w = sqrt(ring_w[p]);
  const size_t o = (size_t)m * npairs + p;
  const int gs = lst_g[o];
  const double2 s0 = lst_s[o];
  const double z = pair_z[p];
  const double is2 = 1.0 / ((1.0 - z) * (1.0 + z));
  const double mm = (double)m;
  const int64_t base = mstart[m];
  const int nsteps = lmax - m + 1;
  double v0 = 0.0, v1 = 0.0;
  for (int st = 0; st < nsteps; ++st) {
    if (st % kStartGroup == 0 && st / kStartGroup == gs) {
      v0 = s0.x;
      v1 = s0.y;
    }
    const double lprev = st > 0 ? kappa[base + st - 1] * v1 : 0.0;   // lambda_{l-1, m}
    const double mu = fma(alpha[base + st] * z, v1, -v0);
    v0 = v1;
    v1 = mu;
    if (st >= q && ((st - q) & 1) == 0) {
      const int l = m + st;
      if (l >= lmin && l >= 2) {
        const double dl = (double)l;
        const double lam = kappa[base + st] * mu;
        const double f = sqrt((2.0 * dl + 1.0) / (2.0 * dl - 1.0) * (dl * dl - mm * mm));
        const double nl = 1.0 / sqrt((dl - 1.0) * dl * (dl + 1.0) * (dl + 2.0));
        const double W = (-2.0 * ((dl - mm * mm) * is2 + 0.5 * dl * (dl - 1.0)) * lam + 2.0 * z * f * is2 * lprev) * nl;
        const double X = -2.0 * mm * is2 * ((dl - 1.0) * z * lam - f * lprev) * nl;
        const double sc = bl[l] * w;
        double* row = Lb + (size_t)((st - q) >> 1) * 2 * npairs;
        row[p] = sc * W;
        row[npairs + p] = sc * X;
      }
    }
  }
}

// After C = L L^T (lower triangle, column-major, npad x npad per block): the
// prior sinv_l[sstride l] on kept rows, the identity on rows l < lmin and on
// padding.
__global__ void k_pc_fix(const int* __restrict__ blocks, const int* __restrict__ bm, const int* __restrict__ bq,
                         const int* __restrict__ bn, int lmin, const double* __restrict__ sinv_l, int sstride,
                         int npad, double* __restrict__ C) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  const int blk = blocks[blockIdx.y];
  const int m = bm[blk], q = bq[blk], n = bn[blk];
  double* c = C + (size_t)blockIdx.y * npad * npad + (size_t)i * npad + i;
  const int l = m + q + 2 * i;
  if (i >= n || l < lmin)
    *c = 1.0;
  else
    *c += sinv_l[(size_t)sstride * l];
}

// Storage of an inverse: with S = diag(sqrt(M^-1_ii)), the Jacobi-scaled
// C = S^-1 M^-1 S^-1 has a unit diagonal and, M^-1 being positive definite,
// entries in [-1, 1]; the plan keeps S per vector element (FP32) and C per
// block, full symmetric, n rows of pc_ld(n) entries at the block's float
// offset boff, in FP32 or, where rounding to FP16 provably keeps it positive
// definite with room to spare, in FP16 (half the bytes the application
// streams on every iteration). Test of a block: with E = fl16(C) - C,
// ||E||_2 <= ||E||_F, so if fl16(C) - kHalfMargin ||E||_F I is still positive
// definite (a Cholesky factorisation of it succeeds), the smallest
// eigenvalue of C exceeds (kHalfMargin - 1) ||E||_F >= ||E||_2: the rounding
// moves every eigenvalue of the preconditioned operator by a factor within
// (1 - d, 1 + d), d = ||E||_2 / lambda_min(C) < 1 / (kHalfMargin - 1), and
// in practice (||E||_2 ~ ||E||_F / 10 for these blocks) by a few per cent.
// Low-m blocks of a masked sky, whose smallest eigenvalues of C fall to
// 1e-5 (well-measured modes), stay in FP32.
constexpr double kHalfMargin = 2.0;

// From the inverse (lower triangle from potri, npad x npad column-major per
// batch entry): the FP32 scaled block and S; the lower triangle of
// fl16(C) (padding: the identity) in T for the positivity test, and
// ||fl16(C) - C||_F^2 summed into err2 per batch entry.
__global__ void k_pc_store(const int* __restrict__ blocks, const int* __restrict__ bn,
                           const int64_t* __restrict__ boff, const int64_t* __restrict__ be0, int npad,
                           const double* __restrict__ C, float* __restrict__ inv, float* __restrict__ scale,
                           double* __restrict__ T, double* __restrict__ err2) {
  __shared__ double sh[256];
  const int blk = blocks[blockIdx.z];
  const int n = bn[blk];
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  const double* c = C + (size_t)blockIdx.z * npad * npad;
  double* t = T + (size_t)blockIdx.z * npad * npad;
  double e2 = 0.0;
  if (i < npad) {
    if (i < n && j < n) {
      const double v = i >= j ? c[(size_t)j * npad + i] : c[(size_t)i * npad + j];
      const double si = sqrt(c[(size_t)i * npad + i]), sj = sqrt(c[(size_t)j * npad + j]);
      const double cs = v / (si * sj);
      const double h = (double)(_Float16)cs;
      inv[boff[blk] + (size_t)j * pc_ld(n) + i] = (float)cs;
      if (i == j) scale[be0[blk] + 2 * (int64_t)i] = (float)si;
      if (i >= j) t[(size_t)j * npad + i] = h;
      e2 = (h - cs) * (h - cs);
    } else if (i >= j) {
      t[(size_t)j * npad + i] = i == j ? 1.0 : 0.0;
    }
  }
  e2 = block_sum(e2, sh);
  if (threadIdx.x == 0 && e2 > 0.0) atomicAdd(err2 + blockIdx.z, e2);
}

// T_ii -= kHalfMargin ||E||_F on the block's rows (not the padding)
__global__ void k_pc_shift(const int* __restrict__ blocks, const int* __restrict__ bn, int npad,
                           const double* __restrict__ err2, double* __restrict__ T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bn[blocks[blockIdx.y]]) return;
  T[(size_t)blockIdx.y * npad * npad + (size_t)i * npad + i] -= kHalfMargin * sqrt(err2[blockIdx.y]);
}

// Blocks whose test factorisation succeeded: C in FP16 in the operand order
// of v_mfma_f32_32x32x16_f16, and the per-block flag. Tiles of 32 rows x 16
// columns (1 KiB) in row-tile-major order, ceil(n/32) x ceil(n/16) per block
// from element boff16; in a tile, lane l = i % 32 + 32 ((j % 16) / 8) holds
// the 8 entries C[i][16 tj + 8 (l / 32) + e], e = 0..7, contiguously (zeros
// past n), so every operand load of a wavefront is one contiguous 1 KiB run.
__host__ __device__ __forceinline__ int pc_tiles_i(int n) { return (n + 31) / 32; }
__host__ __device__ __forceinline__ int pc_tiles_j(int n) { return (n + 15) / 16; }
__global__ void k_pc_half(const int* __restrict__ blocks, const int* __restrict__ bn,
                          const int64_t* __restrict__ boff16, int npad, const double* __restrict__ C,
                          const int* __restrict__ info, _Float16* __restrict__ inv16, int* __restrict__ bhalf) {
  const int blk = blocks[blockIdx.z];
  const int n = bn[blk], ntj = pc_tiles_j(n);
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  const bool half = info[blockIdx.z] == 0;
  if (i == 0 && j == 0) bhalf[blk] = half ? 1 : 0;
  if (!half || i >= 32 * pc_tiles_i(n) || j >= 16 * ntj) return;
  _Float16 h = (_Float16)0.0f;
  if (i < n && j < n) {
    const double* c = C + (size_t)blockIdx.z * npad * npad;
    const double v = i >= j ? c[(size_t)j * npad + i] : c[(size_t)i * npad + j];
    const double si = sqrt(c[(size_t)i * npad + i]), sj = sqrt(c[(size_t)j * npad + j]);
    h = (_Float16)(v / (si * sj));
  }
  const int lane = (i & 31) + 32 * ((j & 15) >> 3);
  inv16[boff16[blk] + (((int64_t)(i >> 5) * ntj + (j >> 4)) * 64 + lane) * 8 + (j & 7)] = h;
}

// z = M^-1 r = S C S r for the two parity blocks of one m (one component)
// and 16 right-hand sides (32 real columns) on the matrix cores. A
// workgroup takes rows [r0, r0 + 128) of both blocks: wavefront w of block
// b_w (b_0: l - m even, b_1: odd, -1 if absent). The two blocks'
// coefficients interleave in the vectors, so the workgroup stages one
// contiguous residual range for both (coalesced loads) into an LDS tile of
// kPcJ rows j per parity (FP32 S r; rows padded to 33 floats so the staging
// writes spread over the banks), and both wavefronts' results fill the same
// memory sectors close in time. Each wavefront takes the path of its block's
// storage (both pass the same barriers):
// - FP32 blocks (v_mfma_f32_32x32x2_f32): per K step (rows j, j + 1 of the
//   symmetric C) lane l of half h loads the float4 C[j + h][i0 + 4 l ..
//   i0 + 4 l + 3], so one load instruction reads two contiguous 512-byte
//   runs; component v is the A operand of the v-th of four MFMAs whose 32
//   output rows are i0 + 4 t + v (t = 0 .. 31), each with its own
//   accumulator; the loads of the next kPcPre K steps are in flight while
//   the current ones are multiplied.
// - FP16 blocks (v_mfma_f32_32x32x16_f16): per K step of 16 columns the four
//   32-row tiles of the task are four contiguous 1 KiB loads (the storage is
//   in operand order, see k_pc_half) and feed one MFMA each with the staged
//   S r as the B operand, split into two FP16 parts (hi + lo, 22 bits) after
//   scaling by a power of two per column: the running maximum of |S r| over
//   the steps seen so far sets the exponent, and the accumulators are
//   rescaled (by a power of two, exactly) whenever it grows. The products of
//   a K step take an eighth of the FP32 path's matrix-core time.
// The results are scaled by S (and the FP16 path's exponent) as they are
// written. MFMA lane layouts: 32x32x2 f32: A[i][k] in lane i + 32 k, B[k][c]
// in lane c + 32 k; 32x32x16 f16: A[i][k] in lane i + 32 (k / 8), element
// k % 8, B[k][c] in lane c + 32 (k / 8), element k % 8; both: D[i][c] in
// lane c + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4.
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
constexpr int kPcPre = 4;          // K steps per prefetch group (FP32 path)
constexpr int kPcR = 2 * kPcJ * kPcCols / (kPcWaves * 64);   // residual values staged per thread and tile
constexpr int kF16Shift = 140;     // FP16 path: S r x 2^(kF16Shift - e) < 2^14, e the biased exponent of its maximum

// one residual tile, rows [j0, j0 + kPcJ) of both parities: consecutive
// threads read consecutive coefficients, in batches of kStage to bound the
// registers held by loads in flight; the loads carry no per-lane condition
// (elements outside the blocks or columns read element e00 of column c0 and
// are zeroed by their scale factor), so each batch's loads are in flight
// together
__device__ __forceinline__ void pc_stage(float (*rs)[kPcJ][33], int j0, int c0, int nc, int n0, int n1,
                                         int64_t vlen, int64_t e00, const double2* __restrict__ r,
                                         const float* __restrict__ scale) {
  constexpr int kStage = 4;
  static_assert(kPcR % kStage == 0, "whole staging batches");
#pragma unroll 1
  for (int k0 = 0; k0 < kPcR; k0 += kStage) {
    double2 v[kStage];
    float sv[kStage];
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int e = threadIdx.x + (k0 + k) * kPcWaves * 64;
      const int ee = e % (2 * kPcJ), cc = e / (2 * kPcJ);
      const int q = ee & 1, j = j0 + (ee >> 1);
      const bool in = cc < nc && j < (q ? n1 : n0);
      const int64_t el = in ? e00 + 2 * j0 + ee : e00;
      v[k] = r[(int64_t)(c0 + (in ? cc : 0)) * vlen + el];
      sv[k] = scale[el];
      sv[k] = in ? sv[k] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int e = threadIdx.x + (k0 + k) * kPcWaves * 64;
      const int ee = e % (2 * kPcJ), cc = e / (2 * kPcJ);
      const int q = ee & 1, jj = ee >> 1;
      rs[q][jj][2 * cc] = (float)(v[k].x * sv[k]);
      rs[q][jj][2 * cc + 1] = (float)(v[k].y * sv[k]);
    }
  }
}

// results through LDS (the rs tile, free after the last products), 8
// columns at a time, then written as whole rows of both parities (the
// task's 256 interleaved coefficients of a column are contiguous); fill(stage,
// h) writes this wavefront's results of columns h .. h + 7 as
// stage[column - h][2 (row - i0) + w][re, im]. With part, the per-task
// partials of <r, z>.
template <class Fill, class Z>
__device__ __forceinline__ void pc_output(Fill&& fill, float (*rs)[kPcJ][33], int c0, int nc, int n0, int n1, int i0,
                                          int64_t vlen, int64_t e00, const float* __restrict__ scale,
                                          const double2* __restrict__ r, Z* __restrict__ z,
                                          double* __restrict__ part, int pstride, double wt, double* red, int w,
                                          int lane) {
  float* stage = &rs[0][0][0];   // [8 columns][256 coefficients][re, im]
#pragma unroll 1
  for (int h = 0; h < kPcCols; h += 8) {
    __syncthreads();   // the products (or the previous half's writes) have read the tile
    fill(stage, h);
    __syncthreads();
    // this thread's coefficients are the same for every column: their
    // scales are read once, without per-lane conditions
    constexpr int kOut = 8 * 256 / (kPcWaves * 64);
    float so[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int er = (threadIdx.x + t * kPcWaves * 64) & 255, q = er & 1, row = i0 + (er >> 1);
      so[t] = scale[row < (q ? n1 : n0) ? e00 + 2 * i0 + er : e00];
    }
    // thread t writes coefficients t and t + 128 of columns h .. h + 7;
    // with part, it also sums their terms of <r, z> per column (r loaded
    // in batches, without per-lane conditions)
    double rzp[8];
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) rzp[cc] = 0.0;
    constexpr int kOb = 2;
#pragma unroll
    for (int k0 = 0; k0 < kOut; k0 += kOb) {
      double2 rv[kOb];
      if (part) {
#pragma unroll
        for (int k = 0; k < kOb; ++k) {
          const int idx = threadIdx.x + (k0 + k) * kPcWaves * 64;
          const int cc = idx >> 8, er = idx & 255;
          const int c = h + cc, q = er & 1, row = i0 + (er >> 1);
          const bool in = c < nc && row < (q ? n1 : n0);
          rv[k] = r[(int64_t)(c0 + (in ? c : 0)) * vlen + (in ? e00 + 2 * i0 + er : e00)];
        }
      }
#pragma unroll
      for (int k = 0; k < kOb; ++k) {
        const int idx = threadIdx.x + (k0 + k) * kPcWaves * 64;
        const int cc = idx >> 8, er = idx & 255;
        const int c = h + cc, q = er & 1, row = i0 + (er >> 1);
        if (c < nc && row < (q ? n1 : n0)) {
          const float* v = stage + idx * 2;
          const double sr = (double)so[k & 1];
          const double2 zv = zstore(z + (int64_t)(c0 + c) * vlen + e00 + 2 * i0 + er,
                                    make_double2(sr * (double)v[0], sr * (double)v[1]));
          if (part) rzp[(k0 + k) >> 1] += fma(rv[k].x, zv.x, rv[k].y * zv.y);
        }
      }
    }
    if (part) {
      // per column: sum over the wavefront (fixed butterfly order), then
      // over the two wavefronts; weight 1 for m = 0, 2 otherwise
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        double v = rzp[cc];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        rzp[cc] = v;
      }
      if (lane == 0) {
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) red[w * 8 + cc] = rzp[cc];
      }
      __syncthreads();
      if (threadIdx.x < 8 && h + (int)threadIdx.x < nc)
        part[(int64_t)(c0 + h + threadIdx.x) * pstride + blockIdx.x] = wt * (red[threadIdx.x] + red[8 + threadIdx.x]);
    }
  }
}

// FP32 path of one wavefront: rows [i0, i0 + 128) of its block. Loads
// without per-lane conditions (a branch around each load defeats the overlap
// of the next group's loads with this group's products): rows j >= n read
// row n - 1 and lanes past the padded row width read columns 0 .. 3, all
// finite entries whose products meet zero B operands (rows j >= n of the
// staged tile) or land in output rows never written.
template <class Z>
__device__ __forceinline__ void pc_apply_wave32(const float* __restrict__ Ab, int nrhs, int64_t vlen,
                                                const float* __restrict__ scale, const double2* __restrict__ r,
                                                Z* __restrict__ z, float (*rs)[kPcJ][33], int w, int il,
                                                int kk, int n, int n0, int n1, int ld, int i0, int64_t e00,
                                                double* __restrict__ part, int pstride, double wt, double* red) {
  const int lane = threadIdx.x & 63;
  constexpr int kSteps = kPcJ / 2;   // K steps per LDS tile
  constexpr int kGpt = kSteps / kPcPre;
  const int ntile = (n0 + kPcJ - 1) / kPcJ;
  for (int c0 = 0; c0 < nrhs; c0 += kPcCols) {
    const int nc = min(kPcCols, nrhs - c0);
    f32x16_t acc0 = {}, acc1 = {}, acc2 = {}, acc3 = {};
    // groups of kPcPre K steps over all j; a new LDS tile every kGpt groups;
    // the A operands of group G + 1 are requested before the products of G
    const int ngrp = ntile * kGpt;
    f32x4_t an[kPcPre] = {};
    auto fetch = [&](int G) {
      if (i0 >= n) return;   // wavefront-uniform: no rows of this block here
      const int jg = 2 * G * kPcPre + kk;
#pragma unroll
      for (int u = 0; u < kPcPre; ++u) {
        const int j = min(jg + 2 * u, n - 1);
        an[u] = *reinterpret_cast<const f32x4_t*>(Ab + (size_t)j * ld);
      }
    };
    fetch(0);
#pragma unroll 1
    for (int G = 0; G < ngrp; ++G) {
      const int g0 = G % kGpt;
      if (g0 == 0) {
        __syncthreads();   // previous tile's products have read rs
        pc_stage(rs, (G / kGpt) * kPcJ, c0, nc, n0, n1, vlen, e00, r, scale);
        __syncthreads();
      }
      f32x4_t ac[kPcPre];
#pragma unroll
      for (int u = 0; u < kPcPre; ++u) ac[u] = an[u];
      if (G + 1 < ngrp) fetch(G + 1);
      if (i0 < n) {
#pragma unroll
        for (int u = 0; u < kPcPre; ++u) {
          const float bval = rs[w][2 * (g0 * kPcPre + u) + kk][il];
          acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ac[u][0], bval, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ac[u][1], bval, acc1, 0, 0, 0);
          acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ac[u][2], bval, acc2, 0, 0, 0);
          acc3 = __builtin_amdgcn_mfma_f32_32x32x2f32(ac[u][3], bval, acc3, 0, 0, 0);
        }
      }
    }
    const int rhs = il >> 1, comp = il & 1;
    pc_output(
        [&](float* stage, int h) {
          if (i0 < n && rhs >= h && rhs < h + 8) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const f32x16_t a = v == 0 ? acc0 : v == 1 ? acc1 : v == 2 ? acc2 : acc3;
#pragma unroll
              for (int q = 0; q < 16; ++q) {
                // row i of accumulator v is i0 + 4 i + v, i = 8 (q / 4) + 4 kk + q % 4
                const int ro = 4 * (8 * (q / 4) + 4 * kk + (q % 4)) + v;
                stage[((rhs - h) * 256 + 2 * ro + w) * 2 + comp] = a[q];
              }
            }
          }
        },
        rs, c0, nc, n0, n1, i0, vlen, e00, scale, r, z, part, pstride, wt, red, w, lane);
  }
}

// FP16 path of one wavefront: rows [i0, i0 + 128) of its block, i.e. the
// four row tiles i0 / 32 .. i0 / 32 + 3 (clamped to the block's last tile;
// rows past the block are never written). At: the block's first tile of row
// tile i0 / 32, plus this lane's 8 entries. Steps past the block's last
// column tile read that tile again and meet zero B operands.
template <class Z>
__device__ __forceinline__ void pc_apply_wave16(const _Float16* __restrict__ At, int ntj, int ntr, int nrhs,
                                                int64_t vlen, const float* __restrict__ scale,
                                                const double2* __restrict__ r, Z* __restrict__ z,
                                                float (*rs)[kPcJ][33], int w, int il, int kk, int n, int n0,
                                                int n1, int i0, int64_t e00, double* __restrict__ part,
                                                int pstride, double wt, double* red) {
  const int lane = threadIdx.x & 63;
  constexpr int kSpt = kPcJ / 16;   // K steps of 16 columns per LDS tile
  const int nst = ((n0 + kPcJ - 1) / kPcJ) * kSpt;
  for (int c0 = 0; c0 < nrhs; c0 += kPcCols) {
    const int nc = min(kPcCols, nrhs - c0);
    f32x16_t acc[4] = {};
    int eb = 0;   // biased exponent of the running max of |S r| of this lane's column
    f16x8_t an[4] = {};
    auto fetch = [&](int st) {
      if (i0 >= n) return;   // wavefront-uniform: no rows of this block here
      const int tj = min(st, ntj - 1);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        an[t] = *reinterpret_cast<const f16x8_t*>(At + ((size_t)min(t, ntr - 1) * ntj + tj) * 512);
    };
    fetch(0);
#pragma unroll 1
    for (int st = 0; st < nst; ++st) {
      const int s0 = st % kSpt;
      if (s0 == 0) {
        __syncthreads();   // previous tile's products have read rs
        pc_stage(rs, (st / kSpt) * kPcJ, c0, nc, n0, n1, vlen, e00, r, scale);
        __syncthreads();
      }
      f16x8_t ac[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) ac[t] = an[t];
      if (st + 1 < nst) fetch(st + 1);
      if (i0 < n) {
        // B operand: column il of S r at rows 16 s0 + 8 kk + e, e = 0..7
        float v[8];
        float mx = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          v[e] = rs[w][16 * s0 + 8 * kk + e][il];
          mx = fmaxf(mx, fabsf(v[e]));
        }
        mx = fmaxf(mx, __shfl_xor(mx, 32));   // lanes il and il + 32 hold the same column
        const int ebn = (__float_as_int(mx) >> 23) & 0xff;
        if (ebn > eb) {
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[t][q] = ldexpf(acc[t][q], eb - ebn);
          eb = ebn;
        }
        f16x8_t bh, bl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float y = ldexpf(v[e], kF16Shift - eb);
          const _Float16 hi = (_Float16)y;
          bh[e] = hi;
          bl[e] = (_Float16)(y - (float)hi);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ac[t], bh, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ac[t], bl, acc[t], 0, 0, 0);
        }
      }
    }
    const int rhs = il >> 1, comp = il & 1;
    pc_output(
        [&](float* stage, int h) {
          if (i0 < n && rhs >= h && rhs < h + 8) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
              for (int q = 0; q < 16; ++q) {
                // row i of tile t is i0 + 32 t + i, i = 8 (q / 4) + 4 kk + q % 4
                const int ro = 32 * t + 8 * (q / 4) + 4 * kk + (q % 4);
                stage[((rhs - h) * 256 + 2 * ro + w) * 2 + comp] = ldexpf(acc[t][q], eb - kF16Shift);
              }
          }
        },
        rs, c0, nc, n0, n1, i0, vlen, e00, scale, r, z, part, pstride, wt, red, w, lane);
  }
}

// (three wavefronts per SIMD: more loads in flight per CU)
template <class Z>
__global__ __launch_bounds__(kPcWaves * 64) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_pc_apply(
    int nrhs, int64_t vlen, const int64_t* __restrict__ be0, const int* __restrict__ task_b,
    const int* __restrict__ task_b1, const int* __restrict__ task_r0, const int* __restrict__ bn,
    const int64_t* __restrict__ boff, const int* __restrict__ bhalf, const float* __restrict__ inv,
    const int64_t* __restrict__ boff16, const _Float16* __restrict__ inv16, const float* __restrict__ scale,
    const int* __restrict__ bm, const double2* __restrict__ r, Z* __restrict__ z,
    double* __restrict__ part, int pstride, const int* __restrict__ pred) {
  if (pred && *pred) return;
  static_assert((kPcJ / 2) % kPcPre == 0, "tile must hold whole prefetch groups");
  static_assert(kPcJ % 16 == 0, "tile must hold whole 16-column steps");
  static_assert(kPcWaves == 2, "one wavefront per parity block");
  __shared__ float rs[2][kPcJ][33];
  __shared__ double red[2 * 8];
  const int b0 = task_b[blockIdx.x];
  if (b0 < 0) {   // padding task (uniform per workgroup, before any barrier): zero partials
    if (part)
      for (int c = threadIdx.x; c < nrhs; c += blockDim.x) part[(int64_t)c * pstride + blockIdx.x] = 0.0;
    return;
  }
  const int b1 = task_b1[blockIdx.x];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = w == 0 ? b0 : b1;
  const int n0 = bn[b0];                                    // the even block is the larger one
  const int n1 = b1 >= 0 ? bn[b1] : 0;
  const int n = w == 0 ? n0 : n1;
  const int il = lane & 31, kk = lane >> 5;
  const int i0 = task_r0[blockIdx.x];
  const int64_t e00 = be0[b0];                              // element of row j of block q: e00 + q + 2 j
  const double wt = bm[b0] == 0 ? 1.0 : 2.0;               // real-field inner product weight of m
  if (b >= 0 && bhalf[b]) {
    const int ntj = pc_tiles_j(n);
    const int ntr = pc_tiles_i(n) - i0 / 32;               // row tiles of this task in the block (>= 1)
    pc_apply_wave16(inv16 + boff16[b] + (size_t)(i0 / 32) * ntj * 512 + lane * 8, ntj, ntr, nrhs, vlen, scale, r,
                    z, rs, w, il, kk, n, n0, n1, i0, e00, part, pstride, wt, red);
  } else {
    const int ld = pc_ld(n);
    const int ic = i0 + 4 * il;                             // first of this lane's 4 rows
    const bool colok = ic < ld;                             // padding columns n .. ld - 1 hold zeros
    pc_apply_wave32(inv + (b >= 0 ? boff[b] : 0) + (colok ? ic : 0), nrhs, vlen, scale, r, z, rs, w, il, kk, n,
                    n0, n1, ld, i0, e00, part, pstride, wt, red);
  }
}

// partial <r, z> (row 0) and, with rr, <r, r> (row 1) per column
template <class Z>
__global__ void k_pc_dots(int64_t vlen, const int* __restrict__ idx_m, const double2* __restrict__ r,
                          const Z* __restrict__ z, int rr, double* __restrict__ partial, int npart,
                          const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ double sh[256];
  const int c = blockIdx.y;
  double rz = 0.0, r2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < vlen; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ci = c * vlen + i;
    const int m = idx_m[i];
    const double2 rv = r[ci];
    rz += wdot(m, rv, zload(z + ci));
    if (rr) r2 += wdot(m, rv, rv);
  }
  rz = block_sum(rz, sh);
  if (rr) r2 = block_sum(r2, sh);
  if (threadIdx.x == 0) {
    double* pa = partial + (size_t)c * npart * 4;
    pa[blockIdx.x] = rz;
    if (rr) pa[npart + blockIdx.x] = r2;
  }
}

template <typename T>
int dev_alloc(T** p, size_t n) {
  *p = nullptr;
  if (hipMalloc((void**)p, (n ? n : 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return CR_ENOMEM;
  }
  return CR_OK;
}

template <typename T>
int dev_upload(T** p, const std::vector<T>& h) {
  int rc = dev_alloc(p, h.size());
  if (rc) return rc;
  return hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess ? CR_OK : CR_EDEVICE;
}

}  // namespace

void block_pc_free(BlockPC& pc) {
  void* ptrs[] = {pc.inv, pc.inv16, pc.boff16, pc.scale, pc.bhalf, pc.part, pc.bm, pc.bq, pc.bn, pc.boff, pc.be0,
                  pc.task_b, pc.task_b1, pc.task_r0};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  pc = BlockPC();
}

int block_pc_build(crsht_plan* P, int lmin, const double* ninv, hipStream_t s) {
  const Geometry& g = P->g;
  const int lmax = g.lmax, mmax = g.mmax, np = g.npairs;
  const int ncomp = P->ncomp;
  BlockPC& pc = P->pc;
  // a captured iteration block holds the old preconditioner's device
  // addresses (inverses, tasks): drop it before they are freed, so that the
  // next solve captures again with the new storage
  if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
  P->graph_exec = nullptr;
  P->graph_key = GraphKey();
  for (auto& gx : P->dgraph) {
    if (gx) (void)hipGraphExecDestroy(gx);
    gx = nullptr;
  }
  P->dgraph_key = GraphKey();
  block_pc_free(pc);
  // blocks (component, m, parity), component-major: sizes, vector element of
  // row 0, compact FP32 offsets; then the application tasks
  std::vector<int> bm, bq, bn;
  std::vector<int64_t> boff, be0, boff16;
  int64_t off = 0, off16 = 0;
  for (int k = 0; k < ncomp; ++k) {
    int64_t mst = 0;   // first element of m (m-major storage, l = m .. lmax)
    for (int m = 0; m <= mmax; ++m) {
      for (int qq = 0; qq < 2; ++qq) {
        if (m + qq > lmax) continue;
        const int n = (lmax - m - qq) / 2 + 1;
        bm.push_back(m);
        bq.push_back(qq);
        bn.push_back(n);
        be0.push_back((int64_t)k * g.nalm + mst + qq);
        boff.push_back(off);
        off += (int64_t)n * pc_ld(n);
        boff16.push_back(off16);
        off16 += (int64_t)512 * pc_tiles_i(n) * pc_tiles_j(n);
      }
      mst += lmax - m + 1;
    }
  }
  const int nb = (int)bm.size();
  const int nbc = nb / ncomp;   // blocks per component; block b of component k is k nbc + b
  // Application tasks (even block, odd block or -1, first row): one
  // workgroup per 128 rows of both parity blocks of one (component, m),
  // dealt to the 8 XCDs (workgroup i runs on XCD i mod 8) so that the tasks
  // of one m share the residual lines they read and the result lines they
  // write in that XCD's L2; units are placed largest first on the least
  // loaded XCD, and within an XCD run largest first. Short XCD lists are
  // padded with empty tasks (block -1).
  constexpr int kXcd = 8;
  struct Unit {
    double cost;
    int b0, b1;
  };
  std::vector<Unit> units;
  for (int b = 0; b < nb; ++b)
    if (bq[b] == 0) {
      const int b1 = (b + 1 < nb && bq[b + 1] == 1 && bm[b + 1] == bm[b]) ? b + 1 : -1;
      double cost = (double)bn[b] * bn[b];
      if (b1 >= 0) cost += (double)bn[b1] * bn[b1];
      units.push_back({cost, b, b1});
    }
  std::stable_sort(units.begin(), units.end(), [](const Unit& x, const Unit& y) { return x.cost > y.cost; });
  std::vector<std::vector<int>> xb(kXcd), xb1(kXcd), xr(kXcd);
  std::vector<double> load(kXcd, 0.0);
  for (const Unit& u : units) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[x] += u.cost;
    for (int r0 = 0; r0 < bn[u.b0]; r0 += kPcRows) {   // the even block has the most rows
      xb[x].push_back(u.b0);
      xb1[x].push_back(u.b1);
      xr[x].push_back(r0);
    }
  }
  size_t per = 0;
  for (int x = 0; x < kXcd; ++x) per = std::max(per, xb[x].size());
  std::vector<int> tb(per * kXcd, -1), tb1(per * kXcd, -1), tr(per * kXcd, 0);
  for (int x = 0; x < kXcd; ++x)
    for (size_t k = 0; k < xb[x].size(); ++k) {
      tb[k * kXcd + x] = xb[x][k];
      tb1[k * kXcd + x] = xb1[x][k];
      tr[k * kXcd + x] = xr[x][k];
    }
  int rc;
  if ((rc = dev_upload(&pc.bm, bm)) || (rc = dev_upload(&pc.bq, bq)) || (rc = dev_upload(&pc.bn, bn)) ||
      (rc = dev_upload(&pc.boff, boff)) || (rc = dev_upload(&pc.be0, be0)) || (rc = dev_upload(&pc.task_b, tb)) || (rc = dev_upload(&pc.task_b1, tb1)) ||
      (rc = dev_upload(&pc.task_r0, tr)) || (rc = dev_alloc(&pc.inv, (size_t)off)) ||
      (rc = dev_upload(&pc.boff16, boff16)) || (rc = dev_alloc(&pc.inv16, (size_t)off16)) ||
      (rc = dev_alloc(&pc.scale, (size_t)ncomp * g.nalm)) || (rc = dev_alloc(&pc.bhalf, (size_t)nb)) ||
      (rc = dev_alloc(&pc.part, (size_t)P->nrhs_max * tb.size()))) {
    block_pc_free(pc);
    return rc;
  }
  pc.nblocks = nb;
  pc.ntasks = (int)tb.size();
  pc.inv_elems = off;
  // padding columns n .. ld - 1 of every row stay zero (read by the application kernel)
  if (hipMemsetAsync(pc.inv, 0, (size_t)off * sizeof(float), s) != hipSuccess ||
      hipMemsetAsync(pc.bhalf, 0, (size_t)nb * sizeof(int), s) != hipSuccess) {
    block_pc_free(pc);
    return CR_EDEVICE;
  }

  // per-l inputs left on the device by the problem set-up: b_l (row 2 of
  // perl) and the priors (perl row 0 = 1/C_l; T+Q+U: sblk entries TT, EE, BB)
  const double* dbl = P->w.perl + 2 * (lmax + 1);
  double *L = nullptr, *C = nullptr, *T = nullptr, *err2 = nullptr;
  int *dblocks = nullptr, *dinfo = nullptr, *dinfo2 = nullptr;
  rocblas_handle h = nullptr;
  auto cleanup = [&]() {
    if (h) (void)rocblas_destroy_handle(h);
    void* ptrs[] = {L, C, T, err2, dblocks, dinfo, dinfo2};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
  };
  // buckets of equal padded size (per component set), processed in batches
  // bounded by memory; E and B batches hold cnt E blocks then cnt B blocks
  std::vector<std::vector<int>> buckets((lmax + 2) / kPad + 2);
  for (int b = 0; b < nbc; ++b) buckets[(bn[b] + kPad - 1) / kPad].push_back(b);
  const size_t budget = (size_t)1 << 29;   // bytes of L per batch
  const int kmax = ncomp == 3 ? 2 : 1;     // columns of L per ring pair (E/B: W and X)
  size_t maxL = 0, maxC = 0, maxb = 0;
  for (size_t k = 0; k < buckets.size(); ++k) {
    if (buckets[k].empty()) continue;
    const size_t npad = k * kPad;
    const size_t per = std::max<size_t>(1, budget / (npad * np * kmax * sizeof(double)));
    const size_t cnt = std::min(per, buckets[k].size());
    maxL = std::max(maxL, cnt * npad * np * kmax);
    maxC = std::max(maxC, cnt * npad * npad * kmax);
    maxb = std::max(maxb, cnt * kmax);
  }
  if ((rc = dev_alloc(&L, maxL)) || (rc = dev_alloc(&C, maxC)) || (rc = dev_alloc(&T, maxC)) ||
      (rc = dev_alloc(&err2, maxb)) || (rc = dev_alloc(&dblocks, maxb)) || (rc = dev_alloc(&dinfo, maxb)) ||
      (rc = dev_alloc(&dinfo2, maxb))) {
    cleanup();
    block_pc_free(pc);
    return rc;
  }
  if (rocblas_create_handle(&h) != rocblas_status_success || rocblas_set_stream(h, s) != rocblas_status_success) {
    cleanup();
    block_pc_free(pc);
    return CR_EDEVICE;
  }
  int status = CR_OK;
  std::vector<int> hinfo;
  // pass 0: T (or the only component) with the ring sums of N^-1 (N_T^-1);
  // pass 1 (T+Q+U): E and B with the mean of the Q and U ring sums
  for (int pass = 0; pass < (ncomp == 3 ? 2 : 1) && status == CR_OK; ++pass) {
    const bool spin = pass == 1;
    const int kc = spin ? 2 : 1;   // L columns per pair
    const int nset = spin ? 2 : 1;  // block sets sharing one Gram matrix (E, B)
    const hipError_t we = spin ? launch_ring_weights(P, ninv + g.npix, P->w.ring_w, s, ninv + 2 * g.npix, 0.5)
                               : launch_ring_weights(P, ninv, P->w.ring_w, s);
    if (we != hipSuccess) {
      status = CR_EDEVICE;
      break;
    }
    for (size_t k = 0; k < buckets.size() && status == CR_OK; ++k) {
      if (buckets[k].empty()) continue;   // (k = 0 is always empty: every block has n >= 1)
      const int npad = (int)k * kPad;
      const std::vector<int>& bl_k = buckets[k];
      const size_t per = std::max<size_t>(1, budget / ((size_t)npad * np * kmax * sizeof(double)));
      for (size_t a = 0; a < bl_k.size() && status == CR_OK; a += per) {
        const int cnt = (int)std::min(per, bl_k.size() - a);
        // global block ids: T pass k = 0; spin pass E (k = 1) then B (k = 2)
        std::vector<int> ids;
        for (int set = 0; set < nset; ++set)
          for (int t = 0; t < cnt; ++t) ids.push_back((spin ? 1 + set : 0) * nbc + bl_k[a + t]);
        const size_t lsz = (size_t)npad * np * kc, csz = (size_t)npad * npad;
        bool ok = hipMemcpyAsync(dblocks, ids.data(), ids.size() * sizeof(int), hipMemcpyHostToDevice, s) ==
                  hipSuccess;
        ok = ok && hipMemsetAsync(L, 0, (size_t)cnt * lsz * sizeof(double), s) == hipSuccess;
        if (ok) {
          if (spin)
            hipLaunchKernelGGL(k_pc_spin, dim3((np + 255) / 256, cnt), dim3(256), 0, s, lmax, np, lmin, P->t.pair_z,
                               P->t.rec_alpha, P->t.rec_kappa, P->t.lst_g, P->t.lst_s, P->t.mstart, P->w.ring_w, dbl,
                               dblocks, pc.bm, pc.bq, npad, L);
          else
            hipLaunchKernelGGL(k_pc_lambda, dim3((np + 255) / 256, cnt), dim3(256), 0, s, lmax, np, lmin,
                               P->t.pair_z, P->t.rec_alpha, P->t.rec_kappa, P->t.lst_g, P->t.lst_s, P->t.mstart,
                               P->w.ring_w, dbl, dblocks, pc.bm, pc.bq, npad, L);
          ok = hipGetLastError() == hipSuccess;
        }
        const double one = 1.0, zero = 0.0;
        // C = L L^T: L is row-major [npad][kc np], i.e. column-major (kc np) x npad, so C = A^T A
        const int kdim = kc * np;
        ok = ok && rocblas_dsyrk_strided_batched(h, rocblas_fill_lower, rocblas_operation_transpose, npad, kdim, &one,
                                                 L, kdim, (rocblas_stride)lsz, &zero, C, npad,
                                                 (rocblas_stride)csz, cnt) == rocblas_status_success;
        // the B blocks start from the same Gram matrices
        if (spin)
          ok = ok && hipMemcpyAsync(C + (size_t)cnt * csz, C, (size_t)cnt * csz * sizeof(double),
                                    hipMemcpyDeviceToDevice, s) == hipSuccess;
        for (int set = 0; set < nset && ok; ++set) {
          // prior: perl row 0 (temperature plans) or the sblk entry TT (0), EE (2), BB (3)
          const double* prior = ncomp == 3 ? P->w.sblk + (spin ? 2 + set : 0) : P->w.perl;
          hipLaunchKernelGGL(k_pc_fix, dim3((npad + 255) / 256, cnt), dim3(256), 0, s, dblocks + set * cnt, pc.bm,
                             pc.bq, pc.bn, lmin, prior, ncomp == 3 ? 8 : 1, npad, C + (size_t)set * cnt * csz);
          ok = hipGetLastError() == hipSuccess;
        }
        const int nbat = nset * cnt;
        ok = ok && rocsolver_dpotrf_strided_batched(h, rocblas_fill_lower, npad, C, npad, (rocblas_stride)csz, dinfo,
                                                    nbat) == rocblas_status_success;
        hinfo.assign(nbat, 0);
        ok = ok && hipMemcpyAsync(hinfo.data(), dinfo, nbat * sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess &&
             hipStreamSynchronize(s) == hipSuccess;
        if (!ok) {
          status = CR_EDEVICE;
          break;
        }
        for (int v : hinfo)
          if (v != 0) status = CR_EINVAL;   // a block is not positive definite
        if (status != CR_OK) break;
        ok = rocsolver_dpotri_strided_batched(h, rocblas_fill_lower, npad, C, npad, (rocblas_stride)csz, dinfo,
                                              nbat) == rocblas_status_success;
        // FP32 scaled storage, then the FP16 test (a Cholesky factorisation of
        // fl16(C) - kHalfMargin ||E||_F I) and FP16 storage where it succeeds
        ok = ok && hipMemsetAsync(err2, 0, (size_t)nbat * sizeof(double), s) == hipSuccess;
        if (ok) {
          hipLaunchKernelGGL(k_pc_store, dim3((npad + 255) / 256, npad, nbat), dim3(256), 0, s, dblocks, pc.bn,
                             pc.boff, pc.be0, npad, C, pc.inv, pc.scale, T, err2);
          hipLaunchKernelGGL(k_pc_shift, dim3((npad + 255) / 256, nbat), dim3(256), 0, s, dblocks, pc.bn, npad,
                             err2, T);
          ok = hipGetLastError() == hipSuccess;
        }
        ok = ok && rocsolver_dpotrf_strided_batched(h, rocblas_fill_lower, npad, T, npad, (rocblas_stride)csz,
                                                    dinfo2, nbat) == rocblas_status_success;
        if (ok) {
          hipLaunchKernelGGL(k_pc_half, dim3((npad + 255) / 256, npad, nbat), dim3(256), 0, s, dblocks, pc.bn,
                             pc.boff16, npad, C, dinfo2, pc.inv16, pc.bhalf);
          ok = hipGetLastError() == hipSuccess;
        }
        ok = ok && hipStreamSynchronize(s) == hipSuccess;   // scratch is reused by the next batch
        if (!ok) status = CR_EDEVICE;
      }
    }
  }
  cleanup();
  if (status != CR_OK) {
    block_pc_free(pc);
    return status;
  }
  // bytes of the n x n entries of the stored inverses (one application reads each once)
  std::vector<int> hh(nb);
  if (hipMemcpy(hh.data(), pc.bhalf, nb * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
    block_pc_free(pc);
    return CR_EDEVICE;
  }
  pc.stored_bytes = 0;
  pc.nhalf = 0;
  for (int b = 0; b < nb; ++b) {
    pc.stored_bytes += (int64_t)bn[b] * bn[b] * (hh[b] ? 2 : 4);
    pc.nhalf += hh[b] ? 1 : 0;
  }
  pc.built = true;
  pc.lmin = lmin;
  return CR_OK;
}

hipError_t launch_pc_apply(const crsht_plan* P, int nrhs, const double2* r, double2* z, hipStream_t s, bool dots,
                           bool z32) {
  const BlockPC& pc = P->pc;
  timing_begin(P, 5, s);
  if (z32)
    hipLaunchKernelGGL(k_pc_apply<float2>, dim3(pc.ntasks), dim3(kPcWaves * 64), 0, s, nrhs, vlen(P), pc.be0,
                       pc.task_b, pc.task_b1, pc.task_r0, pc.bn, pc.boff, pc.bhalf, pc.inv, pc.boff16, pc.inv16,
                       pc.scale, pc.bm, r, reinterpret_cast<float2*>(z), dots ? pc.part : nullptr, pc.ntasks,
                       P->pred);
  else
    hipLaunchKernelGGL(k_pc_apply<double2>, dim3(pc.ntasks), dim3(kPcWaves * 64), 0, s, nrhs, vlen(P), pc.be0,
                       pc.task_b, pc.task_b1, pc.task_r0, pc.bn, pc.boff, pc.bhalf, pc.inv, pc.boff16, pc.inv16,
                       pc.scale, pc.bm, r, z, dots ? pc.part : nullptr, pc.ntasks, P->pred);
  timing_end(P, 5, s);
  return hipGetLastError();
}

hipError_t launch_pc_dots(const crsht_plan* P, int nrhs, const double2* r, const double2* z, bool rr,
                          hipStream_t s, bool z32) {
  const int nb = vec_reduce_blocks(P);
  if (z32)
    hipLaunchKernelGGL(k_pc_dots<float2>, dim3(nb, nrhs), dim3(256), 0, s, vlen(P), P->t.idx_mv, r,
                       reinterpret_cast<const float2*>(z), rr ? 1 : 0, P->w.partial, P->w.npart, P->pred);
  else
    hipLaunchKernelGGL(k_pc_dots<double2>, dim3(nb, nrhs), dim3(256), 0, s, vlen(P), P->t.idx_mv, r, z, rr ? 1 : 0,
                       P->w.partial, P->w.npart, P->pred);
  return hipGetLastError();
}

}  // namespace crsht
