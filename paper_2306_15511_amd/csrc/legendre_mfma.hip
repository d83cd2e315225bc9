// Mixed-precision Legendre step on the matrix cores (gfx950 MFMA).
//
// For one m the Legendre sums are small dense products:
//   synthesis  F[pair, col] = sum_l mu_lm(z_pair) A[l, col]
//   adjoint    R[l, col]    = sum_pair mu_lm(z_pair) G[pair, col]
// with col = 2 * rhs + (re, im). mu_lm comes from the FP64 recurrence
// (unchanged: same start tables, same arithmetic as the FP64 kernels); it is
// rounded to float and split into bf16 hi + lo parts, and so are the a_lm / G
// operands, and each product is evaluated as hi*hi + hi*lo + lo*hi on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation ("bf16x3"; relative error
// about 2^-16 per product). Even and odd l - m are separate K slices, as in
// the FP64 kernels (north/south parity).
//
// MFMA 32x32x16 bf16 lane layout (checked on the device): A[i][k] in lane
// i + 32 (k / 8), element k % 8; B[k][j] in lane j + 32 (k / 8), element k % 8;
// D[i][j] in lane j + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4.
#include <algorithm>

#include "internal.h"

namespace crsht {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kNever = 0x7fffffff;
constexpr int kGroup = kStartGroup;   // start-table group (steps)
constexpr int kSynChunk = 32;   // steps per synthesis K chunk (16 even + 16 odd)
constexpr int kAdjTile = 64;    // steps per adjoint output tile (32 even + 32 odd)
constexpr int kAdjWaves = 4;

// Blocks are dealt to the 8 XCDs round-robin by linear block index. The m of
// the j-th m-slot of an XCD: each XCD takes 4 consecutive m out of every 32,
// which balances long and short m over the XCDs and keeps neighbouring m (and
// all ring-pair blocks of one m) in one L2.
__host__ __device__ __forceinline__ int xcd_m(int j, int xcd) { return (j >> 2) * 32 + xcd * 4 + (j & 3); }
__host__ __device__ __forceinline__ int m_xcd(int m) { return (m & 31) >> 2; }

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

// double -> float, kept as a separate rounding step (the empty asm stops the
// compiler from folding double -> float -> bf16 into a direct double -> bf16
// conversion, which it emulates with round-to-odd at several times the cost)
__device__ __forceinline__ float to_f32(double x) {
  float f = (float)x;
  asm("" : "+v"(f));
  return f;
}

// float -> (hi, lo) bf16 with hi = RNE(x), lo = RNE(x - hi)
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// 32 consecutive doubles at a wave-uniform address (scalar loads)
__device__ __forceinline__ void load_alpha32(double* dst, const double* __restrict__ alpha, int64_t idx) {
  const double* __restrict__ p = alpha + __builtin_amdgcn_readfirstlane((int)idx);
#pragma unroll
  for (int s = 0; s < kSynChunk; ++s) dst[s] = p[s];
}

// bf16 hi / lo vectors of x[2 v + q], v = 0..7 (one parity of 16 steps):
// hi = RNE(x) converted two at a time, its float value recovered from the
// packed bits, lo = RNE(x - hi), also two at a time
__device__ __forceinline__ void split8(const float* x, int q, bf16x8& hi, bf16x8& lo) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  u32x4 h4, l4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float a = x[2 * (2 * i) + q], b = x[2 * (2 * i + 1) + q];
    const unsigned hp = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2));
    const float ha = __uint_as_float(hp << 16), hb = __uint_as_float(hp & 0xffff0000u);
    h4[i] = hp;
    l4[i] = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a - ha, b - hb}, bf16x2));
  }
  hi = __builtin_bit_cast(bf16x8, h4);
  lo = __builtin_bit_cast(bf16x8, l4);
}

// bf16 hi / lo vectors of x[0..7], as split8
__device__ __forceinline__ void split8c(const float* x, bf16x8& hi, bf16x8& lo) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  u32x4 h4, l4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float a = x[2 * i], b = x[2 * i + 1];
    const unsigned hp = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2));
    const float ha = __uint_as_float(hp << 16), hb = __uint_as_float(hp & 0xffff0000u);
    h4[i] = hp;
    l4[i] = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a - ha, b - hb}, bf16x2));
  }
  hi = __builtin_bit_cast(bf16x8, h4);
  lo = __builtin_bit_cast(bf16x8, l4);
}

// bf16 hi / mid / lo vectors of x[0..7] (three parts: x - hi - mid - lo is
// below 2^-24 |x|), two values per conversion
__device__ __forceinline__ void split8c3(const float* x, bf16x8& hi, bf16x8& mid, bf16x8& lo) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  u32x4 h4, m4, l4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float a = x[2 * i], b = x[2 * i + 1];
    const unsigned hp = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2));
    const float ra = a - __uint_as_float(hp << 16), rb = b - __uint_as_float(hp & 0xffff0000u);
    const unsigned mp = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){ra, rb}, bf16x2));
    const float sa = ra - __uint_as_float(mp << 16), sb = rb - __uint_as_float(mp & 0xffff0000u);
    h4[i] = hp;
    m4[i] = mp;
    l4[i] = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){sa, sb}, bf16x2));
  }
  hi = __builtin_bit_cast(bf16x8, h4);
  mid = __builtin_bit_cast(bf16x8, m4);
  lo = __builtin_bit_cast(bf16x8, l4);
}

// NS bf16 parts of the 8 values x[0..7] (NS = 2: hi, lo; 3: hi, mid, lo)
template <int NS>
__device__ __forceinline__ void split_parts(const float* x, bf16x8 (&pt)[NS]) {
  if constexpr (NS == 2) split8c(x, pt[0], pt[1]);
  else split8c3(x, pt[0], pt[1], pt[2]);
}

// v_permlane32_swap per dword: t0 = (lanes 0-31: k0 own, lanes 32-63: k1 of
// lane - 32), t1 = (lanes 0-31: k0 of lane + 32, lanes 32-63: k1 own)
// (lane layout checked on the device)
__device__ __forceinline__ void swap_halves(bf16x8 k0, bf16x8 k1, bf16x8& t0, bf16x8& t1) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 a = __builtin_bit_cast(u32x4, k0), b = __builtin_bit_cast(u32x4, k1);
  u32x4 r0, r1;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(a[i], b[i], false, false);
    r0[i] = r[0];
    r1[i] = r[1];
  }
  t0 = __builtin_bit_cast(bf16x8, r0);
  t1 = __builtin_bit_cast(bf16x8, r1);
}

__device__ __forceinline__ f32x16 mfma3(bf16x8 ah, bf16x8 al, bf16x8 bh, bf16x8 bl, f32x16 d) {
  d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, d, 0, 0, 0);
  return d;
}

// split products: NS = 2 (bf16x3): hi hi + hi lo + lo hi; NS = 3 (bf16x6):
// the six products of parts whose orders add up to at most 2
template <int NS>
__device__ __forceinline__ f32x16 mfma_parts(const bf16x8 (&a)[NS], const bf16x8 (&b)[NS], f32x16 d) {
  if constexpr (NS == 2) {
    return mfma3(a[0], a[1], b[0], b[1], d);
  } else {
    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[0], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[1], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[0], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[2], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[1], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[0], d, 0, 0, 0);
    return d;
  }
}

// ------------------------------------------------------------- checkpoints
// State (mu_{l-2}, mu_{l-1}) before step 64 T of every (m, pair), computed
// with exactly the recurrence of the transform kernels (zero before the
// pair's start group, the start state at it).
__global__ __launch_bounds__(256) void k_checkpoints(int lmax, int mmax, int npairs, const double* __restrict__ pair_z,
                                                     const double* __restrict__ alpha, const int* __restrict__ lst_g,
                                                     const double2* __restrict__ lst_s,
                                                     const int64_t* __restrict__ mstart,
                                                     const int64_t* __restrict__ tstart,
                                                     double2* __restrict__ ckpt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (p >= npairs || m > mmax) return;
  const size_t o = (size_t)m * npairs + p;
  const double z = pair_z[p];
  const int gs = lst_g[o];
  const double2 s0 = lst_s[o];
  const int64_t base = mstart[m];
  const int nsteps = lmax - m + 1;
  const int64_t t0 = tstart[m];
  double v0 = 0.0, v1 = 0.0;
  for (int st = 0; st < nsteps; ++st) {
    if (st % kAdjTile == 0) ckpt[(size_t)(t0 + st / kAdjTile) * npairs + p] = make_double2(v0, v1);
    if (st % kGroup == 0 && st / kGroup == gs) {
      v0 = s0.x;
      v1 = s0.y;
    }
    const double mu = fma(alpha[base + st] * z, v1, -v0);
    v0 = v1;
    v1 = mu;
  }
}

// ------------------------------------------------------ synthesis operands
// ab tiles: for each (m, chunk c of 32 steps), parity q, half h, the MFMA B
// operand B[k][j] = f_idx * alm[rhs][idx], idx = (l = m + 32 c + 2 k + q, m),
// j = 2 rhs + (re, im), in lane order (lane j + 32 (k/8) holds 8 bf16). The
// block reads each column's 32 steps coalesced (lane -> step) and stages
// f * alm (float) in LDS as [q][rhs][comp][16 steps], from which each lane
// reads its 8 steps contiguously.
template <int NS>
__global__ __launch_bounds__(64) void k_prep_synth(int lmax, int nrhs, const int64_t* __restrict__ mstart,
                                                   const int64_t* __restrict__ cstart, const double2* __restrict__ alm,
                                                   int64_t alm_stride, const double* __restrict__ f,
                                                   bf16x8* __restrict__ ab, int64_t ab_gstride,
                                                   const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ __attribute__((aligned(16))) float st_lds[2][16][2][16];
  const int m = blockIdx.y, c = blockIdx.x, grp = blockIdx.z;   // group grp: right-hand sides 16 grp ..
  nrhs -= 16 * grp;
  alm += (int64_t)16 * grp * alm_stride;
  ab += grp * ab_gstride;
  const int nsteps = lmax - m + 1;
  if (c * kSynChunk >= nsteps) return;
  const int lane = threadIdx.x;
  const int64_t base = mstart[m];
  // element phase: lane -> step lane & 31, columns (lane >> 5) + 2 i
  const int st = c * kSynChunk + (lane & 31);
  const bool live = st < nsteps;
  const double fv = live ? f[base + st] : 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int rhs = (lane >> 5) + 2 * i;
    const double2 a = (rhs < nrhs && live) ? alm[rhs * alm_stride + base + st] : make_double2(0.0, 0.0);
    const int q = (lane & 31) & 1, n = (lane & 31) >> 1;
    st_lds[q][rhs][0][n] = to_f32(fv * a.x);
    st_lds[q][rhs][1][n] = to_f32(fv * a.y);
  }
  __syncthreads();
  // tile phase: lane j + 32 kg, j = 2 rhs + comp, holds steps 2 (8 kg + v) + q
  const int j = lane & 31, kg = lane >> 5;
  bf16x8* dst = ab + (size_t)(cstart[m] + c) * (2 * NS) * 64;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const float* src = &st_lds[q][j >> 1][j & 1][8 * kg];
    const float4 a4 = *reinterpret_cast<const float4*>(src), b4 = *reinterpret_cast<const float4*>(src + 4);
    const float x[8] = {a4.x, a4.y, a4.z, a4.w, b4.x, b4.y, b4.z, b4.w};
    bf16x8 pt[NS];
    split_parts<NS>(x, pt);
#pragma unroll
    for (int u = 0; u < NS; ++u) dst[(q * NS + u) * 64 + lane] = pt[u];
  }
}

// PCG direction update fused with the synthesis operands: for the chunk
// (m, c), p = z + beta p per column (unless the column is done or `update` is
// 0), written back in FP64, and the ab tiles built from bk * p. z, p: [rhs][nalm]
// at column stride nalm; the block stages bk * p (float) in LDS as
// [q][rhs][comp][16 steps] so that each lane reads its 8 steps contiguously.
// Z: the stored type of z (float2 after the block preconditioner). x
// (optional): the pending solution update x += scal[S_XA] p, with the p read
// here before its update.
template <typename Z>
__global__ __launch_bounds__(64) void k_pupdate_prep(int lmax, int nrhs, int64_t nalm, const int64_t* __restrict__ mstart,
                                                     const int64_t* __restrict__ cstart, const double* __restrict__ bk,
                                                     const Z* __restrict__ z, double2* __restrict__ p,
                                                     double2* __restrict__ x, const double* __restrict__ scal,
                                                     int update, bf16x8* __restrict__ ab, int64_t ab_gstride,
                                                     const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ __attribute__((aligned(16))) float st_lds[2][16][2][16];
  const int m = blockIdx.y, c = blockIdx.x, grp = blockIdx.z;   // group grp: right-hand sides 16 grp ..
  nrhs -= 16 * grp;
  z += (int64_t)16 * grp * nalm;
  p += (int64_t)16 * grp * nalm;
  if (x) x += (int64_t)16 * grp * nalm;
  scal += 16 * grp * kScalSlots;
  ab += grp * ab_gstride;
  const int nsteps = lmax - m + 1;
  if (c * kSynChunk >= nsteps) return;
  const int lane = threadIdx.x;
  const int64_t base = mstart[m];
  // element phase: lane -> step lane & 31, columns (lane >> 5) + 2 i
  const int st = c * kSynChunk + (lane & 31);
  const bool live = st < nsteps;
  const double f = live ? bk[base + st] : 0.0;
  // every load first and without per-lane conditions (a load under one is
  // waited for at once): elements outside the chunk or the columns read the
  // m's first element of column 0, and their values are not used
  double2 pv[8], zv[8], xv[8];
  double done[8], beta[8], xa[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int rhs = (lane >> 5) + 2 * i;
    const bool ok = rhs < nrhs && live;
    const int64_t e = ok ? rhs * nalm + base + st : base;
    pv[i] = p[e];
    const double* sc = scal + (ok ? rhs : 0) * kScalSlots;
    if (x) {
      xv[i] = x[e];
      xa[i] = sc[S_XA];
    }
    if (update) {
      zv[i] = zload(z + e);
      done[i] = sc[S_DONE];
      beta[i] = sc[S_BETA];
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int rhs = (lane >> 5) + 2 * i;
    double2 v = make_double2(0.0, 0.0);
    if (rhs < nrhs && live) {
      v = pv[i];
      if (x && xa[i] != 0.0) {
        xv[i].x = fma(xa[i], v.x, xv[i].x);
        xv[i].y = fma(xa[i], v.y, xv[i].y);
        x[rhs * nalm + base + st] = xv[i];
      }
      if (update && done[i] == 0.0) {
        v.x = fma(beta[i], v.x, zv[i].x);
        v.y = fma(beta[i], v.y, zv[i].y);
        p[rhs * nalm + base + st] = v;
      }
    }
    const int q = (lane & 31) & 1, n = (lane & 31) >> 1;
    st_lds[q][rhs][0][n] = to_f32(f * v.x);
    st_lds[q][rhs][1][n] = to_f32(f * v.y);
  }
  __syncthreads();
  // tile phase: lane j + 32 kg, j = 2 rhs + comp, holds steps 2 (8 kg + v) + q
  const int j = lane & 31, kg = lane >> 5;
  bf16x8* dst = ab + (size_t)(cstart[m] + c) * 4 * 64;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const float* src = &st_lds[q][j >> 1][j & 1][8 * kg];
    const float4 a4 = *reinterpret_cast<const float4*>(src), b4 = *reinterpret_cast<const float4*>(src + 4);
    const float x[8] = {a4.x, a4.y, a4.z, a4.w, b4.x, b4.y, b4.z, b4.w};
    bf16x8 hi, lo;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      __bf16 h, l;
      split_bf16(x[v], h, l);
      hi[v] = h;
      lo[v] = l;
    }
    dst[(q * 2 + 0) * 64 + lane] = hi;
    dst[(q * 2 + 1) * 64 + lane] = lo;
  }
}

// ----------------------------------------------------------------- synthesis
// One workgroup of 4 wavefronts per (4 consecutive m, block of 64 ring
// pairs); wavefront w takes m = m0 + w. Lane p runs the recurrence of pair p
// for a chunk of 32 steps, splits mu into bf16 hi and lo (even and odd steps
// apart) in registers, then the wavefront multiplies the two 32-pair M tiles
// by the chunk's ab tiles. Chunks before the first live group of the 64 pairs
// are skipped. The sums of the 4 m leave through LDS as one 64-byte run
// (m0 .. m0 + 3, E and O) per (column, pair) of the [column][pair][m][E, O]
// layout, instead of 16-byte pieces per wavefront.
constexpr int kSynWaves = 4;                       // m per workgroup
constexpr int kSynRow = kSynWaves * 4;             // floats per (column, pair) run: [m][E.re, E.im, O.re, O.im]
constexpr int kSynRhsStride = 32 * kSynRow + 2;    // floats per column in LDS (32 pairs), padded against bank conflicts
template <int NG, int NS>
__global__ __launch_bounds__(256) void k_synth_mfma(int lmax, int mmax, int npairs, int nrhs,
                                                    const double* __restrict__ pair_z, const double* __restrict__ alpha,
                                                    const int* __restrict__ lst_g, const double2* __restrict__ lst_s,
                                                    const int64_t* __restrict__ mstart,
                                                    const int64_t* __restrict__ cstart,
                                                    const bf16x8* __restrict__ ab, int64_t ab_gstride,
                                                    float2* __restrict__ eo, int64_t eo_stride,
                                                    const int* __restrict__ pred) {
  if (pred && *pred) return;
  // results of one pair half (32 pairs) of the 16 columns of a group
  __shared__ __attribute__((aligned(16))) float res[16 * kSynRhsStride];
  const int npb = (npairs + 63) / 64;
  const int q8 = blockIdx.x >> 3;
  // each XCD takes 4 consecutive m out of every 32 (xcd_m): the 4 m of one workgroup
  const int m0 = xcd_m(4 * (q8 / npb), blockIdx.x & 7), pb = q8 % npb;
  const int w = threadIdx.x >> 6;
  const int m = m0 + w;
  const bool mlive = m <= mmax;   // every wavefront stays for the barriers
  const int lane = threadIdx.x & 63;
  const int p = pb * 64 + lane;
  const bool valid = p < npairs && mlive;
  const int pp = p < npairs ? p : npairs - 1;
  const int mm = mlive ? m : mmax;
  const size_t o = (size_t)mm * npairs + pp;
  const double z = pair_z[pp];
  const int gs = valid ? lst_g[o] : kNever;
  const double2 s0 = lst_s[o];
  const int gmin = __builtin_amdgcn_readfirstlane(wave_min(gs));   // wave-uniform: scalar loop control
  const int64_t base = mstart[mm];
  const int nsteps = lmax - mm + 1;

  f32x16 dE0[NG], dE1[NG], dO0[NG], dO1[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) dE0[g] = dE1[g] = dO0[g] = dO1[g] = f32x16{};
  if (gmin != kNever) {
    const int nch = (nsteps + kSynChunk - 1) / kSynChunk;
    double v0 = 0.0, v1 = 0.0;
    const bf16x8* abm = ab + (size_t)cstart[mm] * (2 * NS) * 64 + lane;
    const int cfirst = (gmin * kGroup) / kSynChunk;
    for (int c = cfirst; c < nch; ++c) {
      // operands of this chunk, consumed after the recurrence (which hides
      // their latency)
      bf16x8 bE[NG][NS], bO[NG][NS];
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const bf16x8* src = abm + g * ab_gstride + (size_t)c * (2 * NS * 64);
#pragma unroll
        for (int u = 0; u < NS; ++u) {
          bE[g][u] = src[u * 64];
          bO[g][u] = src[(NS + u) * 64];
        }
      }
      const int st0 = c * kSynChunk;
      float mu32[kSynChunk];
      if (st0 + kSynChunk <= nsteps) {
        // alpha is wave-uniform: all 32 scalar loads issued before the first
        // use (one wait per chunk)
        double a[kSynChunk];
        load_alpha32(a, alpha, base + st0);
#pragma unroll
        for (int s = 0; s < kSynChunk; ++s) {
          if (s % kGroup == 0) {
            const bool inj = (st0 + s) / kGroup == gs;
            v0 = inj ? s0.x : v0;
            v1 = inj ? s0.y : v1;
          }
          const double mu = fma(a[s] * z, v1, -v0);
          v0 = v1;
          v1 = mu;
          mu32[s] = to_f32(mu);
        }
      } else {
        const double* __restrict__ ac = alpha + __builtin_amdgcn_readfirstlane((int)(base + st0));
#pragma unroll
        for (int s = 0; s < kSynChunk; ++s) {
          if (s % kGroup == 0) {
            const bool inj = (st0 + s) / kGroup == gs;
            v0 = inj ? s0.x : v0;
            v1 = inj ? s0.y : v1;
          }
          double mu = 0.0;
          if (st0 + s < nsteps) {
            mu = fma(ac[s] * z, v1, -v0);
            v0 = v1;
            v1 = mu;
          }
          mu32[s] = to_f32(mu);
        }
      }
      bf16x8 e[2][NS], o[2][NS];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if constexpr (NS == 2) {
          split8(mu32 + 16 * h, 0, e[h][0], e[h][1]);
          split8(mu32 + 16 * h, 1, o[h][0], o[h][1]);
        } else {
          float xe[8], xo[8];
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            xe[v] = mu32[16 * h + 2 * v];
            xo[v] = mu32[16 * h + 2 * v + 1];
          }
          split_parts<NS>(xe, e[h]);
          split_parts<NS>(xo, o[h]);
        }
      }
      // A fragments (lane row + 32 kg holds A[row][8 kg .. 8 kg + 7] of M tile t,
      // pairs 32 t + row): lane p owns all 16 k of its pair, so one
      // permlane32 swap of (k 0..7, k 8..15) gives both tiles' fragments
      bf16x8 aE0[NS], aE1[NS], aO0[NS], aO1[NS];
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        swap_halves(e[0][u], e[1][u], aE0[u], aE1[u]);
        swap_halves(o[0][u], o[1][u], aO0[u], aO1[u]);
      }
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        dE0[g] = mfma_parts<NS>(aE0, bE[g], dE0[g]);
        dE1[g] = mfma_parts<NS>(aE1, bE[g], dE1[g]);
        dO0[g] = mfma_parts<NS>(aO0, bO[g], dO0[g]);
        dO1[g] = mfma_parts<NS>(aO1, bO[g], dO1[g]);
      }
    }
  }
  // D[i][j]: lane j + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4, i the pair
  // within the tile, j = 2 rhs + comp. Per group and pair half t the
  // wavefronts put their values at res[rhs][pair][w][E.re, E.im, O.re, O.im];
  // then the 64-byte run of each (rhs, pair) -- the 4 m of the workgroup,
  // contiguous in eo -- is written by 4 consecutive threads, 16 bytes each,
  // so that every store instruction covers whole runs.
  const int j = lane & 31;
  const int comp = j & 1;
  const int nm = min(kSynWaves, mmax + 1 - m0);   // live m of the workgroup (>= 1)
#pragma unroll
  for (int g = 0; g < NG; ++g) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      float* rw = res + (j >> 1) * kSynRhsStride + w * 4 + comp;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
        rw[i * kSynRow] = t ? dE1[g][r] : dE0[g][r];
        rw[i * kSynRow + 2] = t ? dO1[g][r] : dO0[g][r];
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int e = threadIdx.x + 256 * h;   // (run, u): 512 runs x 4 m
        const int run = e >> 2, u = e & 3;
        const int rl = run >> 5, pr = run & 31;
        const int rhs = 16 * g + rl, pair = pb * 64 + 32 * t + pr;
        if (u < nm && rhs < nrhs && pair < npairs) {
          const float* src = res + rl * kSynRhsStride + pr * kSynRow + 4 * u;
          float4* dst = reinterpret_cast<float4*>(eo + rhs * eo_stride + ((size_t)pair * (mmax + 1) + m0 + u) * 2);
          *dst = make_float4(src[0], src[1], src[2], src[3]);
        }
      }
      __syncthreads();
    }
  }
}

// -------------------------------------------------------- adjoint operands
// ag tiles: for each (m, block of 16 pairs), parity q, half h, the MFMA A
// operand A[c][k] = G_q[pair = 16 kb + k][col c] in lane order (lane
// c + 32 (k/8) holds 8 bf16), from the ring-pass output geo
// [rhs][pair][m][q] (float2). A block transposes 16 pairs x 8 m x 16
// columns through LDS: rows (rhs, pair) of 8 m are read coalesced, the
// operand vectors are written contiguously.
constexpr int kPrepM = 8;                       // m per block
constexpr int kPrepMS = 2 * 16 * 2 * 16 + 8;   // floats per m in LDS ([q][rhs][comp][pair], padded)
template <int NS>
__global__ __launch_bounds__(256) void k_prep_adj(int lmax, int mmax, int npairs, int nrhs,
                                                  const int* __restrict__ lst_g, const float2* __restrict__ geo,
                                                  int64_t geo_stride, bf16x8* __restrict__ ag, int64_t ag_gstride,
                                                  const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ __attribute__((aligned(16))) float G[kPrepM * kPrepMS];
  __shared__ int live[kPrepM];            // m holds a live pair of this block of 16
  __shared__ unsigned char livep[kPrepM][16];   // (m, pair) live
  const int kb = blockIdx.x, m0 = blockIdx.y * kPrepM, grp = blockIdx.z;   // right-hand sides 16 grp ..
  nrhs -= 16 * grp;
  geo += (int64_t)16 * grp * geo_stride;
  ag += grp * ag_gstride;
  const int nkb = (npairs + 15) / 16;
  const int t = threadIdx.x;
  // (m, block of 16 pairs) tiles in which no pair starts before the last
  // step of m hold mu = 0 for every l: the adjoint skips their products
  // (the same test per tile of steps), so they are neither read nor written
  if (t < kPrepM) live[t] = 0;
  __syncthreads();
  if (t < kPrepM * 16) {
    const int mm = t >> 4, pair = kb * 16 + (t & 15), m = m0 + mm;
    const bool lv = pair < npairs && m <= mmax && lst_g[(size_t)m * npairs + pair] <= (lmax - m) / kGroup;
    livep[mm][t & 15] = lv ? 1 : 0;
    if (lv) live[mm] = 1;
  }
  __syncthreads();
  // load: row = rhs * 16 + pair (256 rows), 8 m per row, one float4 (q = 0, 1) per (row, m)
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int e = t + i * 256;             // (row, m) item
    const int mm = e & (kPrepM - 1), row = e >> 3;
    const int rhs = row >> 4, pr = row & 15;
    const int pair = kb * 16 + pr, m = m0 + mm;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    // pairs not live at m take 0 (their mu are 0; the FP32 fused ring pass
    // writes no m above the pair's largest live m)
    if (rhs < nrhs && livep[mm][pr])
      v = *reinterpret_cast<const float4*>(geo + rhs * geo_stride + ((size_t)pair * (mmax + 1) + m) * 2);
    float* d = G + mm * kPrepMS + rhs * 32 + pr;
    d[0 * 512 + 0] = v.x;    // q = 0, re
    d[0 * 512 + 16] = v.y;   // q = 0, im
    d[1 * 512 + 0] = v.z;    // q = 1, re
    d[1 * 512 + 16] = v.w;   // q = 1, im
  }
  __syncthreads();
  // write: thread (q, lane) of one m builds the hi and lo operand vectors
  const int q = (t >> 6) & 1, lane = t & 63;
  const int c = lane & 31, kg = lane >> 5;
#pragma unroll
  for (int pass = 0; pass < kPrepM / 2; ++pass) {
    const int mm = pass * 2 + (t >> 7), m = m0 + mm;
    if (m > mmax || !live[mm]) continue;
    const float* src = G + mm * kPrepMS + q * 512 + c * 16 + kg * 8;
    const float4 lo4 = *reinterpret_cast<const float4*>(src), hi4 = *reinterpret_cast<const float4*>(src + 4);
    const float x[8] = {lo4.x, lo4.y, lo4.z, lo4.w, hi4.x, hi4.y, hi4.z, hi4.w};
    bf16x8 pt[NS];
    split_parts<NS>(x, pt);
    bf16x8* dst = ag + ((size_t)m * nkb + kb) * (2 * NS) * 64;
#pragma unroll
    for (int u = 0; u < NS; ++u) dst[(q * NS + u) * 64 + lane] = pt[u];
  }
}

// ------------------------------------------------------------------- adjoint
// One block (4 wavefronts) per (m, tile of 64 steps). Wavefront w covers the
// ring pairs [w * per, (w + 1) * per) in rounds of 64: lane p loads the
// checkpointed recurrence state of its pair at the tile start, runs the 64
// steps and writes mu as FP32 into an LDS tile [q][step / 2][pair]; then
// R_q[col][n] += sum over 4 blocks of 16 pairs of G_q^T (ag) x mu_q, for the
// 32 even (q = 0) and 32 odd (q = 1) steps, with the bf16 hi / lo split of mu
// taken when the operand is read (two values per conversion). The 4 partial
// results are summed in LDS and written as raw FP64 sums out[rhs][idx(l, m)].
// The tile's alpha are staged once per block in LDS and read as broadcasts.
constexpr int kRowF = 64;   // floats per LDS row: 64 pairs
// float offset of pair p in row n: 16-byte chunks XOR-swizzled by the row so
// that the 8 rows read by one group of lanes of a B-fragment load fall on
// different LDS banks
__device__ __forceinline__ int swzf(int n, int p) { return ((((p >> 2) ^ (n & 7)) << 2) | (p & 3)); }

// One tile of the recurrence for this lane's ring pair: mu (FP32) of the 64
// steps into the wavefront's LDS tile [q][step / 2][pair]. The start state is
// injected by selects at the 16-step group boundaries. Past the last step of
// m (alpha = 0 there) the values are finite and reach only output steps that
// are not written. The alpha of the next 8 steps are read while 8 steps run.
__device__ __forceinline__ void adj_tile_steps(float* my, const double2* al, int lane, int st0, int gs, double2 s0,
                                               double z, double v0, double v1) {
  constexpr int kB = 8;   // steps per alpha batch
  int off[8];             // swizzled offset of this lane's pair in rows n with n % 8 = r
#pragma unroll
  for (int r = 0; r < 8; ++r) off[r] = swzf(r, lane);
  double2 ac[kB / 2], an[kB / 2];
#pragma unroll
  for (int i = 0; i < kB / 2; ++i) ac[i] = al[i];
#pragma unroll
  for (int b = 0; b < kAdjTile / kB; ++b) {
    if (b + 1 < kAdjTile / kB) {
#pragma unroll
      for (int i = 0; i < kB / 2; ++i) an[i] = al[(b + 1) * (kB / 2) + i];
    }
    __builtin_amdgcn_sched_barrier(0);
    if ((b * kB) % kGroup == 0) {
      const bool inj = (st0 + b * kB) / kGroup == gs;
      v0 = inj ? s0.x : v0;
      v1 = inj ? s0.y : v1;
    }
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const double a = (j & 1) ? ac[j >> 1].y : ac[j >> 1].x;
      const double mu = fma(a * z, v1, -v0);
      v0 = v1;
      v1 = mu;
      const int s = b * kB + j, q = s & 1, n = s >> 1;   // row n of parity q
      my[(q * 32 + n) * kRowF + off[n & 7]] = to_f32(mu);
    }
#pragma unroll
    for (int i = 0; i < kB / 2; ++i) ac[i] = an[i];
  }
}

template <int NG, int NS>
__global__ __launch_bounds__(256) void k_adj_mfma(int lmax, int mmax, int npairs, int nrhs,
                                                  const double* __restrict__ pair_z, const double* __restrict__ alpha,
                                                  const int* __restrict__ lst_g, const double2* __restrict__ lst_s,
                                                  const int64_t* __restrict__ mstart,
                                                  const int64_t* __restrict__ tstart,
                                                  const int* __restrict__ tile_m, const int* __restrict__ order,
                                                  int maxq, const double2* __restrict__ ckpt,
                                                  const bf16x8* __restrict__ ag, int64_t ag_gstride,
                                                  double2* __restrict__ out, float2* __restrict__ q32,
                                                  int64_t out_stride,
                                                  const double2* __restrict__ qp, const double* __restrict__ sinv,
                                                  const double2* __restrict__ camp, const double* __restrict__ bk,
                                                  double* __restrict__ part, int64_t ntiles,
                                                  const int* __restrict__ pred) {
  if (pred && *pred) return;
  // per wavefront: FP32 [q][32 steps][kRowF pairs]; reused for the partial results
  __shared__ __attribute__((aligned(16))) float lds[kAdjWaves][2][32][kRowF];
  __shared__ double2 al[kAdjTile / 2];   // alpha of the tile's steps (0 past the last step)
  const int tid = order[(blockIdx.x & 7) * maxq + (blockIdx.x >> 3)];   // tiles of one m stay on one XCD
  if (tid < 0) return;
  const int m = tile_m[tid];
  const int T = tid - (int)tstart[m];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t base = mstart[m];
  const int nsteps = lmax - m + 1;
  const int st0 = T * kAdjTile;
  const int slim = min(kAdjTile, nsteps - st0);
  if (threadIdx.x < kAdjTile)
    reinterpret_cast<double*>(al)[threadIdx.x] = (int)threadIdx.x < slim ? alpha[base + st0 + threadIdx.x] : 0.0;
  __syncthreads();
  const int nkb = (npairs + 15) / 16;
  const int per = ((npairs + kAdjWaves * 64 - 1) / (kAdjWaves * 64)) * 64;   // pairs per wavefront
  f32x16 dE[NG], dO[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) dE[g] = dO[g] = f32x16{};
  const int row = lane & 31, kg = lane >> 5;
  float* my = &lds[w][0][0][0];

  // per-pair data of a round (start group, z, start state, checkpoint)
  struct PairData {
    int gs;
    double z;
    double2 s0, ck;
  };
  const int rend = min(npairs, (w + 1) * per);
  auto load_pairs = [&](int r0) {
    PairData d;
    const int p = r0 + lane;
    const bool valid = p < npairs;
    const int pp = valid ? p : npairs - 1;
    const size_t o = (size_t)m * npairs + pp;
    d.gs = valid ? lst_g[o] : kNever;
    d.z = pair_z[pp];
    d.s0 = lst_s[o];
    d.ck = valid ? ckpt[(size_t)(tstart[m] + T) * npairs + pp] : make_double2(0.0, 0.0);
    return d;
  };
  PairData cur = load_pairs(min(w * per, npairs - 1));
  for (int r0 = w * per; r0 < rend; r0 += 64) {
    // the next round's pair data is loaded while this round runs
    PairData nxt = cur;
    if (r0 + 64 < rend) nxt = load_pairs(r0 + 64);
    const int gs = cur.gs;
    // skip the round when no pair becomes live before the end of the tile,
    // and within it the blocks of 16 pairs of which none does: their mu are
    // exactly 0 in this tile, and their operand tiles may not have been
    // written (k_prep_adj skips (m, 16-pair) tiles that stay 0 for every l)
    const uint64_t livemask = __ballot(gs <= (st0 + kAdjTile - 1) / kGroup);
    if (livemask != 0) {
      // G operands of the round's 4 blocks of 16 pairs, issued before the recurrence
      bf16x8 aq[4][2][NS];   // [block of 16 pairs][parity][part]
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int gkb = min(r0 / 16 + kb, nkb - 1);
        const bf16x8* a = ag + ((size_t)m * nkb + gkb) * (2 * NS) * 64;
#pragma unroll
        for (int u = 0; u < 2 * NS; ++u) aq[kb][u / NS][u % NS] = a[u * 64 + lane];
      }
      __builtin_amdgcn_sched_barrier(0);   // keep the operand loads ahead of the recurrence
      const double z = cur.z;
      const double2 s0 = cur.s0;
      adj_tile_steps(my, al, lane, st0, gs, s0, z, cur.ck.x, cur.ck.y);
      // the tile is private to this wavefront and LDS accesses of one
      // wavefront complete in order: a compiler barrier suffices
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        if (g > 0) {
          // operands of the next column group, loaded after the previous
          // group's products are issued (keeps one group in registers)
#pragma unroll
          for (int kb = 0; kb < 4; ++kb) {
            const int gkb = min(r0 / 16 + kb, nkb - 1);
            const bf16x8* a = ag + g * ag_gstride + ((size_t)m * nkb + gkb) * (2 * NS) * 64;
#pragma unroll
            for (int u = 0; u < 2 * NS; ++u) aq[kb][u / NS][u % NS] = a[u * 64 + lane];
          }
        }
        // blocks of 16 pairs past the last pair: their mu are 0 (no start
        // state, zero checkpoint) and they are skipped like blocks of pairs
        // not yet live
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          if (((livemask >> (16 * kb)) & 0xffffull) == 0) continue;   // wavefront-uniform
          // B[k][n] = mu(pair 16 kb + k, step pair n): lane n + 32 (k/8) reads 8 pairs of row n
          const int p0 = 16 * kb + 8 * kg;
          float xe[8], xo[8];
          *reinterpret_cast<float4*>(xe) = *reinterpret_cast<const float4*>(my + row * kRowF + swzf(row, p0));
          *reinterpret_cast<float4*>(xe + 4) = *reinterpret_cast<const float4*>(my + row * kRowF + swzf(row, p0 + 4));
          *reinterpret_cast<float4*>(xo) = *reinterpret_cast<const float4*>(my + (32 + row) * kRowF + swzf(row, p0));
          *reinterpret_cast<float4*>(xo + 4) =
              *reinterpret_cast<const float4*>(my + (32 + row) * kRowF + swzf(row, p0 + 4));
          bf16x8 bE[NS], bO[NS];
          split_parts<NS>(xe, bE);
          split_parts<NS>(xo, bO);
          dE[g] = mfma_parts<NS>(aq[kb][0], bE, dE[g]);
          dO[g] = mfma_parts<NS>(aq[kb][1], bO, dO[g]);
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    cur = nxt;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      // the accumulators stay in AGPRs across rounds (no copies around the recurrence)
      asm volatile("" : "+a"(dE[g]));
      asm volatile("" : "+a"(dO[g]));
    }
  }
  // PCG form: the operands of q (p, S^-1, B, the column amplitudes) are
  // loaded now, without per-lane conditions (out-of-range elements read the
  // tile's first coefficient of column 0), so that their latency overlaps the
  // reduction below. Thread (w, lane) handles component w & 1 of columns
  // 4 k + 2 (lane >> 5) + (w >> 1), k = 0..3, at steps 2 (lane & 31) + q.
  double qpv[4][2], qsi[2], qbk[2], qca[4];
  if (qp) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int st = st0 + 2 * (lane & 31) + q;
      const int64_t i = base + (st < nsteps ? st : st0);
      qsi[q] = sinv ? sinv[i] : 0.0;
      qbk[q] = bk[i];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int rhs = 4 * k + 2 * (lane >> 5) + (w >> 1);
        const bool ok = rhs < nrhs && st < nsteps;
        qpv[k][q] = reinterpret_cast<const double*>(qp + (ok ? rhs : 0) * out_stride + (ok ? i : base + st0))[w & 1];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int rhs = 4 * k + 2 * (lane >> 5) + (w >> 1);
      qca[k] = camp[rhs < nrhs ? rhs : 0].x;
    }
  }
  // one block-wide barrier, reached once by every wavefront; each wavefront
  // reuses its own tile area for its partial result red[w][q][r][lane]
  // (NG x 8 KiB of the wavefront's 16 KiB tile area)
  float* redw = my;
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      redw[((2 * g + 0) * 16 + r) * 64 + lane] = dE[g][r];
      redw[((2 * g + 1) * 16 + r) * 64 + lane] = dO[g][r];
    }
  __syncthreads();
  // D[c][n] at lane n + 32 ((c/4)%2), register 4 (c/8) + c%4; sum the wavefronts
  if (!qp) {
    for (int e = threadIdx.x; e < NG * 2 * 16 * 64; e += blockDim.x) {
      const int g = e / (2 * 16 * 64), q = (e / (16 * 64)) % 2, r = (e / 64) % 16, ln = e % 64;
      float acc = 0.f;
#pragma unroll
      for (int ww = 0; ww < kAdjWaves; ++ww)
        acc += (&lds[ww][0][0][0])[((2 * g + q) * 16 + r) * 64 + ln];
      const int c = 8 * (r / 4) + 4 * (ln >> 5) + (r % 4);
      const int n = ln & 31;
      const int rhs = 16 * g + (c >> 1), comp = c & 1;
      const int st = st0 + 2 * n + q;
      if (rhs < nrhs && st < nsteps)
        reinterpret_cast<double*>(out + rhs * out_stride + base + st)[comp] = (double)acc;
    }
    return;
  }
  // PCG form (one column group): q = camp.x sinv p + bk raw, component by
  // component, stored as FP32 into q32, and the tile's partial of <p, q> of
  // the stored (rounded) q, so that alpha and the update r -= alpha q use the
  // same q
  static_assert(NG == 1 && kAdjWaves == 4, "PCG form: one column group, four wavefronts");
  const int ln = lane, comp = w & 1;
  const int n = ln & 31;
  double pz[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) pz[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int rhs = 4 * k + 2 * (ln >> 5) + (w >> 1);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int r = w + 4 * k;
      float acc = 0.f;
#pragma unroll
      for (int ww = 0; ww < kAdjWaves; ++ww) acc += (&lds[ww][0][0][0])[(q * 16 + r) * 64 + ln];
      const int st = st0 + 2 * n + q;
      if (rhs < nrhs && st < nsteps) {
        const float qv = (float)fma(qca[k] * qsi[q], qpv[k][q], qbk[q] * (double)acc);
        reinterpret_cast<float*>(q32 + rhs * out_stride + base + st)[comp] = qv;
        pz[k] = fma(qpv[k][q], (double)qv, pz[k]);
      }
    }
  }
  // sums over the 32 lanes of each half wavefront (fixed butterfly order),
  // then the two components; weight 1 for m = 0, 2 otherwise
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double v = pz[k];
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o);
    pz[k] = v;
  }
  __syncthreads();   // the tile area is read above; its start holds the sums below
  double* red = reinterpret_cast<double*>(&lds[0][0][0][0]);   // [w][half][k]
  if ((ln & 31) == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) red[(w * 2 + (ln >> 5)) * 4 + k] = pz[k];
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    const int rhs = threadIdx.x;
    const int k = rhs >> 2, half = (rhs >> 1) & 1, wg = rhs & 1;
    if (rhs < nrhs) {
      const double v = red[((2 * wg + 0) * 2 + half) * 4 + k] + red[((2 * wg + 1) * 2 + half) * 4 + k];
      part[rhs * ntiles + tid] = (m == 0 ? 1.0 : 2.0) * v;
    }
  }
}

}  // namespace

// sizes of the mixed-precision tables and buffers
int64_t mixed_synth_chunks(const Geometry& g) {
  int64_t n = 0;
  for (int m = 0; m <= g.mmax; ++m) n += (g.lmax - m + 1 + kSynChunk - 1) / kSynChunk;
  return n;
}
int64_t mixed_adj_tiles(const Geometry& g) {
  int64_t n = 0;
  for (int m = 0; m <= g.mmax; ++m) n += (g.lmax - m + 1 + kAdjTile - 1) / kAdjTile;
  return n;
}
// operand tiles of one group of 16 right-hand sides (bf16x8 units) and the
// buffers for kMaxGroups groups
int64_t ab_group(const Geometry& g) { return mixed_synth_chunks(g) * 4 * 64; }
int64_t ag_group(const Geometry& g) { return (int64_t)(g.mmax + 1) * ((g.npairs + 15) / 16) * 4 * 64; }
// (the bf16x6 form takes one group with three parts instead of two: 3/4 of
// the synthesis buffer of kMaxGroups = 2 groups, 3/2 of the adjoint buffer)
int64_t mixed_ab_bytes(const Geometry& g) { return kMaxGroups * ab_group(g) * 16; }
int64_t mixed_ag_bytes(const Geometry& g) { return kAdjGroups * ag_group(g) * 16 * 3 / 2; }
void mixed_starts(const Geometry& g, std::vector<int64_t>& cst, std::vector<int64_t>& tst, std::vector<int>& tm,
                  std::vector<int>& order, int& maxq) {
  cst.assign(g.mmax + 2, 0);
  tst.assign(g.mmax + 2, 0);
  tm.clear();
  for (int m = 0; m <= g.mmax; ++m) {
    const int ns = g.lmax - m + 1;
    cst[m + 1] = cst[m] + (ns + kSynChunk - 1) / kSynChunk;
    const int nt = (ns + kAdjTile - 1) / kAdjTile;
    tst[m + 1] = tst[m] + nt;
    for (int t = 0; t < nt; ++t) tm.push_back(m);
  }
  // adjoint launch order: per XCD the tiles of its m (xcd_m), m ascending
  std::vector<std::vector<int>> per(8);
  for (int m = 0; m <= g.mmax; ++m)
    for (int64_t t = tst[m]; t < tst[m + 1]; ++t) per[m_xcd(m)].push_back((int)t);
  maxq = 0;
  for (auto& v : per) maxq = std::max(maxq, (int)v.size());
  order.assign((size_t)8 * maxq, -1);
  for (int x = 0; x < 8; ++x)
    for (size_t q = 0; q < per[x].size(); ++q) order[(size_t)x * maxq + q] = per[x][q];
}

// workgroups of k_synth_mfma: per XCD one m quad out of every 32 m, times
// the blocks of 64 ring pairs
int synth_mfma_blocks(const Geometry& g) {
  const int npb = (g.npairs + 63) / 64;
  const int nquad = (g.mmax + 32) / 32;   // quads per XCD covering m = 0..mmax
  return 8 * nquad * npb;
}

hipError_t launch_checkpoints(const crsht_plan* P, hipStream_t s) {
  const Geometry& g = P->g;
  dim3 grid((g.npairs + 255) / 256, g.mmax + 1);
  hipLaunchKernelGGL(k_checkpoints, grid, dim3(256), 0, s, g.lmax, g.mmax, g.npairs, P->t.pair_z, P->t.rec_alpha,
                     P->t.lst_g, P->t.lst_s, P->t.mstart, P->t.mx_tstart, P->t.mx_ckpt);
  return hipGetLastError();
}

// Columns go in launches of at most kMaxGroups groups of 16 right-hand sides
// (kMixedCols / 2); the recurrence of a launch is shared by all its columns.
int launch_groups(int nr) { return (nr + kMixedCols / 2 - 1) / (kMixedCols / 2); }

hipError_t synth_mfma_launch(const crsht_plan* P, int nr, int ns, const bf16x8* ab, float2* eo, int64_t eo_stride,
                             hipStream_t s) {
  const Geometry& g = P->g;
  dim3 gs(synth_mfma_blocks(g));
  const int tid = ns == 3 ? -1 : 3;   // timed: the bf16x3 launches
  timing_begin(P, tid, s);
#define CRSHT_SYNTH_LAUNCH(NG, NS)                                                                                \
  hipLaunchKernelGGL((k_synth_mfma<NG, NS>), gs, dim3(256), 0, s, g.lmax, g.mmax, g.npairs, nr, P->t.pair_z,      \
                     P->t.rec_alpha, P->t.lst_g, P->t.lst_s, P->t.mstart, P->t.mx_cstart, ab, ab_group(g), eo,    \
                     eo_stride, P->pred)
  if (ns == 3)
    CRSHT_SYNTH_LAUNCH(1, 3);
  else if (launch_groups(nr) > 1)
    CRSHT_SYNTH_LAUNCH(2, 2);
  else
    CRSHT_SYNTH_LAUNCH(1, 2);
#undef CRSHT_SYNTH_LAUNCH
  timing_end(P, tid, s);
  return hipGetLastError();
}

hipError_t launch_legendre_synth_mixed(const crsht_plan* P, int nrhs, const double2* alm, const double* f,
                                       float2* eo, hipStream_t s) {
  if (!f) f = P->t.ones;
  const Geometry& g = P->g;
  const int ns = P->mx_split == 3 ? 3 : 2;
  const int64_t eo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  bf16x8* ab = reinterpret_cast<bf16x8*>(P->w.mx_ab);
  const int per = (ns == 3 ? 1 : kMaxGroups) * (kMixedCols / 2);
  for (int c0 = 0; c0 < nrhs; c0 += per) {
    const int nr = min(nrhs - c0, per);
    dim3 gp((g.lmax + kSynChunk) / kSynChunk, g.mmax + 1, launch_groups(nr));
    if (ns == 3)
      hipLaunchKernelGGL(k_prep_synth<3>, gp, dim3(64), 0, s, g.lmax, nr, P->t.mstart, P->t.mx_cstart,
                         alm + (int64_t)c0 * g.nalm, (int64_t)g.nalm, f, ab, ab_group(g), P->pred);
    else
      hipLaunchKernelGGL(k_prep_synth<2>, gp, dim3(64), 0, s, g.lmax, nr, P->t.mstart, P->t.mx_cstart,
                         alm + (int64_t)c0 * g.nalm, (int64_t)g.nalm, f, ab, ab_group(g), P->pred);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = synth_mfma_launch(P, nr, ns, ab, eo + (int64_t)c0 * eo_stride, eo_stride, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// (the PCG inner operator: bf16x3 always)
hipError_t launch_legendre_synth_mixed_cg(const crsht_plan* P, int nrhs, const double2* z, double2* p, bool update,
                                          float2* eo, hipStream_t s, bool z32, double2* x) {
  const Geometry& g = P->g;
  const int64_t eo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  bf16x8* ab = reinterpret_cast<bf16x8*>(P->w.mx_ab);
  const int per = kMaxGroups * (kMixedCols / 2);
  for (int c0 = 0; c0 < nrhs; c0 += per) {
    const int nr = min(nrhs - c0, per);
    dim3 gp((g.lmax + kSynChunk) / kSynChunk, g.mmax + 1, launch_groups(nr));
    if (z32)
      hipLaunchKernelGGL(k_pupdate_prep<float2>, gp, dim3(64), 0, s, g.lmax, nr, g.nalm, P->t.mstart,
                         P->t.mx_cstart, P->w.bk, reinterpret_cast<const float2*>(z) + (int64_t)c0 * g.nalm,
                         p + (int64_t)c0 * g.nalm, x ? x + (int64_t)c0 * g.nalm : nullptr,
                         P->w.scal + (int64_t)c0 * kScalSlots, update ? 1 : 0, ab, ab_group(g), P->pred);
    else
      hipLaunchKernelGGL(k_pupdate_prep<double2>, gp, dim3(64), 0, s, g.lmax, nr, g.nalm, P->t.mstart,
                         P->t.mx_cstart, P->w.bk, z + (int64_t)c0 * g.nalm, p + (int64_t)c0 * g.nalm,
                         x ? x + (int64_t)c0 * g.nalm : nullptr, P->w.scal + (int64_t)c0 * kScalSlots,
                         update ? 1 : 0, ab, ab_group(g), P->pred);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = synth_mfma_launch(P, nr, 2, ab, eo + (int64_t)c0 * eo_stride, eo_stride, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_legendre_adjoint_mixed(const crsht_plan* P, int nrhs, const float2* geo, double2* raw,
                                         hipStream_t s) {
  const Geometry& g = P->g;
  const int ns = P->mx_split == 3 ? 3 : 2;
  const int64_t geo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  bf16x8* ag = reinterpret_cast<bf16x8*>(P->w.mx_ag);
  // one column group per adjoint launch: two groups raise the register use
  // to one wavefront per SIMD, which costs more than the shared recurrence
  // saves (measured at Nside 512)
  const int per = kAdjGroups * (kMixedCols / 2);
  for (int c0 = 0; c0 < nrhs; c0 += per) {
    const int nr = min(nrhs - c0, per);
    dim3 gp((g.npairs + 15) / 16, (g.mmax + kPrepM) / kPrepM, 1);
    if (ns == 3)
      hipLaunchKernelGGL(k_prep_adj<3>, gp, dim3(256), 0, s, g.lmax, g.mmax, g.npairs, nr, P->t.lst_g,
                         geo + (int64_t)c0 * geo_stride,
                         geo_stride, ag, ag_group(g), P->pred);
    else
      hipLaunchKernelGGL(k_prep_adj<2>, gp, dim3(256), 0, s, g.lmax, g.mmax, g.npairs, nr, P->t.lst_g,
                         geo + (int64_t)c0 * geo_stride,
                         geo_stride, ag, ag_group(g), P->pred);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    timing_begin(P, ns == 3 ? -1 : 4, s);   // timed: the bf16x3 launches
#define CRSHT_ADJ_LAUNCH(NS)                                                                                       \
  hipLaunchKernelGGL((k_adj_mfma<1, NS>), dim3(8u * (unsigned)P->t.mx_maxq), dim3(kAdjWaves * 64), 0, s, g.lmax,   \
                     g.mmax, g.npairs, nr, P->t.pair_z, P->t.rec_alpha, P->t.lst_g, P->t.lst_s, P->t.mstart,        \
                     P->t.mx_tstart, P->t.mx_tile_m, P->t.mx_order, P->t.mx_maxq, P->t.mx_ckpt, (const bf16x8*)ag, \
                     ag_group(g), raw + (int64_t)c0 * g.nalm, nullptr, (int64_t)g.nalm, nullptr, nullptr, nullptr,   \
                     nullptr, nullptr, 0, P->pred)
    if (ns == 3)
      CRSHT_ADJ_LAUNCH(3);
    else
      CRSHT_ADJ_LAUNCH(2);
#undef CRSHT_ADJ_LAUNCH
    timing_end(P, ns == 3 ? -1 : 4, s);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_legendre_adjoint_mixed_q(const crsht_plan* P, int nrhs, const float2* geo, const double2* p,
                                           float2* q, hipStream_t s) {
  const Geometry& g = P->g;
  const int64_t geo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  bf16x8* ag = reinterpret_cast<bf16x8*>(P->w.mx_ag);
  const int per = kAdjGroups * (kMixedCols / 2);
  for (int c0 = 0; c0 < nrhs; c0 += per) {
    const int nr = min(nrhs - c0, per);
    dim3 gp((g.npairs + 15) / 16, (g.mmax + kPrepM) / kPrepM, 1);
    hipLaunchKernelGGL(k_prep_adj<2>, gp, dim3(256), 0, s, g.lmax, g.mmax, g.npairs, nr, P->t.lst_g,
                       geo + (int64_t)c0 * geo_stride,
                       geo_stride, ag, ag_group(g), P->pred);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    timing_begin(P, 4, s);
    hipLaunchKernelGGL((k_adj_mfma<1, 2>), dim3(8u * (unsigned)P->t.mx_maxq), dim3(kAdjWaves * 64), 0, s, g.lmax,
                       g.mmax, g.npairs, nr, P->t.pair_z, P->t.rec_alpha, P->t.lst_g, P->t.lst_s, P->t.mstart,
                       P->t.mx_tstart, P->t.mx_tile_m, P->t.mx_order, P->t.mx_maxq, P->t.mx_ckpt, (const bf16x8*)ag,
                       ag_group(g), nullptr, q + (int64_t)c0 * g.nalm, (int64_t)g.nalm, p + (int64_t)c0 * g.nalm,
                       (const double*)P->w.sinv, (const double2*)P->w.camp + c0, (const double*)P->w.bk,
                       P->w.adj_part + (int64_t)c0 * P->t.mx_ntiles, P->t.mx_ntiles, P->pred);
    timing_end(P, 4, s);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace crsht
