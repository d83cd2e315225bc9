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
#include "internal.h"

namespace crsht {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kNever = 0x7fffffff;
constexpr int kGroup = 16;      // start-table group (steps)
constexpr int kSynChunk = 32;   // steps per synthesis K chunk (16 even + 16 odd)
constexpr int kAdjTile = 64;    // steps per adjoint output tile (32 even + 32 odd)
constexpr int kAdjWaves = 4;

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

// float -> (hi, lo) bf16 with hi = RNE(x), lo = RNE(x - hi)
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

__device__ __forceinline__ f32x16 mfma3(bf16x8 ah, bf16x8 al, bf16x8 bh, bf16x8 bl, f32x16 d) {
  d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, d, 0, 0, 0);
  return d;
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
// j = 2 rhs + (re, im), in lane order (lane j + 32 (k/8) holds 8 bf16).
__global__ __launch_bounds__(64) void k_prep_synth(int lmax, int nrhs, const int64_t* __restrict__ mstart,
                                                   const int64_t* __restrict__ cstart, const double2* __restrict__ alm,
                                                   int64_t alm_stride, const double* __restrict__ f,
                                                   bf16x8* __restrict__ ab) {
  const int m = blockIdx.y, c = blockIdx.x;
  const int nsteps = lmax - m + 1;
  if (c * kSynChunk >= nsteps) return;
  const int lane = threadIdx.x;
  const int j = lane & 31, kg = lane >> 5;
  const int rhs = j >> 1, comp = j & 1;
  const int64_t base = mstart[m];
  bf16x8* dst = ab + (size_t)(cstart[m] + c) * 4 * 64;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    bf16x8 hi, lo;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int st = c * kSynChunk + 2 * (8 * kg + v) + q;
      double x = 0.0;
      if (rhs < nrhs && st < nsteps) {
        const double2 a = alm[rhs * alm_stride + base + st];
        x = f[base + st] * (comp ? a.y : a.x);
      }
      __bf16 h, l;
      split_bf16((float)x, h, l);
      hi[v] = h;
      lo[v] = l;
    }
    dst[(q * 2 + 0) * 64 + lane] = hi;
    dst[(q * 2 + 1) * 64 + lane] = lo;
  }
}

// ----------------------------------------------------------------- synthesis
// One wavefront per (m, block of 64 ring pairs): lane p runs the recurrence
// of pair p for a chunk of 32 steps, writes mu (bf16 hi, lo; even and odd
// steps apart) to an LDS tile [pair][k], then the wavefront multiplies the
// two 32-pair M tiles by the chunk's ab tiles. Chunks before the first live
// group of the 64 pairs are skipped.
__global__ __launch_bounds__(64) void k_synth_mfma(int lmax, int mmax, int npairs, int nrhs,
                                                   const double* __restrict__ pair_z, const double* __restrict__ alpha,
                                                   const int* __restrict__ lst_g, const double2* __restrict__ lst_s,
                                                   const int64_t* __restrict__ mstart,
                                                   const int64_t* __restrict__ cstart,
                                                   const bf16x8* __restrict__ ab, float2* __restrict__ eo,
                                                   int64_t eo_stride) {
  // tile[q][h][pair][16 k] bf16: 2 x 2 x 64 x 32 bytes
  __shared__ bf16x8 tile[2][2][64][2];
  const int m = blockIdx.x;
  const int lane = threadIdx.x;
  const int p = blockIdx.y * 64 + lane;
  const bool valid = p < npairs;
  const int pp = valid ? p : npairs - 1;
  const size_t o = (size_t)m * npairs + pp;
  const double z = pair_z[pp];
  const int gs = valid ? lst_g[o] : kNever;
  const double2 s0 = lst_s[o];
  const int gmin = wave_min(gs);
  const int64_t base = mstart[m];
  const int nsteps = lmax - m + 1;

  f32x16 dE0 = {}, dE1 = {}, dO0 = {}, dO1 = {};
  if (gmin != kNever) {
    const int nch = (nsteps + kSynChunk - 1) / kSynChunk;
    double v0 = 0.0, v1 = 0.0;
    const int row = lane & 31, kg = lane >> 5;
    for (int c = (gmin * kGroup) / kSynChunk; c < nch; ++c) {
      // operands of this chunk (independent of the recurrence: issue first)
      const bf16x8* src = ab + (size_t)(cstart[m] + c) * 4 * 64;
      const bf16x8 bEh = src[0 * 64 + lane], bEl = src[1 * 64 + lane];
      const bf16x8 bOh = src[2 * 64 + lane], bOl = src[3 * 64 + lane];
      float mu32[kSynChunk];
#pragma unroll
      for (int s = 0; s < kSynChunk; ++s) {
        const int st = c * kSynChunk + s;
        if (s % kGroup == 0 && st / kGroup == gs) {
          v0 = s0.x;
          v1 = s0.y;
        }
        double mu = 0.0;
        if (st < nsteps) {
          mu = fma(alpha[base + st] * z, v1, -v0);
          v0 = v1;
          v1 = mu;
        }
        mu32[s] = (float)mu;
      }
      bf16x8 eh[2], el[2], oh[2], ol[2];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          __bf16 a, b;
          split_bf16(mu32[2 * (8 * h + v)], a, b);
          eh[h][v] = a;
          el[h][v] = b;
          split_bf16(mu32[2 * (8 * h + v) + 1], a, b);
          oh[h][v] = a;
          ol[h][v] = b;
        }
      __syncthreads();   // previous chunk's tile reads are done
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        tile[0][0][lane][h] = eh[h];
        tile[0][1][lane][h] = el[h];
        tile[1][0][lane][h] = oh[h];
        tile[1][1][lane][h] = ol[h];
      }
      __syncthreads();
      // A fragments: lane holds A[row][8 kg .. 8 kg + 7] of M tile t (pairs 32 t + row)
      const bf16x8 aEh0 = tile[0][0][row][kg], aEl0 = tile[0][1][row][kg];
      const bf16x8 aOh0 = tile[1][0][row][kg], aOl0 = tile[1][1][row][kg];
      const bf16x8 aEh1 = tile[0][0][32 + row][kg], aEl1 = tile[0][1][32 + row][kg];
      const bf16x8 aOh1 = tile[1][0][32 + row][kg], aOl1 = tile[1][1][32 + row][kg];
      dE0 = mfma3(aEh0, aEl0, bEh, bEl, dE0);
      dE1 = mfma3(aEh1, aEl1, bEh, bEl, dE1);
      dO0 = mfma3(aOh0, aOl0, bOh, bOl, dO0);
      dO1 = mfma3(aOh1, aOl1, bOh, bOl, dO1);
    }
  }
  // D[i][j]: lane j + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4
  const int j = lane & 31;
  const int rhs = j >> 1, comp = j & 1;
  if (rhs >= nrhs) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int pr = blockIdx.y * 64 + 32 * t + i;
      if (pr >= npairs) continue;
      float* dst = reinterpret_cast<float*>(eo + rhs * eo_stride + ((size_t)pr * (mmax + 1) + m) * 2);
      dst[comp] = t ? dE1[r] : dE0[r];
      dst[2 + comp] = t ? dO1[r] : dO0[r];
    }
  }
}

// -------------------------------------------------------- adjoint operands
// ag tiles: for each (m, block of 16 pairs), parity q, half h, the MFMA A
// operand A[c][k] = G_q[pair = 16 kb + k][col c] in lane order (lane
// c + 32 (k/8) holds 8 bf16), from the FP64 ring-pass output geo.
__global__ __launch_bounds__(64) void k_prep_adj(int mmax, int npairs, int nrhs, const float2* __restrict__ geo,
                                                 int64_t geo_stride, bf16x8* __restrict__ ag) {
  const int kb = blockIdx.x, m = blockIdx.y;
  const int nkb = (npairs + 15) / 16;
  const int lane = threadIdx.x;
  const int cidx = lane & 31, kg = lane >> 5;
  const int rhs = cidx >> 1, comp = cidx & 1;
  bf16x8* dst = ag + ((size_t)m * nkb + kb) * 4 * 64;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    bf16x8 hi, lo;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int pr = kb * 16 + 8 * kg + v;
      float x = 0.0f;
      if (rhs < nrhs && pr < npairs) {
        const float2 g = geo[rhs * geo_stride + ((size_t)pr * (mmax + 1) + m) * 2 + q];
        x = comp ? g.y : g.x;
      }
      __bf16 h, l;
      split_bf16(x, h, l);
      hi[v] = h;
      lo[v] = l;
    }
    dst[(q * 2 + 0) * 64 + lane] = hi;
    dst[(q * 2 + 1) * 64 + lane] = lo;
  }
}

// ------------------------------------------------------------------- adjoint
// One block (4 wavefronts) per (m, tile of 64 steps). Wavefront w covers the
// ring pairs [w * per, (w + 1) * per) in rounds of 64: lane p loads the
// checkpointed recurrence state of its pair at the tile start, runs the 64
// steps, and writes mu (bf16 hi, lo) into an LDS tile [step][pair]; then
// R_q[col][n] += sum over 4 blocks of 16 pairs of G_q^T (ag) x mu_q, for the
// 32 even (q = 0) and 32 odd (q = 1) steps. The 4 partial results are summed
// in LDS and written as raw FP64 sums out[rhs][idx(l, m)].
constexpr int kRowB = 64 * 2;   // bytes per LDS row: 64 pairs of bf16
// 16-byte chunk of 8 pairs, XOR-swizzled by the row so that the 32 rows read by
// one B-fragment load fall on different LDS banks
__device__ __forceinline__ int swz(int row, int chunk) { return ((chunk ^ (row & 7)) << 4); }

__global__ __launch_bounds__(256) void k_adj_mfma(int lmax, int mmax, int npairs, int nrhs,
                                                  const double* __restrict__ pair_z, const double* __restrict__ alpha,
                                                  const int* __restrict__ lst_g, const double2* __restrict__ lst_s,
                                                  const int64_t* __restrict__ mstart,
                                                  const int64_t* __restrict__ tstart,
                                                  const int* __restrict__ tile_m, const double2* __restrict__ ckpt,
                                                  const bf16x8* __restrict__ ag, double2* __restrict__ out,
                                                  int64_t out_stride) {
  // per wavefront: [q][h][32 steps][kRowB bytes]; reused for the partial results
  __shared__ __attribute__((aligned(16))) unsigned char lds[kAdjWaves][2][2][32][kRowB];
  const int tid = blockIdx.x;                 // global tile id
  const int m = tile_m[tid];
  const int T = tid - (int)tstart[m];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t base = mstart[m];
  const int nsteps = lmax - m + 1;
  const int st0 = T * kAdjTile;
  const int nkb = (npairs + 15) / 16;
  const int per = ((npairs + kAdjWaves * 64 - 1) / (kAdjWaves * 64)) * 64;   // pairs per wavefront
  f32x16 dE = {}, dO = {};
  const int row = lane & 31, kg = lane >> 5;
  unsigned char* my = &lds[w][0][0][0][0];

  for (int r0 = w * per; r0 < min(npairs, (w + 1) * per); r0 += 64) {
    const int p = r0 + lane;
    const bool valid = p < npairs;
    const int pp = valid ? p : npairs - 1;
    const size_t o = (size_t)m * npairs + pp;
    const int gs = valid ? lst_g[o] : kNever;
    // skip the round when no pair becomes live before the end of the tile
    if (wave_min(gs) > (st0 + kAdjTile - 1) / kGroup) continue;
    const double z = pair_z[pp];
    const double2 s0 = lst_s[o];
    const double2 ck = valid ? ckpt[(size_t)(tstart[m] + T) * npairs + pp] : make_double2(0.0, 0.0);
    double v0 = ck.x, v1 = ck.y;
#pragma unroll 4
    for (int s = 0; s < kAdjTile; ++s) {
      const int st = st0 + s;
      if (s % kGroup == 0 && st / kGroup == gs) {
        v0 = s0.x;
        v1 = s0.y;
      }
      double mu = 0.0;
      if (st < nsteps) {
        mu = fma(alpha[base + st] * z, v1, -v0);
        v0 = v1;
        v1 = mu;
      }
      __bf16 h, l;
      split_bf16((float)mu, h, l);
      const int q = s & 1, n = s >> 1;
      const int cb = swz(n, lane >> 3) + (lane & 7) * 2;
      *reinterpret_cast<__bf16*>(my + ((q * 2 + 0) * 32 + n) * kRowB + cb) = h;
      *reinterpret_cast<__bf16*>(my + ((q * 2 + 1) * 32 + n) * kRowB + cb) = l;
    }
    // the tile is private to this wavefront and LDS accesses of one
    // wavefront complete in order: a compiler barrier suffices
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const int gkb = r0 / 16 + kb;
      if (gkb >= nkb) break;
      const bf16x8* a = ag + ((size_t)m * nkb + gkb) * 4 * 64;
      const bf16x8 aEh = a[0 * 64 + lane], aEl = a[1 * 64 + lane];
      const bf16x8 aOh = a[2 * 64 + lane], aOl = a[3 * 64 + lane];
      // B[k][n] = mu(pair 16 kb + k, step pair n): lane n + 32 (k/8) reads 8 pairs of row n
      const int off = swz(row, 2 * kb + kg);
      const bf16x8 bEh = *reinterpret_cast<const bf16x8*>(my + ((0 * 2 + 0) * 32 + row) * kRowB + off);
      const bf16x8 bEl = *reinterpret_cast<const bf16x8*>(my + ((0 * 2 + 1) * 32 + row) * kRowB + off);
      const bf16x8 bOh = *reinterpret_cast<const bf16x8*>(my + ((1 * 2 + 0) * 32 + row) * kRowB + off);
      const bf16x8 bOl = *reinterpret_cast<const bf16x8*>(my + ((1 * 2 + 1) * 32 + row) * kRowB + off);
      dE = mfma3(aEh, aEl, bEh, bEl, dE);
      dO = mfma3(aOh, aOl, bOh, bOl, dO);
    }
    __builtin_amdgcn_wave_barrier();
  }
  // one block-wide barrier, reached once by every wavefront; each wavefront
  // reuses its own tile area for its partial result red[w][q][r][lane]
  float* redw = reinterpret_cast<float*>(my);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    redw[(0 * 16 + r) * 64 + lane] = dE[r];
    redw[(1 * 16 + r) * 64 + lane] = dO[r];
  }
  __syncthreads();
  // D[c][n] at lane n + 32 ((c/4)%2), register 4 (c/8) + c%4; sum the wavefronts
  for (int e = threadIdx.x; e < 2 * 16 * 64; e += blockDim.x) {
    const int q = e / (16 * 64), r = (e / 64) % 16, ln = e % 64;
    float acc = 0.f;
#pragma unroll
    for (int ww = 0; ww < kAdjWaves; ++ww)
      acc += reinterpret_cast<const float*>(&lds[ww][0][0][0][0])[(q * 16 + r) * 64 + ln];
    const int c = 8 * (r / 4) + 4 * (ln >> 5) + (r % 4);
    const int n = ln & 31;
    const int rhs = c >> 1, comp = c & 1;
    const int st = st0 + 2 * n + q;
    if (rhs < nrhs && st < nsteps)
      reinterpret_cast<double*>(out + rhs * out_stride + base + st)[comp] = (double)acc;
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
int64_t mixed_ab_bytes(const Geometry& g) { return mixed_synth_chunks(g) * 4 * 64 * 16; }
int64_t mixed_ag_bytes(const Geometry& g) { return (int64_t)(g.mmax + 1) * ((g.npairs + 15) / 16) * 4 * 64 * 16; }
void mixed_starts(const Geometry& g, std::vector<int64_t>& cst, std::vector<int64_t>& tst, std::vector<int>& tm) {
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
}

hipError_t launch_checkpoints(const crsht_plan* P, hipStream_t s) {
  const Geometry& g = P->g;
  dim3 grid((g.npairs + 255) / 256, g.mmax + 1);
  hipLaunchKernelGGL(k_checkpoints, grid, dim3(256), 0, s, g.lmax, g.mmax, g.npairs, P->t.pair_z, P->t.rec_alpha,
                     P->t.lst_g, P->t.lst_s, P->t.mstart, P->t.mx_tstart, P->t.mx_ckpt);
  return hipGetLastError();
}

// columns of one group: at most kMixedCols / 2 right-hand sides
hipError_t launch_legendre_synth_mixed(const crsht_plan* P, int nrhs, const double2* alm, const double* f,
                                       float2* eo, hipStream_t s) {
  if (!f) f = P->t.ones;
  const Geometry& g = P->g;
  const int64_t eo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  bf16x8* ab = reinterpret_cast<bf16x8*>(P->w.mx_ab);
  for (int c0 = 0; c0 < nrhs; c0 += kMixedCols / 2) {
    const int nr = min(nrhs - c0, kMixedCols / 2);
    dim3 gp((g.lmax + kSynChunk) / kSynChunk, g.mmax + 1);
    hipLaunchKernelGGL(k_prep_synth, gp, dim3(64), 0, s, g.lmax, nr, P->t.mstart, P->t.mx_cstart,
                       alm + (int64_t)c0 * g.nalm, (int64_t)g.nalm, f, ab);
    timing_begin(P, 3, s);
    dim3 gs(g.mmax + 1, (g.npairs + 63) / 64);
    hipLaunchKernelGGL(k_synth_mfma, gs, dim3(64), 0, s, g.lmax, g.mmax, g.npairs, nr, P->t.pair_z, P->t.rec_alpha,
                       P->t.lst_g, P->t.lst_s, P->t.mstart, P->t.mx_cstart, (const bf16x8*)ab,
                       eo + (int64_t)c0 * eo_stride, eo_stride);
    timing_end(P, 3, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_legendre_adjoint_mixed(const crsht_plan* P, int nrhs, const float2* geo, double2* raw,
                                         hipStream_t s) {
  const Geometry& g = P->g;
  const int64_t geo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  bf16x8* ag = reinterpret_cast<bf16x8*>(P->w.mx_ag);
  for (int c0 = 0; c0 < nrhs; c0 += kMixedCols / 2) {
    const int nr = min(nrhs - c0, kMixedCols / 2);
    dim3 gp((g.npairs + 15) / 16, g.mmax + 1);
    hipLaunchKernelGGL(k_prep_adj, gp, dim3(64), 0, s, g.mmax, g.npairs, nr, geo + (int64_t)c0 * geo_stride,
                       geo_stride, ag);
    timing_begin(P, 4, s);
    hipLaunchKernelGGL(k_adj_mfma, dim3((unsigned)P->t.mx_ntiles), dim3(kAdjWaves * 64), 0, s, g.lmax, g.mmax,
                       g.npairs, nr, P->t.pair_z, P->t.rec_alpha, P->t.lst_g, P->t.lst_s, P->t.mstart,
                       P->t.mx_tstart, P->t.mx_tile_m, P->t.mx_ckpt, (const bf16x8*)ag,
                       raw + (int64_t)c0 * g.nalm, (int64_t)g.nalm);
    timing_end(P, 4, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace crsht
