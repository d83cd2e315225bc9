// Legendre step of the spherical-harmonic transforms, FP64 vector-ALU form.
//
// lambda_lm(z) = Delta_lm P_lm(z) (paper App. A) is evaluated by the standard
// three-term recurrence written for mu_l = lambda_l / kappa_l, which needs one
// multiply and one FMA per step:
//     mu_m = lambda_mm,  mu_{m-1} = 0,  mu_l = (alpha_lm z) mu_{l-1} - mu_{l-2}.
// kappa_lm is folded into the a_lm before synthesis and into the outputs of
// the adjoint. lambda_mm ~ sin^m(theta) underflows near the poles at large m;
// values there carry an integer scale (see kScaleBits) and contribute only
// once they reach the double range.
//
// North/south symmetry lambda_lm(-z) = (-1)^{l+m} lambda_lm(z) (App. A,
// parity of P_lm) lets one recurrence serve a ring and its mirror: synthesis
// produces E (sum over even l-m) and O (odd l-m) per ring pair, the ring
// kernel forms F_N = E + O and F_S = E - O; the adjoint consumes
// G_N + G_S (even l-m) and G_N - G_S (odd l-m).
#include <algorithm>

#include "internal.h"

namespace crsht {
namespace {

constexpr int kSynthBlock = 64;   // ring pairs per block (one wavefront, one pair per lane)
constexpr int kSynthMT = 4;       // consecutive m per thread: 4 x (E,O) = 128 contiguous bytes per column
constexpr int kChunk = 64;        // l steps per coefficient chunk staged in LDS
constexpr int kGroup = 16;        // l steps per start group (see k_legendre_start)
constexpr int kNever = 0x7fffffff;
constexpr int kAdjBlock = 256;    // threads per block of the adjoint (one m per block)
constexpr int kAdjOutputs = 16;   // doubles reduced across the block per chunk

// Start tables. lambda_lm(z) for large m is far below the double range for
// all l before the turning region, and contributes nothing there. At plan
// creation k_legendre_start runs the recurrence once in scaled arithmetic
// (value v * 2^(600 k), k <= 0) for every (m, ring pair) and records the
// first group of kGroup steps (l - m = 16 g .. 16 g + 15) in which
// |mu| >= 2^-100, together with the exact state (mu_{l-2}, mu_{l-1}) at the
// start of that group as ordinary doubles (>= 2^-308 in magnitude, since a
// value grows by at most 2^13 per step). The transform kernels start every
// pair from zero, load that state when they reach its group, and skip
// groups in which no pair of a wavefront is live.
__device__ __forceinline__ void rescale(double& v0, double& v1, int& k) {
  if (k < 0 && fabs(v1) > kRescaleAbove) {
    v0 *= kRescaleBy;
    v1 *= kRescaleBy;
    ++k;
  }
}

__global__ __launch_bounds__(256) void k_legendre_start(int lmax, int mmax, int npairs,
                                                       const double* __restrict__ pair_z,
                                                       const double* __restrict__ alpha,
                                                       const double* __restrict__ lmm_v, const int* __restrict__ lmm_k,
                                                       const int64_t* __restrict__ mstart, int* __restrict__ lst_g,
                                                       double2* __restrict__ lst_s) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (p >= npairs || m > mmax) return;
  const size_t o = (size_t)m * npairs + p;
  const double z = pair_z[p];
  const int64_t base = mstart[m];
  const int nsteps = lmax - m + 1;
  double v0 = -lmm_v[o], v1 = 0.0;
  int k = lmm_k[o];
  double s0 = v0, s1 = v1;
  int sk = k;
  int g = kNever;
  for (int st = 0; st < nsteps; ++st) {
    if (st % kGroup == 0) {
      s0 = v0;
      s1 = v1;
      sk = k;
    }
    const double mu = fma(alpha[base + st] * z, v1, -v0);
    v0 = v1;
    v1 = mu;
    rescale(v0, v1, k);
    if (k == 0) {
      g = st / kGroup;
      break;
    }
  }
  lst_g[o] = g;
  lst_s[o] = (g == kNever) ? make_double2(0.0, 0.0)
                           : make_double2(ldexp(s0, kScaleBits * sk), ldexp(s1, kScaleBits * sk));
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

// ------------------------------------------------------------------ synthesis
// Block = one wavefront of 64 ring pairs; each lane walks kSynthMT
// consecutive m. For each m the step l = m .. lmax is generic:
// mu_l = (alpha_lm z) mu_{l-1} - mu_{l-2} (alpha_mm = 0 and the start state
// (-lambda_mm, 0) give mu_m = lambda_mm). Coefficients (alpha and the
// kappa-scaled a_lm of NR columns) are staged through LDS in chunks of 64
// steps, the next chunk being fetched into registers while the current one
// is consumed. Chunks before the wavefront's first live group are skipped.
template <int NR>
__global__ __launch_bounds__(kSynthBlock) void k_legendre_synth(
    int lmax, int mmax, int npairs, const double* __restrict__ pair_z, const double* __restrict__ alpha,
    const int* __restrict__ lst_g, const double2* __restrict__ lst_s, const int64_t* __restrict__ mstart,
    const double2* __restrict__ alms, int64_t alm_stride, double2* __restrict__ eo, int64_t eo_stride,
    const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ double s_al[2][kChunk];
  __shared__ double2 s_a[2][NR][kChunk];
  const int lane = threadIdx.x;
  const int p = blockIdx.y * kSynthBlock + lane;
  const bool valid = p < npairs;
  const int pp = valid ? p : npairs - 1;
  const double z = pair_z[pp];
  const int mfirst = blockIdx.x * kSynthMT;
#pragma unroll 1
  for (int mi = 0; mi < kSynthMT; ++mi) {
    const int m = mfirst + mi;
    if (m > mmax) break;
    const int64_t base = mstart[m];
    const int nsteps = lmax - m + 1;
    const size_t o = (size_t)m * npairs + pp;
    const int gs = valid ? lst_g[o] : kNever;
    const double2 st0 = lst_s[o];
    const int gmin = wave_min(gs);
    double2 E[NR], O[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) E[c] = O[c] = make_double2(0.0, 0.0);
    if (gmin != kNever) {
      double v0 = 0.0, v1 = 0.0;
      const int ch0 = (gmin * kGroup) / kChunk;
      {
        const int st = ch0 * kChunk + lane;
        const bool in = st < nsteps;
        s_al[0][lane] = in ? alpha[base + st] : 0.0;
#pragma unroll
        for (int c = 0; c < NR; ++c) s_a[0][c][lane] = in ? alms[c * alm_stride + base + st] : make_double2(0.0, 0.0);
      }
      __syncthreads();
      const int nch = (nsteps + kChunk - 1) / kChunk;
      int cur = 0;
#pragma unroll 1
      for (int ch = ch0; ch < nch; ++ch) {
        // fetch the next chunk into registers
        const int nx = (ch + 1) * kChunk + lane;
        const bool in = nx < nsteps;
        const double pal = in ? alpha[base + nx] : 0.0;
        double2 pa[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) pa[c] = in ? alms[c * alm_stride + base + nx] : make_double2(0.0, 0.0);

        const int cnt = min(kChunk, nsteps - ch * kChunk);
        if (cnt == kChunk) {
#pragma unroll
          for (int q = 0; q < kChunk / kGroup; ++q) {
            if (ch * (kChunk / kGroup) + q == gs) {
              v0 = st0.x;
              v1 = st0.y;
            }
#pragma unroll
            for (int j = q * kGroup; j < (q + 1) * kGroup; j += 2) {
              const double mu1 = fma(s_al[cur][j] * z, v1, -v0);
              const double mu2 = fma(s_al[cur][j + 1] * z, mu1, -v1);
              v0 = mu1;
              v1 = mu2;
#pragma unroll
              for (int c = 0; c < NR; ++c) {
                const double2 ae = s_a[cur][c][j], ao = s_a[cur][c][j + 1];
                E[c].x = fma(mu1, ae.x, E[c].x);
                E[c].y = fma(mu1, ae.y, E[c].y);
                O[c].x = fma(mu2, ao.x, O[c].x);
                O[c].y = fma(mu2, ao.y, O[c].y);
              }
            }
          }
        } else {
          for (int j = 0; j < cnt; ++j) {
            if (j % kGroup == 0 && ch * (kChunk / kGroup) + j / kGroup == gs) {
              v0 = st0.x;
              v1 = st0.y;
            }
            const double mu = fma(s_al[cur][j] * z, v1, -v0);
            v0 = v1;
            v1 = mu;
#pragma unroll
            for (int c = 0; c < NR; ++c) {
              double2& acc = (j & 1) ? O[c] : E[c];
              acc.x = fma(mu, s_a[cur][c][j].x, acc.x);
              acc.y = fma(mu, s_a[cur][c][j].y, acc.y);
            }
          }
        }
        // publish the next chunk
        s_al[cur ^ 1][lane] = pal;
#pragma unroll
        for (int c = 0; c < NR; ++c) s_a[cur ^ 1][c][lane] = pa[c];
        __syncthreads();
        cur ^= 1;
      }
    }
    if (valid) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        double2* dst = eo + c * eo_stride + ((size_t)p * (mmax + 1) + m) * 2;
        dst[0] = E[c];
        dst[1] = O[c];
      }
    }
  }
}

// -------------------------------------------------------------------- adjoint
// One block per m. Thread t owns the RPT consecutive ring pairs
// t*RPT .. t*RPT+RPT-1; each step adds mu_lm(z_p) * G_p over its pairs, and
// every C steps the block reduces the per-thread partial sums through LDS and
// writes the raw sums raw[c][idx(l,m)] = sum_p mu_lm(z_p) G_p (G = G_N + G_S
// for even l - m, G_N - G_S for odd). MODE_DIAG sums mu^2 W_p instead (the
// preconditioner diagonal; W_p the ring-pair sum of N^-1). All scaling (kappa,
// b_l, 1/C_l) happens in the vector kernels. alpha of the m is staged in LDS.
enum { MODE_RAW = 0, MODE_DIAG = 2 };

__device__ __forceinline__ int block_to_m(int b) {
  // blocks are dealt to the 8 XCDs round-robin; give each XCD four
  // consecutive m so the 128-byte lines of G they share stay in one L2
  const int xcd = b & 7, q = b >> 3;
  return (q >> 2) * 32 + xcd * 4 + (q & 3);
}

template <int NR, int RPT, int MODE>
__global__ __launch_bounds__(kAdjBlock) void k_legendre_adj(
    int lmax, int mmax, int npairs, const double* __restrict__ pair_z, const double* __restrict__ alpha,
    const int* __restrict__ lst_g, const double2* __restrict__ lst_s, const int64_t* __restrict__ mstart,
    const double2* __restrict__ geo, int64_t geo_stride, const double* __restrict__ ringw,
    double2* __restrict__ out, int64_t out_stride, const int* __restrict__ pred) {
  if (pred && *pred) return;
  constexpr int C = kAdjOutputs / (2 * NR);          // l steps per reduction chunk (divides kGroup)
  constexpr int TPO = kAdjBlock / kAdjOutputs;        // threads per reduced output
  extern __shared__ double s_al[];                    // [lmax+1] alpha of this m
  __shared__ double red[kAdjOutputs][kAdjBlock];

  const int m = block_to_m(blockIdx.x);
  if (m > mmax) return;
  const int t = threadIdx.x;
  const int64_t base = mstart[m];
  const int nsteps = lmax - m + 1;
  for (int j = t; j < nsteps; j += kAdjBlock) s_al[j] = alpha[base + j];

  double z[RPT], v0[RPT], v1[RPT];
  int gs[RPT];
  double2 st[RPT];
  double2 ge[RPT][NR], go[RPT][NR];
  int gmin = kNever;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int p = t * RPT + j;
    const bool ok = p < npairs;
    const int pp = ok ? p : 0;
    const size_t o = (size_t)m * npairs + pp;
    z[j] = pair_z[pp];
    v0[j] = 0.0;
    v1[j] = 0.0;
    gs[j] = ok ? lst_g[o] : kNever;
    st[j] = lst_s[o];
    gmin = min(gmin, gs[j]);
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      if (MODE == MODE_DIAG) {
        const double wgt = ok ? ringw[pp] : 0.0;
        ge[j][c] = make_double2(wgt, 0.0);
        go[j][c] = ge[j][c];
      } else {
        const double2* g = geo + c * geo_stride + ((size_t)pp * (mmax + 1) + m) * 2;
        ge[j][c] = ok ? g[0] : make_double2(0.0, 0.0);
        go[j][c] = ok ? g[1] : make_double2(0.0, 0.0);
      }
    }
  }
  gmin = wave_min(gmin);   // first live group of this wavefront
  __syncthreads();

  const int o = t / TPO;        // output this thread reduces: (jj, c, re/im)
  const int s = t % TPO;
  const int o_jj = o / (2 * NR), o_c = (o / 2) % NR, o_ri = o & 1;

  for (int l0 = 0; l0 < nsteps; l0 += C) {
    double2 part[C][NR];
#pragma unroll
    for (int jj = 0; jj < C; ++jj)
#pragma unroll
      for (int c = 0; c < NR; ++c) part[jj][c] = make_double2(0.0, 0.0);

    const int grp = l0 / kGroup;
    if (grp >= gmin) {
      if (l0 % kGroup == 0) {
#pragma unroll
        for (int j = 0; j < RPT; ++j)
          if (gs[j] == grp) {
            v0[j] = st[j].x;
            v1[j] = st[j].y;
          }
      }
#pragma unroll
      for (int jj = 0; jj < C; ++jj) {
        if (C > 1 && l0 + jj >= nsteps) break;
        const double a = s_al[l0 + jj];
        const bool odd = (C % 2 == 0) ? (jj & 1) : ((l0 + jj) & 1);   // C even: l0 even
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const double mu = fma(a * z[j], v1[j], -v0[j]);
          v0[j] = v1[j];
          v1[j] = mu;
          const double w = (MODE == MODE_DIAG) ? mu * mu : mu;
#pragma unroll
          for (int c = 0; c < NR; ++c) {
            const double2 g = odd ? go[j][c] : ge[j][c];
            part[jj][c].x = fma(w, g.x, part[jj][c].x);
            part[jj][c].y = fma(w, g.y, part[jj][c].y);
          }
        }
      }
    }

#pragma unroll
    for (int jj = 0; jj < C; ++jj)
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        red[(jj * NR + c) * 2 + 0][t] = part[jj][c].x;
        red[(jj * NR + c) * 2 + 1][t] = part[jj][c].y;
      }
    __syncthreads();
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < kAdjBlock / TPO; ++i) sum += red[o][s + TPO * i];
#pragma unroll
    for (int off = TPO / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, TPO);
    const int sto = l0 + o_jj;
    if (s == 0 && sto < nsteps) reinterpret_cast<double*>(out + o_c * out_stride + base + sto)[o_ri] = sum;
    __syncthreads();
  }
}

// ------------------------------------------------- adjoint on FP64 matrix cores
// The adjoint sums raw[c](l) = sum_p mu_lm(z_p) G_c(p) are a contraction over
// the ring pairs p, so the matrix cores can take the sum over p that the
// vector kernel above does by cross-thread reduction. One block per m with
// kAmWaves wavefronts; wavefront w owns the ring pairs 128 w .. 128 w + 127 as
// two subsets of 64 (lane q: pairs 128 w + q and 128 w + 64 + q). Per chunk of
// 32 l-steps, for each subset every lane runs the recurrence of its pair for
// 32 steps and writes mu to the wavefront's own LDS rows (row = lane, 33
// doubles: conflict-free reads of the operand below); the wavefront then
// accumulates, with v_mfma_f64_16x16x4_f64 over 16 K-steps of 4 pairs,
//   D_par[i][j] += sum_k mu(l0 + 2 i + par, p_k) G_par(p_k, j),
// par = E (even l - m, G_N + G_S) and O (odd, G_N - G_S), j = 2 c + (re, im)
// over up to 8 complex columns. The G operands of the wavefront's 128 pairs
// stay in registers for the whole m. After both subsets the kAmWaves
// wavefronts' 16 x 16 tiles are summed through LDS in a fixed order
// (deterministic) and the 32 l-steps x ncols results written. A block covers
// kAmPairs ring pairs from p_off; grids with more pairs take one launch per
// kAmPairs, the later ones adding to what the earlier wrote (accumulate = 1),
// in launch order. All products and sums are FP64. Four wavefronts per block
// (two launches at Nside 512) rather than eight (one launch): a CU then holds
// two independent blocks, whose barriers (two per chunk) do not hold each
// other, so one block's recurrence overlaps the other's matrix products
// (1.98 against 2.36 ms per 16-column transform at Nside 512, although the
// later launch re-reads the sums the earlier one wrote); with eight
// wavefronts, one block per CU, both wavefronts of a SIMD left each barrier
// together and competed for the same unit.
// FP64 MFMA 16x16x4 lane layout: A[i][k] in lane i + 16 k, B[k][j] in lane
// j + 16 k, D[i][j] in lane j + 16 (i % 4), register i / 4.
typedef double f64x4_t __attribute__((ext_vector_type(4)));
constexpr int kAmWaves = 4;
constexpr int kAmChunk = 32;     // l-steps per chunk: 16 rows of each parity
constexpr int kAmRow = 33;       // LDS row stride (doubles) of the mu staging
constexpr int kAmCols = 8;       // complex columns per launch (16 real MFMA columns)
constexpr int kAmPairs = kAmWaves * 128;   // ring pairs one block covers

__global__ __launch_bounds__(kAmWaves * 64) void k_legendre_adj_mfma(
    int lmax, int mmax, int npairs, int plim, int p_off, int accumulate, int ncols, const double* __restrict__ pair_z,
    const double* __restrict__ alpha, const int* __restrict__ lst_g, const double2* __restrict__ lst_s,
    const int64_t* __restrict__ mstart, const double2* __restrict__ geo, int64_t geo_stride, double2* __restrict__ out,
    int64_t out_stride, const int* __restrict__ pred) {
  if (pred && *pred) return;
  extern __shared__ double am_lds[];   // [kAmWaves][64][kAmRow]
  const int m = block_to_m(blockIdx.x);
  if (m > mmax) return;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  double* my = am_lds + (size_t)w * 64 * kAmRow;
  const int64_t base = mstart[m];
  const int nsteps = lmax - m + 1;

  double z[2], v0[2], v1[2];
  int gs[2];
  double2 st[2];
  int wmin = kNever;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int p = p_off + 128 * w + 64 * u + lane;
    const bool ok = p < plim;   // pairs below plim only (tables have npairs per m)
    const int pp = ok ? p : 0;
    const size_t o = (size_t)m * npairs + pp;
    z[u] = pair_z[pp];
    v0[u] = 0.0;
    v1[u] = 0.0;
    gs[u] = ok ? lst_g[o] : kNever;
    st[u] = lst_s[o];
    wmin = min(wmin, gs[u]);
  }
  wmin = wave_min(wmin);   // first live group of this wavefront
  __shared__ int wmin_s[kAmWaves];
  if (lane == 0) wmin_s[w] = wmin;
  __syncthreads();
  int bmin = kNever;   // first live group of the workgroup
#pragma unroll
  for (int ww = 0; ww < kAmWaves; ++ww) bmin = min(bmin, wmin_s[ww]);
  // B operands: G_par(p, j) for p = 128 w + 64 u + 4 s + (lane / 16), j = lane % 16
  const int kq = lane >> 4, jc = lane & 15, col = jc >> 1, ri = jc & 1;
  double b[2][16][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int sk = 0; sk < 16; ++sk) {
      const int p = p_off + 128 * w + 64 * u + 4 * sk + kq;
      const bool ok = p < plim && col < ncols;
      const double* g =
          reinterpret_cast<const double*>(geo + (ok ? col : 0) * geo_stride + ((size_t)(ok ? p : 0) * (mmax + 1) + m) * 2);
      b[u][sk][0] = ok ? g[ri] : 0.0;
      b[u][sk][1] = ok ? g[2 + ri] : 0.0;
    }
  const int ai = lane & 15;   // A row (l index within the parity) of this lane

#pragma unroll 1
  for (int l0 = 0; l0 < nsteps; l0 += kAmChunk) {
    if (accumulate && l0 / kGroup + 1 < bmin) continue;   // no live pair: the sums would add zeros
    f64x4_t acc[2][2];
#pragma unroll
    for (int par = 0; par < 2; ++par) acc[par][0] = acc[par][1] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    if (l0 / kGroup + 1 >= wmin) {   // the chunk reaches this wavefront's first live group
      // alpha of the chunk in one batch of loads. Past the last step of this
      // m they are the next m's (or the table's zero padding): the rows of
      // those l-steps only reach D rows whose outputs are not written.
      double al[kAmChunk];
#pragma unroll
      for (int sp = 0; sp < kAmChunk; ++sp) al[sp] = alpha[base + l0 + sp];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int sp = 0; sp < kAmChunk; ++sp) {
          if (sp % kGroup == 0 && (l0 + sp) / kGroup == gs[u]) {
            v0[u] = st[u].x;
            v1[u] = st[u].y;
          }
          const double mu = fma(al[sp] * z[u], v1[u], -v0[u]);
          v0[u] = v1[u];
          v1[u] = mu;
          my[lane * kAmRow + sp] = mu;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int sk = 0; sk < 16; ++sk)
#pragma unroll
          for (int par = 0; par < 2; ++par) {
            const double a = my[(4 * sk + kq) * kAmRow + 2 * ai + par];
            acc[par][sk & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[u][sk][par], acc[par][sk & 1], 0, 0, 0);
          }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    // this wavefront's tiles into its own rows (its products have read them)
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int r = 0; r < 4; ++r) my[par * 256 + r * 64 + lane] = acc[par][0][r] + acc[par][1][r];
    __syncthreads();
    {
      // thread t: columns t / 64 + kAmWaves k, l-step l0 + (t % 64) / 2,
      // re/im t % 2 (coalesced stores)
      const int sq = (t & 63) >> 1, rr = t & 1;
      const int stp = l0 + sq;
      for (int c = t >> 6; c < ncols && stp < nsteps; c += kAmWaves) {
        const int par = sq & 1, i = sq >> 1;
        const int idx = par * 256 + (i >> 2) * 64 + (2 * c + rr) + 16 * (i & 3);
        double sum = 0.0;
#pragma unroll
        for (int ww = 0; ww < kAmWaves; ++ww) sum += am_lds[(size_t)ww * 64 * kAmRow + idx];
        double* o = reinterpret_cast<double*>(out + c * out_stride + base + stp) + rr;
        *o = accumulate ? *o + sum : sum;
      }
    }
    __syncthreads();   // the rows are rewritten by the next chunk
  }
}

// ----------------------------------------------- synthesis on FP64 matrix cores
// The synthesis sums F_par(p, c) = sum_l mu_lm(z_p) a'_c(l) (par = parity of
// l - m) are a contraction over l. One wavefront per (m, group of 64 ring
// pairs); lane q runs the recurrence of pair 64 g + q. Per chunk of 32
// l-steps the wavefront writes mu to its LDS tile (row = l-step, 72 doubles:
// conflict-free operand reads) and accumulates, for each of its 4 tiles of 16
// pairs and each parity, 4 K-steps of 4 l-steps on v_mfma_f64_16x16x4_f64:
//   A[i][k] = mu(l0 + 2 (4 s + k) + par, pair 16 t + i),
//   B[k][j] = a'_{j/2}(l0 + 2 (4 s + k) + par).(re, im),
// up to 8 complex columns (16 real MFMA columns). The blocks of one m run on
// one XCD (workgroup i runs on XCD i mod 8), so the coefficient lines they
// all read stay in that L2. Chunks before the wavefront's first live start
// group are skipped; all products and sums are FP64.
constexpr int kSmRow = 72;       // LDS row stride (doubles) of the mu tile

__global__ __launch_bounds__(64) void k_legendre_synth_mfma(
    int lmax, int mmax, int npairs, int plim, int ncols, int ngroups, const double* __restrict__ pair_z,
    const double* __restrict__ alpha, const int* __restrict__ lst_g, const double2* __restrict__ lst_s,
    const int64_t* __restrict__ mstart, const double2* __restrict__ alms, int64_t alm_stride,
    double2* __restrict__ eo, int64_t eo_stride, const int* __restrict__ pred) {
  if (pred && *pred) return;
  __shared__ double mu_s[kAmChunk * kSmRow];
  const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
  const int g = q % ngroups, m = (q / ngroups) * 8 + xcd;
  if (m > mmax) return;
  const int lane = threadIdx.x;
  const int p = 64 * g + lane;
  const bool ok = p < plim;   // pairs [0, plim) of the npairs (tables have npairs per m)
  const int pp = ok ? p : 0;
  const size_t o = (size_t)m * npairs + pp;
  const double z = pair_z[pp];
  const int gs = ok ? lst_g[o] : kNever;
  const double2 st0 = lst_s[o];
  const int gmin = wave_min(gs);
  const int64_t base = mstart[m];
  const int nsteps = lmax - m + 1;
  const int kq = lane >> 4, jc = lane & 15, col = jc >> 1, ri = jc & 1;
  const bool colok = col < ncols;
  const double* __restrict__ acol = reinterpret_cast<const double*>(alms + (colok ? col : 0) * alm_stride + base) + ri;

  f64x4_t acc[4][2];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t][0] = acc[t][1] = f64x4_t{0.0, 0.0, 0.0, 0.0};
  if (gmin != kNever) {
    double v0 = 0.0, v1 = 0.0;
#pragma unroll 1
    for (int l0 = (gmin * kGroup / kAmChunk) * kAmChunk; l0 < nsteps; l0 += kAmChunk) {
      double al[kAmChunk];   // past the last step: the next m's (or zero padding), times B = 0 below
#pragma unroll
      for (int sp = 0; sp < kAmChunk; ++sp) al[sp] = alpha[base + l0 + sp];
      double b[2][4];
#pragma unroll
      for (int par = 0; par < 2; ++par)
#pragma unroll
        for (int sk = 0; sk < 4; ++sk) {
          const int stp = l0 + 2 * (4 * sk + kq) + par;
          b[par][sk] = (colok && stp < nsteps) ? acol[2 * stp] : 0.0;
        }
#pragma unroll
      for (int sp = 0; sp < kAmChunk; ++sp) {
        if (sp % kGroup == 0 && (l0 + sp) / kGroup == gs) {
          v0 = st0.x;
          v1 = st0.y;
        }
        const double mu = fma(al[sp] * z, v1, -v0);
        v0 = v1;
        v1 = mu;
        mu_s[sp * kSmRow + lane] = mu;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int sk = 0; sk < 4; ++sk)
#pragma unroll
        for (int par = 0; par < 2; ++par)
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const double a = mu_s[(2 * (4 * sk + kq) + par) * kSmRow + 16 * t + jc];
            acc[t][par] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[par][sk], acc[t][par], 0, 0, 0);
          }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // D[i][j] in lane j + 16 (i % 4), register i / 4: pair 64 g + 16 t + i, column j / 2, re/im j % 2
  if (!colok) return;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pr = 64 * g + 16 * t + 4 * r + kq;
      if (pr < plim) {
        double* dst = reinterpret_cast<double*>(eo + col * eo_stride + ((size_t)pr * (mmax + 1) + m) * 2) + ri;
        dst[0] = acc[t][0][r];
        dst[2] = acc[t][1][r];
      }
    }
}

int pick_nr(int n) { return n >= 8 ? 8 : n >= 4 ? 4 : n >= 2 ? 2 : 1; }

template <int NR>
hipError_t synth_pass(const crsht_plan* P, const double2* alms, double2* eo, hipStream_t s) {
  const Geometry& g = P->g;
  dim3 grid((g.mmax + kSynthMT) / kSynthMT, (g.npairs + kSynthBlock - 1) / kSynthBlock);
  const int64_t eo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  timing_begin(P, 0, s);
  hipLaunchKernelGGL(k_legendre_synth<NR>, grid, dim3(kSynthBlock), 0, s, g.lmax, g.mmax, g.npairs, P->t.pair_z,
                     P->t.rec_alpha, P->t.lst_g, P->t.lst_s, P->t.mstart, alms, (int64_t)g.nalm, eo, eo_stride,
                     P->pred);
  timing_end(P, 0, s);
  return hipGetLastError();
}

template <int NR, int RPT>
hipError_t adj_pass_rpt(const crsht_plan* P, const double2* geo, double2* out, bool diag, hipStream_t s) {
  const Geometry& g = P->g;
  const int nb = ((g.mmax + 1 + 31) / 32) * 32;
  const int64_t geo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
  const size_t lds = (size_t)(g.lmax + 1) * sizeof(double);
  if (diag)
    hipLaunchKernelGGL((k_legendre_adj<NR, RPT, MODE_DIAG>), dim3(nb), dim3(kAdjBlock), lds, s, g.lmax, g.mmax,
                       g.npairs, P->t.pair_z, P->t.rec_alpha, P->t.lst_g, P->t.lst_s, P->t.mstart, geo, geo_stride,
                       P->w.ring_w, out, (int64_t)g.nalm, P->pred);
  else
    hipLaunchKernelGGL((k_legendre_adj<NR, RPT, MODE_RAW>), dim3(nb), dim3(kAdjBlock), lds, s, g.lmax, g.mmax,
                       g.npairs, P->t.pair_z, P->t.rec_alpha, P->t.lst_g, P->t.lst_s, P->t.mstart, geo, geo_stride,
                       P->w.ring_w, out, (int64_t)g.nalm, P->pred);
  return hipGetLastError();
}

// ring pairs per thread of the adjoint, and the widest column group that
// keeps the per-thread G values (RPT x NR x 2 complex) within registers
int adj_rpt(const crsht_plan* P) {
  const int r = (P->g.npairs + kAdjBlock - 1) / kAdjBlock;
  return r <= 1 ? 1 : r <= 2 ? 2 : r <= 4 ? 4 : 8;
}
int adj_max_nr(int rpt) { return rpt >= 8 ? 2 : rpt >= 4 ? 4 : 8; }

template <int NR>
hipError_t adj_pass(const crsht_plan* P, const double2* geo, double2* out, bool diag, hipStream_t s) {
  const int rpt = adj_rpt(P);
  if (rpt == 1) return adj_pass_rpt<NR, 1>(P, geo, out, diag, s);
  if (rpt == 2) return adj_pass_rpt<NR, 2>(P, geo, out, diag, s);
  if constexpr (NR <= 4)
    if (rpt == 4) return adj_pass_rpt<NR, 4>(P, geo, out, diag, s);
  if constexpr (NR <= 2)
    if (rpt == 8) return adj_pass_rpt<NR, 8>(P, geo, out, diag, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t legendre_prepare(const crsht_plan* P) {
  (void)P;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_legendre_adj_mfma),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(kAmWaves * 64 * kAmRow * sizeof(double)));
}

hipError_t launch_legendre_start(const crsht_plan* P, hipStream_t s) {
  const Geometry& g = P->g;
  dim3 grid((g.npairs + 255) / 256, g.mmax + 1);
  hipLaunchKernelGGL(k_legendre_start, grid, dim3(256), 0, s, g.lmax, g.mmax, g.npairs, P->t.pair_z, P->t.rec_alpha,
                     P->t.lmm_v, P->t.lmm_k, P->t.mstart, P->t.lst_g, P->t.lst_s);
  return hipGetLastError();
}

hipError_t launch_legendre_synth(const crsht_plan* P, int nrhs, const double2* alms, double2* eo, hipStream_t s) {
  const int64_t eo_stride = (int64_t)P->g.npairs * (P->g.mmax + 1) * 2;
  if (nrhs >= 2) {
    // FP64 matrix cores, 8 columns per launch
    const Geometry& g = P->g;
    const int ngroups = (g.npairs + 63) / 64;
    const int nb = 8 * ngroups * ((g.mmax + 1 + 7) / 8);
    const int cpl = std::max(1, std::min(kAmCols, P->tune.f64_synth_cols));
    // column groups are independent: group k on aux_q(k); timed as a whole
    const int ngrp = (nrhs + cpl - 1) / cpl;
    const int naux = std::min(ngrp - 1, crsht_plan::kAux);
    timing_begin(P, 0, s);
    hipError_t err = aux_fork(P, naux, s);
    for (int c0 = 0; c0 < nrhs && err == hipSuccess; c0 += cpl) {
      const int nc = std::min(cpl, nrhs - c0);
      hipLaunchKernelGGL(k_legendre_synth_mfma, dim3(nb), dim3(64), 0, aux_q(P, c0 / cpl, s), g.lmax, g.mmax,
                         g.npairs, g.npairs, nc, ngroups, P->t.pair_z, P->t.rec_alpha, P->t.lst_g, P->t.lst_s,
                         P->t.mstart, alms + (int64_t)c0 * g.nalm, (int64_t)g.nalm, eo + (int64_t)c0 * eo_stride,
                         eo_stride, P->pred);
      err = hipGetLastError();
    }
    if (err == hipSuccess) err = aux_join(P, naux, s);
    timing_end(P, 0, s);
    return err;
  }
  for (int c0 = 0; c0 < nrhs;) {
    const int nr = pick_nr(nrhs - c0);
    const double2* a = alms + (int64_t)c0 * P->g.nalm;
    double2* e = eo + (int64_t)c0 * eo_stride;
    hipError_t err = nr == 8 ? synth_pass<8>(P, a, e, s)
                   : nr == 4 ? synth_pass<4>(P, a, e, s)
                   : nr == 2 ? synth_pass<2>(P, a, e, s)
                             : synth_pass<1>(P, a, e, s);
    if (err != hipSuccess) return err;
    c0 += nr;
  }
  return hipSuccess;
}

// FP64 matrix-core Legendre sums of the ring pairs [0, plim) only, for the
// polar rings of the T+Q+U mixed path: eo / geo hold plim pairs per column
// (stride eo_stride / geo_stride complex entries); the adjoint adds its sums
// to raw (accumulate) or writes them. nrhs >= 2.
hipError_t launch_legendre_synth_pairs(const crsht_plan* P, int nrhs, const double2* alms, double2* eo,
                                       int64_t eo_stride, int plim, hipStream_t s) {
  const Geometry& g = P->g;
  const int ngroups = (plim + 63) / 64;
  const int nb = 8 * ngroups * ((g.mmax + 1 + 7) / 8);
  for (int c0 = 0; c0 < nrhs; c0 += kAmCols) {
    const int nc = std::min(kAmCols, nrhs - c0);
    hipLaunchKernelGGL(k_legendre_synth_mfma, dim3(nb), dim3(64), 0, s, g.lmax, g.mmax, g.npairs, plim, nc, ngroups,
                       P->t.pair_z, P->t.rec_alpha, P->t.lst_g, P->t.lst_s, P->t.mstart, alms + (int64_t)c0 * g.nalm,
                       (int64_t)g.nalm, eo + (int64_t)c0 * eo_stride, eo_stride, P->pred);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t launch_legendre_adjoint_pairs(const crsht_plan* P, int nrhs, const double2* geo, int64_t geo_stride,
                                         int plim, bool accumulate, double2* raw, hipStream_t s) {
  const Geometry& g = P->g;
  const int nb = ((g.mmax + 1 + 31) / 32) * 32;
  const size_t lds = (size_t)kAmWaves * 64 * kAmRow * sizeof(double);
  for (int c0 = 0; c0 < nrhs; c0 += kAmCols) {
    const int nc = std::min(kAmCols, nrhs - c0);
    for (int p0 = 0; p0 < plim; p0 += kAmPairs) {
      hipLaunchKernelGGL(k_legendre_adj_mfma, dim3(nb), dim3(kAmWaves * 64), lds, s, g.lmax, g.mmax, g.npairs, plim,
                         p0, (accumulate || p0 > 0) ? 1 : 0, nc, P->t.pair_z, P->t.rec_alpha, P->t.lst_g, P->t.lst_s,
                         P->t.mstart, geo + (int64_t)c0 * geo_stride, geo_stride, raw + (int64_t)c0 * g.nalm,
                         (int64_t)g.nalm, P->pred);
      const hipError_t err = hipGetLastError();
      if (err != hipSuccess) return err;
    }
  }
  return hipSuccess;
}

hipError_t launch_legendre_adjoint(const crsht_plan* P, int nrhs, const double2* geo, double2* raw, bool diag,
                                   hipStream_t s) {
  timing_begin(P, 1, s);
  hipError_t err = hipSuccess;
  if (diag) {
    err = adj_pass<1>(P, nullptr, raw, true, s);
  } else if (nrhs >= 2) {
    // FP64 matrix cores, 8 columns and kAmPairs ring pairs per launch
    const Geometry& g = P->g;
    const int64_t geo_stride = (int64_t)g.npairs * (g.mmax + 1) * 2;
    const int nb = ((g.mmax + 1 + 31) / 32) * 32;
    const size_t lds = (size_t)kAmWaves * 64 * kAmRow * sizeof(double);
    const int cpl = std::max(1, std::min(kAmCols, P->tune.f64_adj_cols));
    // column groups are independent: group k on aux_q(k) (the launches over
    // ring pairs of one group stay in order on its stream)
    const int ngrp = (nrhs + cpl - 1) / cpl;
    const int naux = std::min(ngrp - 1, crsht_plan::kAux);
    err = aux_fork(P, naux, s);
    for (int c0 = 0; c0 < nrhs && err == hipSuccess; c0 += cpl) {
      const int nc = std::min(cpl, nrhs - c0);
      hipStream_t q = aux_q(P, c0 / cpl, s);
      for (int p0 = 0; p0 < g.npairs && err == hipSuccess; p0 += kAmPairs) {
        hipLaunchKernelGGL(k_legendre_adj_mfma, dim3(nb), dim3(kAmWaves * 64), lds, q, g.lmax, g.mmax, g.npairs,
                           g.npairs, p0, p0 > 0 ? 1 : 0, nc, P->t.pair_z, P->t.rec_alpha, P->t.lst_g, P->t.lst_s, P->t.mstart,
                           geo + (int64_t)c0 * geo_stride, geo_stride, raw + (int64_t)c0 * g.nalm, (int64_t)g.nalm,
                           P->pred);
        err = hipGetLastError();
      }
    }
    if (err == hipSuccess) err = aux_join(P, naux, s);
  } else {
    const int64_t geo_stride = (int64_t)P->g.npairs * (P->g.mmax + 1) * 2;
    const int nr_cap = adj_max_nr(adj_rpt(P));
    for (int c0 = 0; c0 < nrhs && err == hipSuccess;) {
      int nr = pick_nr(nrhs - c0);
      if (nr > nr_cap) nr = nr_cap;
      const double2* gi = geo + (int64_t)c0 * geo_stride;
      double2* oo = raw + (int64_t)c0 * P->g.nalm;
      err = nr == 8 ? adj_pass<8>(P, gi, oo, false, s)
          : nr == 4 ? adj_pass<4>(P, gi, oo, false, s)
          : nr == 2 ? adj_pass<2>(P, gi, oo, false, s)
                    : adj_pass<1>(P, gi, oo, false, s);
      c0 += nr;
    }
  }
  timing_end(P, 1, s);
  return err;
}

}  // namespace crsht
