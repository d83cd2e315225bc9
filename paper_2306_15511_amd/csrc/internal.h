// Internal declarations shared by the translation units of libcrsht.
// Nothing here is part of the public C ABI (include/crsht.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <utility>
#include <vector>

#include "../../include/crsht.h"

namespace crsht {

// Underflow handling of the Legendre recurrence. A recurrence value is carried
// as v * 2^(kScaleBits * k) with an integer k <= 0. While k < 0 the true value
// is below 2^-100 (|v| <= 2^500) and contributes nothing at double precision;
// each time |v| exceeds 2^500 the pair (v_{l-1}, v_l) is multiplied by
// 2^-kScaleBits and k grows by one. At k == 0 the value is an ordinary double.
constexpr int kScaleBits = 600;
constexpr double kRescaleAbove = 0x1p500;     // |v| above this triggers rescaling
constexpr double kRescaleBy = 0x1p-600;       // 2^-kScaleBits
// l - m steps per group of the start table (lst_g counts groups): a ring pair
// contributes at m iff its first live group g satisfies g <= (lmax - m) / kStartGroup
constexpr int kStartGroup = 16;

// Sizes of a plan.
struct Geometry {
  int nside = 0, lmax = 0, mmax = 0;
  int nrings = 0;     // 4 nside - 1
  int npairs = 0;     // 2 nside: north ring i and its mirror 4 nside - i; the equator is paired with itself
  int64_t npix = 0;
  int64_t nalm = 0;   // stored complex coefficients, m-major
  int fft_max = 0;    // largest FFT length used by the ring kernels (power of two)
};

// Device-resident tables of a plan (all owned by the plan).
struct Tables {
  // per ring pair p (index 0 .. npairs-1; north ring index p, south ring nrings-1-p)
  double* pair_z = nullptr;        // cos(theta) of the north ring
  int* pair_nphi = nullptr;        // pixels per ring
  double* pair_phi0 = nullptr;     // azimuth of the first pixel
  int64_t* pair_first_n = nullptr; // first pixel of the north ring
  int64_t* pair_first_s = nullptr; // first pixel of the south ring (== north for the equator)
  int* pair_fft_len = nullptr;     // FFT length: nphi if a power of two, else Bluestein length
  int64_t* pair_bs_off = nullptr;  // offset into bs_chirp (nphi entries) / bs_kern (fft_len entries); -1 if unused
  int64_t* pair_bk_off = nullptr;
  double2* bs_chirp = nullptr;     // exp(-i pi j^2 / n), j < n
  double2* bs_kern = nullptr;      // FFT of the conjugate chirp filter, scaled by 1/L
  double2* twiddle = nullptr;      // exp(-2 pi i j / fft_max), j < fft_max
  float2* bs_chirp32 = nullptr;    // the same three tables rounded to float (mixed-precision ring pass)
  float2* bs_kern32 = nullptr;
  float2* twiddle32 = nullptr;
  int* ring_pairs = nullptr;       // ring pairs grouped by FFT-length class (RingClass::off, count)

  // Legendre recurrence (scaled form mu_l = lambda_l / kappa_l):
  //   mu_m = lambda_mm, mu_{m-1} = 0, mu_l = alpha_lm z mu_{l-1} - mu_{l-2} for l > m
  double* rec_alpha = nullptr;     // [nalm + 32] alpha_lm (index of (l,m)); alpha_{m+1,m} = 1, alpha_mm unused; 32 zeros after
  double* rec_kappa = nullptr;     // [nalm] kappa_lm, lambda_lm = kappa_lm mu_lm
  double* lmm_v = nullptr;         // [mmax+1][npairs] start value mantissa
  int* lmm_k = nullptr;            // [mmax+1][npairs] start scale index k <= 0
  int* lst_g = nullptr;            // [mmax+1][npairs] first live group of 16 steps (INT_MAX: never)
  int* pair_mtop = nullptr;        // [npairs] largest m at which the pair's recurrence starts by l = lmax:
                                   // above it lambda_lm of the pair stays 0 for every l
  int64_t live_pair_m = 0;         // sum over pairs of pair_mtop + 1
  double2* lst_s = nullptr;        // [mmax+1][npairs] (mu_{l-2}, mu_{l-1}) at the start of that group
  int64_t* mstart = nullptr;       // [mmax+2] index of a_{m,m}; mstart[mmax+1] = nalm
  double* ones = nullptr;          // [nalm] 1.0
  // mixed-precision (MFMA) Legendre step
  int64_t* mx_cstart = nullptr;    // [mmax+2] first 32-step synthesis chunk of each m
  int64_t* mx_tstart = nullptr;    // [mmax+2] first 64-step adjoint tile of each m
  int* mx_tile_m = nullptr;        // [ntiles] m of each adjoint tile
  int* mx_order = nullptr;         // [8][mx_maxq] adjoint tile of (XCD, slot), -1 past the end
  int mx_maxq = 0;
  double2* mx_ckpt = nullptr;      // [ntiles][npairs] recurrence state at each tile start
  int64_t mx_ntiles = 0;
  int* idx_l = nullptr;            // [nalm] l of each stored coefficient
  int* idx_m = nullptr;            // [nalm] m of each stored coefficient
  int* idx_mv = nullptr;           // [ncomp * nalm] m of each element of a solver vector
};

// Ring pairs of one FFT-length class: t.ring_pairs[off .. off + count) all have
// an FFT length <= L (L is a power of two; the ring kernel's LDS and block size).
struct RingClass {
  int L = 0, off = 0, count = 0;
};

// Run-time tile choices of a plan (crsht_autotune): threads per workgroup of
// the ring pass per FFT-length class (L / ring_div[k], ring_div 8 or 4), and
// complex columns per launch of the FP64 matrix-core Legendre kernels (2, 4
// or 8). The defaults are the shapes the kernels were written around.
constexpr int kMaxRingClasses = 8;
struct Tuning {
  int ring_div[kMaxRingClasses] = {8, 8, 8, 8, 8, 8, 8, 8};
  int f64_synth_cols = 8;
  int f64_adj_cols = 8;
};

// Workspace, allocated once at plan creation for nrhs_max columns.
struct Workspace {
  double2* eo = nullptr;       // [nrhs][npairs][mmax+1][2]  (E, O) Legendre sums (float2 in the mixed path)
  double2* geo = nullptr;      // [nrhs][npairs][mmax+1][2]  (G_N + G_S, G_N - G_S) (float2 in the mixed path)
  double2* alm_a = nullptr;    // [nrhs][nalm] scratch a_lm vectors
  double2* alm_b = nullptr;
  double2* cg_x = nullptr, *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_q = nullptr, *cg_b = nullptr;
  double2* cg_d = nullptr;     // refinement correction
  double2* alm_c = nullptr;    // [nalm] joint-move mean field at the proposal
  double2* alm_d = nullptr;    // [nalm] joint-move rescaled fluctuation
  double* map_a = nullptr;     // [nrhs][npix] scratch maps
  double* ring_w = nullptr;    // [npairs] ring sums of N^-1 (north + south)
  double* diag = nullptr;      // [nalm] Jacobi diagonal D_lm
  double* sinv = nullptr;      // [nalm] 1/C_l on kept modes, 0 otherwise
  double* sinvhalf = nullptr;  // [nalm] C_l^-1/2
  double* bk = nullptr;        // [ncomp * nalm] b_l kappa_lm on kept modes (repeated per component)
  double* bl_keep = nullptr;   // [nalm] b_l on kept modes
  double* sblk = nullptr;      // [lmax+1][8] T+Q+U: S^-1 (TT, TE, EE, BB) and S^-1/2 (TT, TE, EE, BB)
  double* perl = nullptr;      // [4][lmax+1] per-l 1/C_l, C_l^-1/2, b_l, keep (device)
  double* partial = nullptr;   // [nrhs][npart] block partial sums
  double* scal = nullptr;      // [nrhs][kScalSlots] CG scalars
  double* host_scal = nullptr; // pinned mirror of scal
  double2* cg_xacc = nullptr;  // [nrhs][nalm] refinement: accumulated solution
  double2* cg_bin = nullptr;   // [nrhs][nalm] refinement: right-hand side of the inner solve
  int* bin_edges = nullptr;    // [lmax+2] multipole bin edges of a gradient call
  double* bin_part = nullptr;  // [lmax+1][kBinSlices][3] per-bin partial sums
  double* bin_grad = nullptr;  // [lmax+1] per-bin gradient
  double* lfac = nullptr;      // [lmax+1] per-l factors (fluctuation rescaling of a bin move)
  double2* camp = nullptr;     // [nrhs_max] per-column (1/amp, 1/sqrt(amp)) of the problem's S^-1, S^-1/2
  int* ctl = nullptr;          // [kCtlSlots] control block of a device-driven solve
  int* host_exited = nullptr;  // pinned, device-visible: set to 1 by the device once the solve has stopped
  void* dstats = nullptr;      // [nrhs_max] cr_stats written by a device-driven solve (cr_solve_batched)
  void* mx_ab = nullptr;       // bf16 synthesis operand tiles (one group of kMixedCols columns)
  void* mx_ag = nullptr;       // bf16 adjoint operand tiles
  double* adj_part = nullptr;  // [nrhs_max][mixed adjoint tiles] partials of <p, q> (fused adjoint)
  double2* pol = nullptr;      // T+Q+U: [nrhs][9][npol][mmax+1][2] FP64 Legendre sums of the polar ring pairs
  int npart = 0;
};

constexpr int kScalSlots = 24;
constexpr int kBinSlices = 16;   // m slices per multipole bin in the gradient reductions
// T+Q+U mixed transforms: ring pairs with sin^2 theta below this take FP64
// Legendre sums (their Q, U spectra divide cancelling sums by sin^2 theta,
// which magnifies the split-bf16 rounding by up to 3 Nside^2)
constexpr double kPolarSin2 = 0.01;
constexpr int kMixedCols = 32;   // MFMA N: 16 right-hand sides (re, im) per column group
constexpr int kMaxGroups = 2;    // column groups sharing one recurrence pass of an MFMA synthesis launch
constexpr int kAdjGroups = 1;    // column groups per MFMA adjoint launch
// slots of the per-column scalar block
enum ScalSlot {
  S_RZ = 0,      // <r, z>
  S_PQ = 1,      // <p, A p>
  S_ALPHA = 2,
  S_BETA = 3,
  S_RR = 4,      // <r, r>
  S_BB = 5,      // <b, b>
  S_DONE = 6,    // 1 when the column has converged (or broken down)
  S_REL = 7,     // last relative residual
  S_ITERS = 8,   // iterations taken
  S_BREAK = 9,   // 1 on breakdown
  S_RZ_PREV = 10,  // <r, z> of the previous iteration (beta after a residual replacement)
  S_AUX0 = 11,
  S_AUX1 = 12,
  S_AUX2 = 13,
  S_RESTART = 14,  // host flag: the next replacement restarts the direction (beta = 0)
  // device-driven solve (dsolve.hip): per-column state of the refinement
  S_TRIG = 15,     // the column asked for the current residual replacement
  S_LAST = 16,     // true relative residual at the last replacement (1 before the first)
  S_REFINE = 17,   // residual replacements of the column
  S_TRUE = 18,     // last true relative residual
  // mixed-precision T iteration: the x += alpha p of the last update, still
  // to be applied (by the next direction update, which reads that p, or by
  // launch_x_flush before x is used); 0 when none is pending
  S_XA = 19,
};

// Control block of a device-driven solve (int32, plan workspace w.ctl).
// The C_SKIP_* words are the predicates of the enqueued sections: the
// kernels of a section return at once while their word is non-zero.
enum CtlSlot {
  C_SKIP_ITER = 0,   // block of PCG iterations (all columns finished or the solve exited)
  C_SKIP_REPL = 1,   // FP64 true residual of a replacement (not needed at this check)
  C_SKIP_TAIL = 2,   // z, <r,z> and beta from the replaced residual
  C_SKIP_FINAL = 3,  // FP64 true residual at exit (the last one is current)
  C_IT = 4,          // iterations done
  C_NREP = 5,        // replacements done
  C_FRESH = 6,       // the true residuals are those of the current x
  C_PENDING = 7,     // a direction update is pending (after the first block)
  C_EXITED = 8,      // the solve has stopped; later sections are skipped
  C_SKIP_REPL_LOW = 9,  // residual of a replacement with the bf16x6 operator (not needed at this check)
  C_LOW = 10,        // the last replacement used the bf16x6 operator
  kCtlSlots = 16
};
// mixed refinement: an intermediate residual replacement (no column claims
// convergence, every open column's recursive residual at least this) uses
// the bf16x6 operator (relative error about 5e-7) instead of FP64
constexpr double kLowReplaceFloor = 5e-5;
// modes of the control kernel k_dctl
enum DctlMode { DC_INIT = 0, DC_CHECK = 1, DC_AFTER_REPL = 2, DC_PRE_BLOCK = 3, DC_AFTER_BLOCK = 4, DC_FINAL_PRE = 5,
                DC_FINAL_POST = 6 };
struct DctlArgs {
  int nrhs;
  double tol;        // target relative true residual
  double itol;       // replacement each time the recursive residual fell by this factor (0: at convergence only)
  int maxref;        // maximum replacements
  int maxiter;       // iterations
  int every;         // iterations per enqueued block
  int f64;           // stats report no replacements (plain FP64 form)
};

// 0 FP64 Legendre synthesis, 1 FP64 Legendre adjoint, 2 fused ring pass
// (FP32, mixed path), 3 MFMA (bf16x3) Legendre synthesis, 4 MFMA Legendre
// adjoint, 5 block preconditioner application, 6 fused ring pass (FP64)
constexpr int kTimedKernels = 7;
struct Timing {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events[kTimedKernels];
  hipEvent_t open[kTimedKernels] = {};
  hipEvent_t open_end[kTimedKernels] = {};
  double total_ms[kTimedKernels] = {};
  int64_t count[kTimedKernels] = {};
};

}  // namespace crsht

namespace crsht {
// Per-m block preconditioner (blockpc.hip): for each (m, parity q of l - m)
// block of n rows l = m + q + 2 i, the inverse M^-1 = S C S with S =
// diag(sqrt(M^-1_ii)): C (unit diagonal, |C_ij| <= 1) stored in FP16, full
// symmetric, at inv + boff[b], and sqrt(M^-1_ii) in FP32 per vector element
// (scale); application tasks cover 128 rows of both parity blocks of one m
// (task_b: even block, task_b1: odd block or -1).
struct BlockPC {
  bool built = false;
  int lmin = 0;
  int nblocks = 0, ntasks = 0;
  int64_t inv_elems = 0;     // floats of storage (every block sized for FP32)
  int64_t stored_bytes = 0;  // bytes of the n x n entries of the stored inverses
  int nhalf = 0;             // blocks stored in FP16
  float* inv = nullptr;      // Jacobi-scaled inverses of the FP32 blocks ([n][pc_ld(n)] at float offset boff)
  _Float16* inv16 = nullptr; // those of the FP16 blocks in MFMA operand tiles (from element boff16)
  int64_t* boff16 = nullptr; // element offset of each block's FP16 tiles
  float* scale = nullptr;    // [ncomp * nalm] sqrt of the inverse's diagonal, per vector element
  int* bhalf = nullptr;      // per block: 1 if stored in FP16
  double* part = nullptr;    // [nrhs_max][ntasks] partials of <r, z> written by the application
  int *bm = nullptr, *bq = nullptr, *bn = nullptr;
  int64_t* boff = nullptr;   // float offset of each stored inverse
  int64_t* be0 = nullptr;    // vector element of row 0 of each block (component offset included)
  int *task_b = nullptr, *task_b1 = nullptr, *task_r0 = nullptr;
};

// identity of a captured PCG iteration block: replayed only for the same
// launch sequence and arguments
struct GraphKey {
  int kind = -1;            // 0: FP64 PCG block, 1: mixed PCG block
  int nrhs = 0, n = 0;      // columns, iterations in the block
  int first_update = 0;     // mixed: the block starts with a pending direction update
  int pc = 0;               // block preconditioner in use
  const void* ninv = nullptr;
  double tol = 0.0;
  double itol = 0.0;        // device-driven solve: replacement factor, replacement and iteration limits
  int maxref = 0, maxiter = 0;
  bool aux_off = false;     // captured without forked launches (batched solve)
  bool operator==(const GraphKey& o) const {
    return kind == o.kind && nrhs == o.nrhs && n == o.n && first_update == o.first_update && pc == o.pc &&
           ninv == o.ninv && tol == o.tol && itol == o.itol && maxref == o.maxref && maxiter == o.maxiter &&
           aux_off == o.aux_off;
  }
};
}  // namespace crsht

struct crsht_plan {
  crsht::Geometry g;
  // predicate of the solve kernels: while non-null, every kernel of the PCG
  // loop (operator, preconditioner, vector updates, reductions) returns at
  // once when *pred != 0. Set only while a device-driven solve enqueues its
  // predicated sections (dsolve.hip); null otherwise.
  mutable const int* pred = nullptr;
  // bf16 parts per operand of the mixed Legendre transforms: 2 (bf16x3
  // products, the PCG inner operator) or 3 (bf16x6, the CR_BF16X6 transforms);
  // set only for the duration of a CR_BF16X6 call
  mutable int mx_split = 2;
  // pinned staging of the per-call host data (spectra, beam, column
  // amplitudes): slot k is reused only after the copies last enqueued from it
  // have run (event k), so no call has to synchronise its stream
  static constexpr int kStageSlots = 4;
  void* stage_host[kStageSlots] = {};
  hipEvent_t stage_ev[kStageSlots] = {};
  bool stage_used[kStageSlots] = {};
  int stage_next = 0;
  size_t stage_bytes = 0;
  // captured super-steps of the device-driven solve (first block, later blocks)
  hipGraphExec_t dgraph[2] = {};
  crsht::GraphKey dgraph_key;
  // cr_solve_batched: the plan's problem runs on its own stream (created with
  // the plan), forked from and joined to the caller's stream by events; a
  // ring of events paces the enqueued blocks against the device
  hipStream_t exec_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  static constexpr int kRoundEvents = 3;
  hipEvent_t ev_round[kRoundEvents] = {};
  hipStream_t cap_stream = nullptr;     // stream used only to capture iteration blocks
  // independent launches of one operation (ring-pass FFT-length classes,
  // FP64 adjoint column groups) after the first run on these streams,
  // forked from and joined back to the caller's stream (aux_fork / aux_join)
  static constexpr int kAux = 3;
  // set while a batched solve runs the plan (its problems already run
  // concurrently on their own streams): no forks then
  mutable bool aux_off = false;
  hipStream_t aux_stream[kAux] = {};
  hipEvent_t aux_fork_ev = nullptr, aux_join_ev[kAux] = {};
  hipGraphExec_t graph_exec = nullptr;  // last captured block
  crsht::GraphKey graph_key;
  crsht::BlockPC pc;                    // per-m block preconditioner (built on request)
  int ncomp = 1;
  // T+Q+U: ring pairs [0, npol) (sin^2 theta below kPolarSin2) take FP64
  // Legendre sums in the mixed transforms
  int npol = 0;
  int nrhs_max = 1;
  int device = 0;
  int64_t workspace_bytes_ = 0;
  crsht::Tables t;
  crsht::Workspace w;
  crsht::Timing timing;
  crsht::Tuning tune;
  std::vector<crsht::RingClass> ring_cls;
  // host copies used for argument checks and bookkeeping
  std::vector<int> h_nphi;
  std::vector<int64_t> h_first;
  std::vector<double> h_z, h_phi0;
};

namespace crsht {

// elements of one solver vector column: ncomp blocks of nalm coefficients
inline int64_t vlen(const crsht_plan* P) { return (int64_t)P->ncomp * P->g.nalm; }

// element access of a solver vector stored as double2 or as float2 (the
// preconditioned residual z of the mixed-precision T iteration, at the start
// of its buffer with the same element index); zstore returns the value as
// stored, so that dot products use what later kernels read
__device__ __forceinline__ double2 zload(const double2* p) { return *p; }
__device__ __forceinline__ double2 zload(const float2* p) {
  const float2 v = *p;
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ double2 zstore(double2* p, double2 v) {
  *p = v;
  return v;
}
__device__ __forceinline__ double2 zstore(float2* p, double2 v) {
  const float2 f = make_float2((float)v.x, (float)v.y);
  *p = f;
  return make_double2(f.x, f.y);
}

// ---- timing (timing.cpp) ----
void timing_begin(const crsht_plan* P, int id, hipStream_t s);
void timing_end(const crsht_plan* P, int id, hipStream_t s);
void timing_clear(crsht_plan* P);

// ---- Legendre step (legendre.hip) ----
// Start tables (setup, once per plan): see k_legendre_start.
hipError_t launch_legendre_start(const crsht_plan* P, hipStream_t s);
// Synthesis: eo[c][p][m] = (E, O) with E/O the sums over l of even/odd (l-m)
// of mu_lm(z_p) * alms[c][idx(l,m)], alms already multiplied by kappa (and
// whatever diagonal factor the caller folds in).
hipError_t launch_legendre_synth(const crsht_plan* P, int nrhs, const double2* alms, double2* eo,
                                 hipStream_t s);
// FP64 matrix-core sums over the ring pairs [0, plim) only (eo / geo hold plim
// pairs per column, column stride in complex entries; nrhs columns of any
// count); the adjoint adds to raw when accumulate.
hipError_t launch_legendre_synth_pairs(const crsht_plan* P, int nrhs, const double2* alms, double2* eo,
                                       int64_t eo_stride, int plim, hipStream_t s);
hipError_t launch_legendre_adjoint_pairs(const crsht_plan* P, int nrhs, const double2* geo, int64_t geo_stride,
                                         int plim, bool accumulate, double2* raw, hipStream_t s);
// Adjoint: raw[c][idx(l,m)] = sum_p mu_lm(z_p) * (G_E or G_O by parity)[c][p][m]
// (no kappa, no other factor). diag: raw[idx].x = sum_p mu_lm(z_p)^2 W_p with
// W_p = w.ring_w[p] (the preconditioner pass; geo unused, one column).
hipError_t launch_legendre_adjoint(const crsht_plan* P, int nrhs, const double2* geo, double2* raw, bool diag,
                                   hipStream_t s);

// ---- mixed-precision Legendre step (legendre_mfma.hip) ----
int64_t mixed_ab_bytes(const Geometry& g);
int64_t mixed_ag_bytes(const Geometry& g);
void mixed_starts(const Geometry& g, std::vector<int64_t>& cst, std::vector<int64_t>& tst, std::vector<int>& tm,
                  std::vector<int>& order, int& maxq);
hipError_t launch_checkpoints(const crsht_plan* P, hipStream_t s);
// eo = (E, O) sums (float2) with mu (FP64 recurrence) and f * alm rounded to
// bf16x3, FP32 accumulation; f == nullptr means 1
hipError_t launch_legendre_synth_mixed(const crsht_plan* P, int nrhs, const double2* alm, const double* f,
                                       float2* eo, hipStream_t s);
// the same inside PCG: p = z + beta p per column (scalars in w.scal; skipped
// for done columns or when !update) fused with the operand preparation, then
// eo from bk * p
// x (optional): first x += scal[S_XA] p per column, the pending solution
// update of the last iteration (with p before its update)
hipError_t launch_legendre_synth_mixed_cg(const crsht_plan* P, int nrhs, const double2* z, double2* p, bool update,
                                          float2* eo, hipStream_t s, bool z32 = false, double2* x = nullptr);
// raw sums as launch_legendre_adjoint (non-diag) from float2 geo, bf16x3 /
// FP32 accumulation
// T plans, PCG: the bf16x3 adjoint fused with q = camp.x sinv p + bk raw,
// stored as FP32 ([nrhs][nalm] float2), and the per-tile partials of <p, q>
// of the stored q (w.adj_part, [nrhs][t.mx_ntiles])
hipError_t launch_legendre_adjoint_mixed_q(const crsht_plan* P, int nrhs, const float2* geo, const double2* p,
                                           float2* q, hipStream_t s);
hipError_t launch_legendre_adjoint_mixed(const crsht_plan* P, int nrhs, const float2* geo, double2* raw,
                                         hipStream_t s);

// ---- ring step (ring.hip) ----
// mode SYNTH: eo -> map;  ADJOINT: map -> geo;  FUSED: eo -> (map * ninv) -> geo
// eo / geo are double2 arrays, or float2 arrays with f32 (maps and N^-1 FP64)
enum RingMode { RING_SYNTH = 0, RING_ADJOINT = 1, RING_FUSED = 2 };
// Column layout of a ring launch: logical column c (maps c * npix) is
// component k = c % group of group c / group; its Legendre sums are column
// (c / group) * eo_cols + k of eo, (c / group) * geo_cols + k of geo, and its
// N^-1 is ninv + k * ninv_stride. The default is one plain column per map.
struct RingCols {
  int group = 1, eo_cols = 1, geo_cols = 1;
  int64_t ninv_stride = 0;
  // per ring pair, the largest m the pass reads and writes (t.pair_mtop), or
  // null for all m: launch_ring sets it for the FP32 fused pass of T plans,
  // whose consumer (k_prep_adj) reads no m above it
  const int* mtop = nullptr;
};
hipError_t launch_ring(const crsht_plan* P, int nrhs, RingMode mode, const void* eo, double* map,
                       const double* ninv, void* geo, bool f32, hipStream_t s, RingCols cols = RingCols());
void ring_classes(const std::vector<int>& fft_len, std::vector<RingClass>& cls, std::vector<int>& pairs);
// the auxiliary streams 0 .. n - 1 wait for the work so far on s; aux_join:
// s waits for them; aux_q(k): s for k = 0, else auxiliary stream (k - 1) mod kAux
hipError_t aux_fork(const crsht_plan* P, int n, hipStream_t s);
hipError_t aux_join(const crsht_plan* P, int n, hipStream_t s);
hipStream_t aux_q(const crsht_plan* P, int k, hipStream_t s);
// plan set-up: allow the dynamic LDS of the ring kernels the plan's classes need
hipError_t ring_prepare(const crsht_plan* P);
// once per plan: LDS limit of the FP64 matrix-core adjoint
hipError_t legendre_prepare(const crsht_plan* P);
size_t ring_lds_bytes(const crsht_plan* P, bool f32);
// threads per workgroup of ring class k under the plan's tuning
int ring_class_threads(const crsht_plan* P, int k);

// ---- spin-2 part of T+Q+U plans (pol.hip) ----
// alm [nrhs][3][nalm] (times f per element, may be null) -> 9 scalar
// coefficient columns per T+Q+U column [nrhs][9][nalm] (kappa folded in)
hipError_t launch_pol_prep_synth(const crsht_plan* P, int nrhs, const double2* alm, const double* f, double2* out,
                                 hipStream_t s);
// Legendre sums of the 9 columns -> Q, U spectra over group columns 1, 2
// (npairs < 0: all ring pairs; else a buffer of the first npairs pairs)
hipError_t launch_pol_combine_synth(const crsht_plan* P, int nrhs, void* eo, bool f32, hipStream_t s,
                                    int npairs = -1);
// azimuthal adjoints of Q, U (group columns 1, 2 of 7) -> weighted copies in 3..6
hipError_t launch_pol_pre_adjoint(const crsht_plan* P, int nrhs, void* geo, bool f32, hipStream_t s,
                                  int npairs = -1);
// polar ring pairs [0, npol) of the mixed T+Q+U transforms (FP64 in w.pol):
// T, Q, U spectra of the polar pairs -> float2 eo (group columns 0..2 of 9)
hipError_t launch_polar_spectra_to_f32(const crsht_plan* P, int nrhs, const double2* pol64, float2* eo,
                                       hipStream_t s);
// float2 azimuthal adjoints T, Q, U of the polar pairs -> FP64 pol64 (group
// columns 0..2 of 7), and those float2 entries set to 0
hipError_t launch_polar_geo_to_f64(const crsht_plan* P, int nrhs, float2* geo, double2* pol64, hipStream_t s);
// raw Legendre adjoints [nrhs][7][nalm] -> f * (a_T, a_E, a_B) [nrhs][3][nalm]
hipError_t launch_pol_combine_adjoint(const crsht_plan* P, int nrhs, const double2* raw, const double* f,
                                      double2* out, hipStream_t s);
// per-element problem arrays of a T+Q+U plan from w.sblk and the b_l / keep
// rows of perl: sinv, sinvhalf = diagonals of the blocks, bk = b_l kappa_lm
// (x3), bl_keep = b_l on kept modes
hipError_t launch_expand_tqu(const crsht_plan* P, const double* perl, hipStream_t s);
// q = S^-1 p + dterm (3x3 blocks; S^-1 omitted without prior); partial <p, q>
hipError_t launch_cg_q_tqu(const crsht_plan* P, int nrhs, const double2* p, const double2* dterm, double2* q,
                           hipStream_t s, bool prior = true);
hipError_t launch_rhs_finish_tqu(const crsht_plan* P, int nrhs, const double2* dterm, const double2* w0,
                                 double2* out, hipStream_t s);
hipError_t launch_diag_tqu(const crsht_plan* P, const double2* rawt, const double2* rawp, double* diag,
                           hipStream_t s);

// ---- per-m block preconditioner (blockpc.hip) ----
// build from the per-l arrays that set_problem left in the workspace (b_l
// and the priors) and N^-1 (device, [ncomp][npix]); allocates the plan's
// preconditioner storage; CR_EINVAL if a block is not positive definite
int block_pc_build(crsht_plan* P, int lmin, const double* ninv, hipStream_t s);
void block_pc_free(BlockPC& pc);
// z = M^-1 r per column (r, z: [nrhs][vlen])
// with dots, also the per-task partials of <r, z> into pc.part ([nrhs][ntasks]);
// z32: z stored as float2 at the start of the z buffer (zstore)
hipError_t launch_pc_apply(const crsht_plan* P, int nrhs, const double2* r, double2* z, hipStream_t s,
                           bool dots = false, bool z32 = false);
// partial <r, z> (row 0) and, with rr, <r, r> (row 1), nb = vec_reduce_blocks
hipError_t launch_pc_dots(const crsht_plan* P, int nrhs, const double2* r, const double2* z, bool rr,
                          hipStream_t s, bool z32 = false);

// ---- allocation-free synthesis (noalloc.hip) ----
// device address of the static scratch on `device` (current), once per device
int noalloc_setup(int device);

// ---- device-driven solve control (dsolve.hip) ----
// stats: device cr_stats [nrhs] (written by DC_FINAL_POST), may be null for other modes
hipError_t launch_dctl(const crsht_plan* P, int mode, const DctlArgs& a, void* stats_dev, hipStream_t s);

// ---- vector kernels (vec.hip) ----
// Reductions write per-block partial sums to w.partial (column c, row r at
// partial[(c * 4 + r) * npart + block]) and a one-block kernel sums them.
int vec_reduce_blocks(const crsht_plan* P);
hipError_t launch_expand(const crsht_plan* P, const double* perl, hipStream_t s);
hipError_t launch_scale_alm(const crsht_plan* P, int nrhs, const double2* in, const double* f, double2* out,
                            hipStream_t s);
// w[p] = scale * ring sums of ninv (+ ninv2 when given) over both rings of pair p
hipError_t launch_ring_weights(const crsht_plan* P, const double* ninv, double* w, hipStream_t s,
                               const double* ninv2 = nullptr, double scale = 1.0);
hipError_t launch_pix_rhs(const crsht_plan* P, int nrhs, const double* ninv, const double* d, const double* w1,
                          double* u, hipStream_t s);
hipError_t launch_rhs_finish(const crsht_plan* P, int nrhs, const double2* raw, const double2* w0, double2* out,
                             hipStream_t s);
// q = sinv * p + bk * raw per column (sinv term omitted when w.sinv is not
// passed, see operator_core); partial <p, q> per block (row 0)
hipError_t launch_cg_q(const crsht_plan* P, int nrhs, const double2* p, const double2* raw, double2* q,
                       hipStream_t s, bool prior = true);
// D = sinv + bk^2 * raw.x on kept modes, 1 elsewhere
hipError_t launch_diag(const crsht_plan* P, const double2* raw, double* diag, hipStream_t s);
hipError_t launch_project(const crsht_plan* P, int nrhs, const double2* x, double2* out, hipStream_t s);
hipError_t launch_map_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out,
                            hipStream_t s);
hipError_t launch_alm_axpby(int64_t n, double a, const double2* x, double b, const double2* y, double2* out,
                            hipStream_t s);
// zgiven: z already holds the preconditioned residual (block preconditioner),
// as float2 with z32
hipError_t launch_cg_start(const crsht_plan* P, int nrhs, const double2* b, const double2* r, double2* z,
                           double2* p, double2* pt, hipStream_t s, bool zgiven = false, bool z32 = false);
// part0 (optional): row 0 (<r, z>) comes from part0[c * n0 + i], i < n0,
// instead of the block partials (the block preconditioner's own partials)
hipError_t launch_cg_scalars(const crsht_plan* P, int nrhs, int what, int nb, double tol, int restart,
                             hipStream_t s, const double* part0 = nullptr, int n0 = 0);
// noz == false: z = r / D with <r, z> in row 0; true: z untouched, row 0 = 0
// (the block preconditioner follows, with its own <r, z> partials). q32:
// q is read as FP32 from there instead of q, and x is not touched: alpha
// (0 for columns that were done) goes to scal[S_XA] for the next direction
// update (the mixed T iteration)
hipError_t launch_cg_update(const crsht_plan* P, int nrhs, double2* x, double2* r, double2* z, const double2* p,
                            const double2* q, hipStream_t s, bool noz = false, const float2* q32 = nullptr);
// x += scal[S_XA] p per column, then scal[S_XA] = 0 (the pending solution
// update of the mixed T iteration, before x is read)
hipError_t launch_x_flush(const crsht_plan* P, int nrhs, hipStream_t s);
hipError_t launch_cg_replace(const crsht_plan* P, int nrhs, const double2* r, double2* z, hipStream_t s);
hipError_t launch_cg_pupdate(const crsht_plan* P, int nrhs, const double2* z, double2* p, double2* pt,
                             hipStream_t s);
hipError_t launch_residual(const crsht_plan* P, int nrhs, const double2* b, const double2* ax, double2* r,
                           hipStream_t s);
hipError_t launch_sum_rows(const crsht_plan* P, int nrhs, int nb, hipStream_t s);
// u = N^-1 (d - m) per column
hipError_t launch_pix_wres(const crsht_plan* P, int nrhs, const double* ninv, const double* d, const double* m,
                           double* u, hipStream_t s);
// a *= w_m (2 for m > 0), Im a_l0 = 0, in place
hipError_t launch_mweight(const crsht_plan* P, int nrhs, double2* a, hipStream_t s);
// grad[k] = <a,S^-1_k a>/2 + <lam,S^-1/2_k w0>/2 - <lam,S^-1_k f> for the bins of
// edges (device, nbins + 1 entries); w0 may be null
// per-bin d ln pi / d theta_k; mode 0: at fixed w0, w1 (lam = A^-1 M f);
// mode 1: at fixed whitened fluctuation (lam = M f, w0 unused); mode 2: the
// per-bin a^T S^-1_k a alone
hipError_t launch_bin_grad(const crsht_plan* P, int nbins, const int* edges, const double2* ahat,
                           const double2* fhat, const double2* lam, const double2* w0, double* grad,
                           hipStream_t s, int mode = 0);
// d ln pi / d theta_k = <x1,y1>_k/2 + <x2,y2>_k/2 - <x3,y3>_k per bin over all
// components (T+Q+U: x1 = a, y1 = S^-1 a, x2 = lam, y2 = S^-1/2 w0, x3 = lam,
// y3 = S^-1 f); x2 or y2 may be null
hipError_t launch_bin_grad_dots(const crsht_plan* P, int nbins, const int* edges, const double2* x1,
                                const double2* y1, const double2* x2, const double2* y2, const double2* x3,
                                const double2* y3, double* grad, hipStream_t s);
// partials of a^T S^-1 a with the 3x3 blocks of a T+Q+U plan (nb blocks)
hipError_t launch_alm_wquad_tqu(const crsht_plan* P, const double2* a, double* partial, int nb, hipStream_t s);
// Gaussian white draws (Philox4x32-10 + Box-Muller) of nrhs columns: w0
// [nrhs][nalm] white a_lm of a real field, w1 [nrhs][npix]; either may be null
hipError_t launch_white(const crsht_plan* P, int nrhs, uint64_t seed, uint64_t counter, double2* w0, double* w1,
                        hipStream_t s);
// out = fac_l[l] * in (one column of nalm coefficients)
hipError_t launch_scale_per_l(const crsht_plan* P, const double2* in, const double* fac_l, double2* out,
                              hipStream_t s);
hipError_t launch_pix_wsq(const crsht_plan* P, const double* w, const double* x, const double* y, double* partial,
                          int nb, hipStream_t s);
hipError_t launch_alm_wquad(const crsht_plan* P, const double* f, const double2* a, double* partial, int nb,
                            hipStream_t s);

}  // namespace crsht
