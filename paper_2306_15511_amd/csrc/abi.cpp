// Public C entry points: transforms, the constrained-realization operator,
// its right-hand side, preconditioned conjugate gradients and the joint
// amplitude move. Host orchestration only; every arithmetic step runs in the
// kernels of legendre.hip, ring.hip and vec.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace crsht;

namespace {

#define CR_TRY(expr)                           \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return CR_EDEVICE;   \
  } while (0)

#define CR_CHECK(expr)       \
  do {                       \
    int r_ = (expr);         \
    if (r_ != CR_OK) return r_; \
  } while (0)

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

const double2* C2(const double* p) { return reinterpret_cast<const double2*>(p); }
double2* C2(double* p) { return reinterpret_cast<double2*>(p); }
// the Legendre-sum buffers hold float2 values in the mixed-precision path
float2* F2(double2* p) { return reinterpret_cast<float2*>(p); }

int64_t eo_stride(const crsht_plan* P) { return (int64_t)P->g.npairs * (P->g.mmax + 1) * 2; }

int check_plan(const crsht_plan* P, int nrhs) {
  if (!P) return CR_EINVAL;
  if (nrhs < 1 || nrhs > P->nrhs_max) return CR_EINVAL;
  return CR_OK;
}

// Host data of one call (column amplitudes, per-l arrays) packed into the
// plan's next pinned staging slot and copied on the call's stream. A slot is
// reused only after the copies last enqueued from it have executed (its
// event), so the call never synchronises its stream.
struct Stager {
  crsht_plan* P;
  hipStream_t s;
  int slot = 0;
  size_t off = 0;
  bool ok = true;
  Stager(const crsht_plan* Pc, hipStream_t st) : P(const_cast<crsht_plan*>(Pc)), s(st) {
    slot = P->stage_next;
    P->stage_next = (P->stage_next + 1) % crsht_plan::kStageSlots;
    if (P->stage_used[slot]) ok = hipEventSynchronize(P->stage_ev[slot]) == hipSuccess;
  }
  int put(void* dst, const void* src, size_t bytes) {
    if (!ok) return CR_EDEVICE;
    if (off + bytes > P->stage_bytes) return CR_EINVAL;
    unsigned char* h = static_cast<unsigned char*>(P->stage_host[slot]) + off;
    std::memcpy(h, src, bytes);
    off = (off + bytes + 255) & ~size_t(255);
    CR_TRY(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s));
    return CR_OK;
  }
  int done() {
    if (!ok) return CR_EDEVICE;
    if (recorded || off == 0) return CR_OK;
    recorded = true;
    P->stage_used[slot] = true;
    CR_TRY(hipEventRecord(P->stage_ev[slot], s));
    return CR_OK;
  }
  // copies may have been enqueued from the slot before an argument error:
  // its event is recorded in any case
  ~Stager() { (void)done(); }
  bool recorded = false;
};

// ---- T+Q+U problem set-up: per-l 3x3 blocks of S^-1 and S^-1/2 (TT, TE and
// EE coupled, BB apart, TB = EB = 0) for amplitude q. For the symmetric
// positive definite 2x2 block M = [[a, b], [b, c]] of S^-1 the principal
// square root is (M + sqrt(det M) I) / sqrt(tr M + 2 sqrt(det M)).
int set_problem_tqu(const crsht_plan* P, const cr_problem* prob, double q, hipStream_t s, Stager& st) {
  const int lmax = P->g.lmax;
  if (prob->lmin < 2 || prob->lmin > lmax) return CR_EINVAL;   // E and B start at l = 2
  const double* tt = prob->cl;
  const double* ee = prob->cl + (lmax + 1);
  const double* bb = prob->cl + 2 * (lmax + 1);
  const double* te = prob->cl + 3 * (lmax + 1);
  std::vector<double> perl(4 * (size_t)(lmax + 1), 0.0), blk(8 * (size_t)(lmax + 1), 0.0);
  for (int l = 0; l <= lmax; ++l) {
    const double b = prob->bl[l];
    if (!std::isfinite(b)) return CR_EINVAL;
    perl[2 * (lmax + 1) + l] = b;
    if (l < prob->lmin) continue;
    const double ctt = q * tt[l], cee = q * ee[l], cbb = q * bb[l], cte = q * te[l];
    const double det = ctt * cee - cte * cte;
    if (!(ctt > 0.0) || !(cee > 0.0) || !(cbb > 0.0) || !(det > 0.0) || !std::isfinite(det) ||
        !std::isfinite(cbb))
      return CR_EINVAL;
    const double a = cee / det, bo = -cte / det, c = ctt / det;   // S^-1 of the (T, E) block
    const double sd = std::sqrt(a * c - bo * bo);
    const double nrm = 1.0 / std::sqrt(a + c + 2.0 * sd);
    double* o = &blk[8 * (size_t)l];
    o[0] = a;
    o[1] = bo;
    o[2] = c;
    o[3] = 1.0 / cbb;
    o[4] = (a + sd) * nrm;
    o[5] = bo * nrm;
    o[6] = (c + sd) * nrm;
    o[7] = 1.0 / std::sqrt(cbb);
    perl[3 * (lmax + 1) + l] = 1.0;
  }
  CR_CHECK(st.put(P->w.perl, perl.data(), perl.size() * sizeof(double)));
  CR_CHECK(st.put(P->w.sblk, blk.data(), blk.size() * sizeof(double)));
  CR_CHECK(st.done());
  CR_TRY(launch_expand_tqu(P, P->w.perl, s));
  return CR_OK;
}

// per-column amplitudes of prob (columns 0..nrhs-1; nrhs = 0: the caller
// takes none, so prob->amp must be NULL) into w.camp as (1/amp, 1/sqrt(amp)),
// 1 for every column without one
int set_columns(const crsht_plan* P, const cr_problem* prob, int nrhs, Stager& st) {
  if (prob->amp && nrhs < 1) return CR_EINVAL;
  std::vector<double2> f((size_t)P->nrhs_max, make_double2(1.0, 1.0));
  if (prob->amp)
    for (int c = 0; c < nrhs; ++c) {
      const double a = prob->amp[c];
      if (!(a > 0.0) || !std::isfinite(a)) return CR_EINVAL;
      f[c] = make_double2(1.0 / a, 1.0 / std::sqrt(a));
    }
  return st.put(P->w.camp, f.data(), f.size() * sizeof(double2));
}

// ---- problem set-up: per-l factors for amplitude q (C_l -> q C_l); nrhs as
// for set_columns
int set_problem(const crsht_plan* P, const cr_problem* prob, double q, hipStream_t s, int nrhs = 0) {
  if (!prob || !prob->cl || !prob->bl || !prob->ninv) return CR_EINVAL;
  if (!(q > 0.0) || !std::isfinite(q)) return CR_EINVAL;
  Stager st(P, s);
  CR_CHECK(set_columns(P, prob, nrhs, st));
  if (P->ncomp == 3) return set_problem_tqu(P, prob, q, s, st);
  const int lmax = P->g.lmax;
  if (prob->lmin < 0 || prob->lmin > lmax) return CR_EINVAL;
  if (!(q > 0.0) || !std::isfinite(q)) return CR_EINVAL;
  std::vector<double> perl(4 * (size_t)(lmax + 1), 0.0);
  for (int l = 0; l <= lmax; ++l) {
    const double b = prob->bl[l];
    if (!std::isfinite(b)) return CR_EINVAL;
    perl[2 * (lmax + 1) + l] = b;
    if (l < prob->lmin) continue;
    const double c = q * prob->cl[l];
    if (!(c > 0.0) || !std::isfinite(c)) return CR_EINVAL;
    perl[l] = 1.0 / c;
    perl[(lmax + 1) + l] = 1.0 / std::sqrt(c);
    perl[3 * (lmax + 1) + l] = 1.0;
  }
  CR_CHECK(st.put(P->w.perl, perl.data(), perl.size() * sizeof(double)));
  CR_CHECK(st.done());
  CR_TRY(launch_expand(P, P->w.perl, s));
  return CR_OK;
}

// column layout of the ring pass of a T+Q+U plan (maps [nrhs][3][npix])
RingCols tqu_cols(const crsht_plan* P) {
  RingCols c;
  c.group = 3;
  c.eo_cols = 9;
  c.geo_cols = 7;
  c.ninv_stride = P->g.npix;
  return c;
}

// Legendre sums and Q, U spectra of f * (a_T, a_E, a_B) (f per coefficient,
// null = 1) into w.eo; scratch w.alm_a (and w.pol in the mixed form, whose
// polar ring pairs take FP64 sums and an FP64 combination)
int tqu_spectra(const crsht_plan* P, int nrhs, const double2* alm, const double* f, hipStream_t s, bool mixed) {
  Workspace const& w = P->w;
  CR_TRY(launch_pol_prep_synth(P, nrhs, alm, f, w.alm_a, s));
  if (mixed) {
    CR_TRY(launch_legendre_synth_mixed(P, 9 * nrhs, w.alm_a, nullptr, F2(w.eo), s));
    CR_TRY(launch_pol_combine_synth(P, nrhs, w.eo, true, s));
    if (P->npol > 0) {
      const int64_t pst = (int64_t)P->npol * (P->g.mmax + 1) * 2;
      CR_TRY(launch_legendre_synth_pairs(P, 9 * nrhs, w.alm_a, w.pol, pst, P->npol, s));
      CR_TRY(launch_pol_combine_synth(P, nrhs, w.pol, false, s, P->npol));
      CR_TRY(launch_polar_spectra_to_f32(P, nrhs, w.pol, F2(w.eo), s));
    }
    return CR_OK;
  }
  CR_TRY(launch_legendre_synth(P, 9 * nrhs, w.alm_a, w.eo, s));
  CR_TRY(launch_pol_combine_synth(P, nrhs, w.eo, false, s));
  return CR_OK;
}

// f * (a_T, a_E, a_B) from the azimuthal adjoints in w.geo (T, Q, U in group
// columns 0..2); scratch w.alm_b (and w.pol in the mixed form: the polar ring
// pairs' adjoints move to FP64 and take FP64 Legendre sums added to the
// mixed sums of the other pairs)
int tqu_from_geo(const crsht_plan* P, int nrhs, const double* f, double2* out, hipStream_t s, bool mixed) {
  Workspace const& w = P->w;
  if (mixed) {
    if (P->npol > 0) CR_TRY(launch_polar_geo_to_f64(P, nrhs, F2(w.geo), w.pol, s));
    CR_TRY(launch_pol_pre_adjoint(P, nrhs, w.geo, true, s));
    CR_TRY(launch_legendre_adjoint_mixed(P, 7 * nrhs, F2(w.geo), w.alm_b, s));
    if (P->npol > 0) {
      const int64_t pst = (int64_t)P->npol * (P->g.mmax + 1) * 2;
      CR_TRY(launch_pol_pre_adjoint(P, nrhs, w.pol, false, s, P->npol));
      CR_TRY(launch_legendre_adjoint_pairs(P, 7 * nrhs, w.pol, pst, P->npol, true, w.alm_b, s));
    }
  } else {
    CR_TRY(launch_pol_pre_adjoint(P, nrhs, w.geo, false, s));
    CR_TRY(launch_legendre_adjoint(P, 7 * nrhs, w.geo, w.alm_b, false, s));
  }
  CR_TRY(launch_pol_combine_adjoint(P, nrhs, w.alm_b, f, out, s));
  return CR_OK;
}

// T+Q+U operator: out = S^-1 x + B Y^T N^-1 Y B x (S^-1 term only with prior);
// block partials of <x, out> in row 0. Scratch: w.eo, w.geo, w.alm_a, w.alm_b.
int operator_core_tqu(const crsht_plan* P, int nrhs, const double2* x, const double* ninv, double2* out,
                      hipStream_t s, bool mixed, bool prior) {
  Workspace const& w = P->w;
  CR_CHECK(tqu_spectra(P, nrhs, x, w.bl_keep, s, mixed));
  CR_TRY(launch_ring(P, 3 * nrhs, RING_FUSED, w.eo, nullptr, ninv, w.geo, mixed, s, tqu_cols(P)));
  CR_CHECK(tqu_from_geo(P, nrhs, w.bl_keep, w.alm_a, s, mixed));
  CR_TRY(launch_cg_q_tqu(P, nrhs, x, w.alm_a, out, s, prior));
  return CR_OK;
}

// A x for x already projected; pt = bk * x must be in w.alm_a. Uses w.eo,
// w.geo and w.alm_b as scratch (x must not live there).
// out = sinv * x + bk * (Y^T N^-1 Y)(pt); block partials of <x, out> in row 0.
// (T+Q+U plans: pt unused.)
int operator_core(const crsht_plan* P, int nrhs, const double2* x, const double2* pt, const double* ninv,
                  double2* out, hipStream_t s, bool mixed = false, bool prior = true) {
  if (P->ncomp == 3) return operator_core_tqu(P, nrhs, x, ninv, out, s, mixed, prior);
  if (mixed)
    CR_TRY(launch_legendre_synth_mixed(P, nrhs, pt, nullptr, F2(P->w.eo), s));
  else
    CR_TRY(launch_legendre_synth(P, nrhs, pt, P->w.eo, s));
  CR_TRY(launch_ring(P, nrhs, RING_FUSED, P->w.eo, nullptr, ninv, P->w.geo, mixed, s));
  if (mixed)
    CR_TRY(launch_legendre_adjoint_mixed(P, nrhs, F2(P->w.geo), P->w.alm_b, s));
  else
    CR_TRY(launch_legendre_adjoint(P, nrhs, P->w.geo, P->w.alm_b, false, s));
  CR_TRY(launch_cg_q(P, nrhs, x, P->w.alm_b, out, s, prior));
  return CR_OK;
}

// A p inside the mixed-precision PCG: with update, first p = z + beta p per
// column (fused with the MFMA operand preparation). out = sinv * p + bk *
// (Y^T N^-1 Y)(bk p); block partials of <p, out> in row 0.
// and alpha = <r, z> / <p, q> (the T form sums the adjoint's own <p, q>
// partials). The T form stores q in FP32 (float2 at the start of out, the
// precision of the bf16x3 operator that produced it); pcg_update then reads
// it with q32 = cg_q32(P).
// With the block preconditioner the T form also keeps z in FP32 (float2 at
// the start of w.cg_z: the preconditioner's products are FP32), z32 =
// cg_z32(P, pc), for every kernel that writes or reads z in that solve.
bool cg_q32(const crsht_plan* P) { return P->ncomp == 1; }
bool cg_z32(const crsht_plan* P, bool pc) { return pc && P->ncomp == 1; }
int operator_core_cg(const crsht_plan* P, int nrhs, bool update, const double* ninv, double2* out, int nb, double tol,
                     hipStream_t s, bool z32 = false) {
  Workspace const& w = P->w;
  if (P->ncomp == 3) {
    if (update) CR_TRY(launch_cg_pupdate(P, nrhs, w.cg_z, w.cg_p, w.alm_a, s));
    CR_CHECK(operator_core_tqu(P, nrhs, w.cg_p, ninv, out, s, true, true));
    CR_TRY(launch_cg_scalars(P, nrhs, 1, nb, tol, 0, s));
    return CR_OK;
  }
  // T plans: the pending x += alpha p of the last update goes with the
  // direction update, which reads that p anyway (pcg_update defers it)
  CR_TRY(launch_legendre_synth_mixed_cg(P, nrhs, w.cg_z, w.cg_p, update, F2(w.eo), s, z32,
                                        cg_q32(P) ? w.cg_x : nullptr));
  CR_TRY(launch_ring(P, nrhs, RING_FUSED, w.eo, nullptr, ninv, w.geo, true, s));
  CR_TRY(launch_legendre_adjoint_mixed_q(P, nrhs, F2(w.geo), w.cg_p, F2(out), s));
  CR_TRY(launch_cg_scalars(P, nrhs, 1, nb, tol, 0, s, w.adj_part, (int)P->t.mx_ntiles));
  return CR_OK;
}

// Jacobi diagonal into w.diag
int compute_diag(const crsht_plan* P, const double* ninv, hipStream_t s) {
  if (P->ncomp == 3) {
    // T entries with the T ring weights; E and B entries with the mean of the
    // Q and U ring weights (spin-0 functions stand in for the spin-2 ones)
    const int64_t np = P->g.npix, na = P->g.nalm;
    CR_TRY(launch_ring_weights(P, ninv, P->w.ring_w, s));
    CR_TRY(launch_legendre_adjoint(P, 1, nullptr, P->w.alm_b, true, s));
    CR_TRY(launch_ring_weights(P, ninv + np, P->w.ring_w, s, ninv + 2 * np, 0.5));
    CR_TRY(launch_legendre_adjoint(P, 1, nullptr, P->w.alm_b + na, true, s));
    CR_TRY(launch_diag_tqu(P, P->w.alm_b, P->w.alm_b + na, P->w.diag, s));
    return CR_OK;
  }
  CR_TRY(launch_ring_weights(P, ninv, P->w.ring_w, s));
  CR_TRY(launch_legendre_adjoint(P, 1, nullptr, P->w.alm_b, true, s));
  CR_TRY(launch_diag(P, P->w.alm_b, P->w.diag, s));
  return CR_OK;
}

// b = B Y^T (N^-1 d + N^-1/2 w1) + S^-1/2 w0 into out
int assemble_rhs(const crsht_plan* P, int nrhs, const double* ninv, const double* d, const double* w0,
                 const double* w1, double2* out, hipStream_t s) {
  if (P->ncomp == 3) {
    const double2* dterm = nullptr;
    if (d || w1) {
      CR_TRY(launch_pix_rhs(P, nrhs, ninv, d, w1, P->w.map_a, s));
      CR_TRY(launch_ring(P, 3 * nrhs, RING_ADJOINT, nullptr, P->w.map_a, nullptr, P->w.geo, false, s, tqu_cols(P)));
      CR_CHECK(tqu_from_geo(P, nrhs, P->w.bl_keep, P->w.alm_a, s, false));
      dterm = P->w.alm_a;
    }
    CR_TRY(launch_rhs_finish_tqu(P, nrhs, dterm, w0 ? C2(w0) : nullptr, out, s));
    return CR_OK;
  }
  const double2* braw = nullptr;
  if (d || w1) {
    CR_TRY(launch_pix_rhs(P, nrhs, ninv, d, w1, P->w.map_a, s));
    CR_TRY(launch_ring(P, nrhs, RING_ADJOINT, nullptr, P->w.map_a, nullptr, P->w.geo, false, s));
    CR_TRY(launch_legendre_adjoint(P, nrhs, P->w.geo, P->w.alm_b, false, s));
    braw = P->w.alm_b;
  }
  CR_TRY(launch_rhs_finish(P, nrhs, braw, w0 ? C2(w0) : nullptr, out, s));
  return CR_OK;
}

// map = Y (scale * alm). T plans: scale per coefficient with kappa folded in
// (rec_kappa for the plain transform). T+Q+U plans: scale is a per-coefficient
// factor without kappa (null = 1; P->t.rec_kappa is read as null).
int synth_f64(const crsht_plan* P, int nrhs, const double2* alm, const double* scale, double* map, hipStream_t s,
              bool mixed = false) {
  if (P->ncomp == 3) {
    CR_CHECK(tqu_spectra(P, nrhs, alm, scale == P->t.rec_kappa ? nullptr : scale, s, mixed));
    CR_TRY(launch_ring(P, 3 * nrhs, RING_SYNTH, P->w.eo, map, nullptr, nullptr, mixed, s, tqu_cols(P)));
    return CR_OK;
  }
  if (mixed) {
    CR_TRY(launch_legendre_synth_mixed(P, nrhs, alm, scale, F2(P->w.eo), s));
  } else {
    CR_TRY(launch_scale_alm(P, nrhs, alm, scale, P->w.alm_a, s));
    CR_TRY(launch_legendre_synth(P, nrhs, P->w.alm_a, P->w.eo, s));
  }
  CR_TRY(launch_ring(P, nrhs, RING_SYNTH, P->w.eo, map, nullptr, nullptr, mixed, s));
  return CR_OK;
}

int adjoint_f64(const crsht_plan* P, int nrhs, const double* map, double2* alm, hipStream_t s, bool mixed = false) {
  if (P->ncomp == 3) {
    CR_TRY(launch_ring(P, 3 * nrhs, RING_ADJOINT, nullptr, const_cast<double*>(map), nullptr, P->w.geo, mixed, s,
                       tqu_cols(P)));
    return tqu_from_geo(P, nrhs, nullptr, alm, s, mixed);
  }
  CR_TRY(launch_ring(P, nrhs, RING_ADJOINT, nullptr, const_cast<double*>(map), nullptr, P->w.geo, mixed, s));
  if (mixed)
    CR_TRY(launch_legendre_adjoint_mixed(P, nrhs, F2(P->w.geo), alm, s));
  else
    CR_TRY(launch_legendre_adjoint(P, nrhs, P->w.geo, alm, false, s));
  CR_TRY(launch_scale_alm(P, nrhs, alm, P->t.rec_kappa, alm, s));
  return CR_OK;
}

// Runs body(stream) -- a fixed sequence of kernel launches -- on s. With
// use_graph the sequence is captured once on the plan's capture stream into a
// HIP graph (kept with its key) and replayed on s; a different key
// re-captures. Kernel timing (per-launch events) forces direct launches.
template <class F>
int run_block(const crsht_plan* Pc, const GraphKey& key0, bool use_graph, hipStream_t s, F body) {
  crsht_plan* P = const_cast<crsht_plan*>(Pc);
  if (!use_graph || P->timing.on || !P->cap_stream) return body(s);
  GraphKey key = key0;
  key.aux_off = P->aux_off;
  if (!(P->graph_exec && P->graph_key == key)) {
    if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
    P->graph_exec = nullptr;
    P->graph_key = GraphKey();
    CR_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = body(P->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(P->cap_stream, &g);
    if (rc != CR_OK || e != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return rc != CR_OK ? rc : CR_EDEVICE;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return CR_EDEVICE;
    P->graph_exec = ex;
    P->graph_key = key;
  }
  CR_TRY(hipGraphLaunch(P->graph_exec, s));
  return CR_OK;
}

int read_scalars(const crsht_plan* P, int nrhs, hipStream_t s) {
  CR_TRY(hipMemcpyAsync(P->w.host_scal, P->w.scal, (size_t)nrhs * kScalSlots * sizeof(double),
                        hipMemcpyDeviceToHost, s));
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

// Progress of long solves: with the environment variable CRSHT_PROGRESS set
// to a positive integer k, every k-th host check of a PCG loop prints the
// iteration count and the largest recursive residual of the unfinished
// columns to stderr (read from the scalars the check has just copied back).
int progress_every() {
  static const int k = [] {
    const char* e = std::getenv("CRSHT_PROGRESS");
    const int v = e ? std::atoi(e) : 0;
    return v > 0 ? v : 0;
  }();
  return k;
}

void report_progress(const crsht_plan* P, int nrhs, int it, int check, const char* what) {
  const int k = progress_every();
  if (k == 0 || check % k != 0) return;
  double worst = 0.0;
  int open = 0;
  for (int c = 0; c < nrhs; ++c) {
    const double* sc = P->w.host_scal + c * kScalSlots;
    if (sc[S_DONE] != 0.0) continue;
    ++open;
    worst = std::max(worst, sc[S_REL]);
  }
  std::fprintf(stderr, "crsht %s: iteration %d, %d of %d columns open, largest recursive residual %.3e\n", what,
               it, open, nrhs, worst);
  std::fflush(stderr);
}

int write_scalars(const crsht_plan* P, int nrhs, hipStream_t s) {
  CR_TRY(hipMemcpyAsync(P->w.scal, P->w.host_scal, (size_t)nrhs * kScalSlots * sizeof(double),
                        hipMemcpyHostToDevice, s));
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

// true relative residual ||b - A x|| / ||b|| per column into rel[]; leaves r = b - A x
// precisions of the user-visible transforms; CR_BF16X6 runs the mixed
// kernels with three bf16 parts per operand for the duration of the call
bool transform_prec(cr_prec prec) { return prec == CR_F64 || prec == CR_MIXED || prec == CR_BF16X6; }
struct SplitScope {
  const crsht_plan* P;
  SplitScope(const crsht_plan* p, cr_prec prec) : P(p) { P->mx_split = prec == CR_BF16X6 ? 3 : 2; }
  ~SplitScope() { P->mx_split = 2; }
};

// r = b - A x and the relative residuals; A in FP64, or (low) with the bf16x6
// operator (about 5e-7 of ||A x||: for intermediate residual replacements
// far above the tolerance)
int true_residual(const crsht_plan* P, int nrhs, const double* ninv, const double2* x, const double2* b,
                  double2* r, std::vector<double>& rel, hipStream_t s, bool low = false) {
  const int64_t na = P->g.nalm;
  if (P->ncomp == 1) CR_TRY(launch_scale_alm(P, nrhs, x, P->w.bk, P->w.alm_a, s));
  {
    SplitScope sc(P, low ? CR_BF16X6 : CR_F64);
    CR_CHECK(operator_core(P, nrhs, x, P->w.alm_a, ninv, P->w.cg_q, s, low));
  }
  CR_TRY(launch_residual(P, nrhs, b, P->w.cg_q, r, s));
  const int nb = vec_reduce_blocks(P);
  CR_TRY(launch_sum_rows(P, nrhs, nb, s));
  CR_CHECK(read_scalars(P, nrhs, s));
  rel.assign(nrhs, 0.0);
  for (int c = 0; c < nrhs; ++c) {
    const double* sc = P->w.host_scal + c * kScalSlots;
    rel[c] = sc[S_AUX1] > 0.0 ? std::sqrt(sc[S_AUX0] / sc[S_AUX1]) : 0.0;
  }
  (void)na;
  return CR_OK;
}

// PCG on the problem already set up (sinv, bk, diag in the workspace) for the
// right-hand side b (device, [nrhs][nalm]); solution in w.cg_x. Scratch:
// w.cg_r, cg_z, cg_p, cg_q, alm_a, alm_b, eo, geo. With verify, a column
// whose recursive residual meets tol is confirmed against the true FP64
// residual and restarted from it if it does not; rel[] then holds the true
// relative residuals. iters[] receives the iterations per column.
// z = P r and the start of PCG (p = z, <r, z>, <r, r>, <b, b>) for the
// Jacobi (pc false) or the block preconditioner
int pcg_start(const crsht_plan* P, int nrhs, const double2* b, bool pc, hipStream_t s, bool z32 = false) {
  Workspace const& w = P->w;
  if (pc) CR_TRY(launch_pc_apply(P, nrhs, w.cg_r, w.cg_z, s, false, z32));
  CR_TRY(launch_cg_start(P, nrhs, b, w.cg_r, w.cg_z, w.cg_p, w.alm_a, s, pc, z32));
  return CR_OK;
}

// x += alpha p, r -= alpha q, z = P r; <r, z>, <r, r> and beta (the block
// preconditioner sums its own <r, z> partials as it writes z)
int pcg_update(const crsht_plan* P, int nrhs, bool pc, int nb, double tol, hipStream_t s, bool q32 = false,
               bool z32 = false) {
  Workspace const& w = P->w;
  CR_TRY(launch_cg_update(P, nrhs, w.cg_x, w.cg_r, w.cg_z, w.cg_p, w.cg_q, s, pc, q32 ? F2(w.cg_q) : nullptr));
  if (pc) {
    CR_TRY(launch_pc_apply(P, nrhs, w.cg_r, w.cg_z, s, true, z32));
    CR_TRY(launch_cg_scalars(P, nrhs, 2, nb, tol, 0, s, P->pc.part, P->pc.ntasks));
  } else {
    CR_TRY(launch_cg_scalars(P, nrhs, 2, nb, tol, 0, s));
  }
  return CR_OK;
}

int pcg_run(const crsht_plan* P, int nrhs, const double* ninv, const double2* b, double tol, int maxiter,
            int check_every, bool mixed, bool verify, std::vector<int>& iters, std::vector<double>& rel,
            std::vector<int>& broke, hipStream_t s, bool use_graph = false, bool pc = false) {
  const int64_t na = vlen(P);
  const int nb = vec_reduce_blocks(P);
  Workspace const& w = P->w;
  CR_TRY(hipMemsetAsync(w.cg_x, 0, (size_t)nrhs * na * sizeof(double2), s));
  CR_TRY(hipMemcpyAsync(w.cg_r, b, (size_t)nrhs * na * sizeof(double2), hipMemcpyDeviceToDevice, s));
  CR_CHECK(pcg_start(P, nrhs, b, pc, s));
  CR_TRY(launch_cg_scalars(P, nrhs, 0, nb, tol, 0, s));
  CR_CHECK(read_scalars(P, nrhs, s));

  rel.assign(nrhs, 0.0);
  int it = 0, checks = 0;
  for (;;) {
    bool all_done = true;
    for (int c = 0; c < nrhs; ++c) all_done &= P->w.host_scal[c * kScalSlots + S_DONE] != 0.0;
    if (!all_done && it < maxiter) {
      const int n = std::min(check_every, maxiter - it);
      GraphKey key;
      key.kind = mixed ? 2 : 0;
      key.nrhs = nrhs;
      key.n = n;
      key.pc = pc ? 1 : 0;
      key.ninv = ninv;
      key.tol = tol;
      CR_CHECK(run_block(P, key, use_graph, s, [&](hipStream_t q) -> int {
        for (int k = 0; k < n; ++k) {
          CR_CHECK(operator_core(P, nrhs, w.cg_p, w.alm_a, ninv, w.cg_q, q, mixed));
          CR_TRY(launch_cg_scalars(P, nrhs, 1, nb, tol, 0, q));
          CR_CHECK(pcg_update(P, nrhs, pc, nb, tol, q));
          CR_TRY(launch_cg_pupdate(P, nrhs, w.cg_z, w.cg_p, w.alm_a, q));
        }
        return CR_OK;
      }));
      it += n;
      CR_CHECK(read_scalars(P, nrhs, s));
      report_progress(P, nrhs, it, ++checks, "pcg");
      continue;
    }
    if (!verify) {
      for (int c = 0; c < nrhs; ++c) rel[c] = P->w.host_scal[c * kScalSlots + S_REL];
      break;
    }
    // all columns stopped (or out of iterations): confirm with the true residual
    std::vector<double> keep_scal(P->w.host_scal, P->w.host_scal + (size_t)nrhs * kScalSlots);
    CR_CHECK(true_residual(P, nrhs, ninv, w.cg_x, b, w.cg_r, rel, s));
    std::memcpy(P->w.host_scal, keep_scal.data(), keep_scal.size() * sizeof(double));
    bool restart = false;
    for (int c = 0; c < nrhs; ++c) {
      double* sc = P->w.host_scal + c * kScalSlots;
      const bool br = sc[S_BREAK] != 0.0;
      if (!br && rel[c] > tol && it < maxiter && sc[S_BB] > 0.0) {
        sc[S_DONE] = 0.0;  // restart this column from its true residual
        restart = true;
      } else {
        sc[S_DONE] = 1.0;
      }
    }
    if (!restart) break;
    CR_CHECK(write_scalars(P, nrhs, s));
    CR_CHECK(pcg_start(P, nrhs, b, pc, s));
    CR_TRY(launch_cg_scalars(P, nrhs, 0, nb, tol, 1, s));
    CR_CHECK(read_scalars(P, nrhs, s));
  }
  iters.assign(nrhs, 0);
  broke.assign(nrhs, 0);
  for (int c = 0; c < nrhs; ++c) {
    const double* sc = P->w.host_scal + c * kScalSlots;
    iters[c] = (int)sc[S_ITERS];
    broke[c] = sc[S_BREAK] != 0.0 ? 1 : 0;
  }
  return CR_OK;
}

int fill_stats(int nrhs, double tol, const std::vector<int>& iters, const std::vector<int>& refine,
               const std::vector<double>& rel, const std::vector<int>& broke, cr_stats* stats) {
  for (int c = 0; c < nrhs; ++c) {
    stats[c].iters = iters[c];
    stats[c].refinements = refine[c];
    stats[c].rel_resid_true = rel[c];
    if (broke[c] || !std::isfinite(rel[c]))
      stats[c].status = CR_BREAKDOWN;
    else if (rel[c] > tol)
      stats[c].status = CR_NOCONV;
    else
      stats[c].status = CR_OK;
  }
  return CR_OK;
}

// FP64 refinement around the mixed-precision PCG by residual replacement
// ("reliable updates"): PCG runs with the mixed operator, and whenever the
// recursive residual of a column has dropped by inner_tol since the last
// replacement (or claims convergence), the residuals of all columns are
// replaced by the true FP64 residuals b - A x; z and <r,z> are recomputed and
// the search directions kept, so the Krylov space is not discarded. A column
// stops when its true relative residual is at most tol.
int solve_refined(const crsht_plan* P, int nrhs, const double* ninv, const cr_opts* o, std::vector<int>& iters,
                  std::vector<int>& refine, std::vector<double>& rel, std::vector<int>& broke, hipStream_t s,
                  bool pc = false) {
  // PCG on the mixed-precision operator with FP64 vectors and reliable updates:
  // every time a column's recursive residual has fallen by inner_tol since its
  // last replacement (or claims convergence), r is replaced by the FP64 true
  // residual b - A x right after the x, r update and before the direction
  // update, so beta and p continue from the replaced residual.  A column whose
  // true residual did not fall since its last replacement restarts its
  // direction (beta = 0).
  const int64_t na = vlen(P);
  const int nb = vec_reduce_blocks(P);
  Workspace const& w = P->w;
  const int every = o->check_every > 0 ? o->check_every : 8;
  const double itol = (o->inner_tol > 0.0 && o->inner_tol < 1.0) ? o->inner_tol : 1e-2;
  const int maxref = o->max_refine > 0 ? o->max_refine : 1000;
  const double tol = o->tol;
  refine.assign(nrhs, 0);
  CR_TRY(hipMemsetAsync(w.cg_x, 0, (size_t)nrhs * na * sizeof(double2), s));
  CR_TRY(hipMemcpyAsync(w.cg_r, w.cg_b, (size_t)nrhs * na * sizeof(double2), hipMemcpyDeviceToDevice, s));
  const bool z32 = cg_z32(P, pc);
  // the iterations of T plans leave the last x += alpha p pending (scal
  // S_XA): applied before x is read, here and on the host copy of the scalars
  auto flush_x = [&]() -> int {
    if (!cg_q32(P)) return CR_OK;
    CR_TRY(launch_x_flush(P, nrhs, s));
    for (int c = 0; c < nrhs; ++c) P->w.host_scal[c * kScalSlots + S_XA] = 0.0;
    return CR_OK;
  };
  CR_CHECK(pcg_start(P, nrhs, w.cg_b, pc, s, z32));
  CR_TRY(launch_cg_scalars(P, nrhs, 0, nb, tol, 0, s));
  CR_CHECK(read_scalars(P, nrhs, s));
  std::vector<double> last(nrhs, 1.0);   // true relative residual at the last replacement
  rel.assign(nrhs, 1.0);
  int it = 0, nrep = 0, checks = 0;
  bool pending = false;                  // direction update of the last iteration not yet applied
  bool fresh = false;                    // rel[] is the true residual of the current x
  for (;;) {
    bool need = false;
    std::vector<char> trig(nrhs, 0);
    for (int c = 0; c < nrhs; ++c) {
      const double* sc = P->w.host_scal + c * kScalSlots;
      if (sc[S_BREAK] != 0.0 || rel[c] <= tol) continue;
      if (sc[S_DONE] != 0.0 || sc[S_REL] <= itol * last[c]) need = true, trig[c] = 1;
    }
    if (need && pending && nrep < maxref) {
      // an intermediate replacement, while no column claims convergence and
      // every open column's residual is far above the reach of the bf16x6
      // operator, takes that operator; the others (and every decision on
      // convergence) take FP64
      bool low = true;
      for (int c = 0; c < nrhs; ++c) {
        const double* sc = P->w.host_scal + c * kScalSlots;
        if (sc[S_BREAK] != 0.0 || rel[c] <= tol) continue;
        if (sc[S_DONE] != 0.0 || sc[S_REL] < kLowReplaceFloor) low = false;
      }
      CR_CHECK(flush_x());
      std::vector<double> keep(P->w.host_scal, P->w.host_scal + (size_t)nrhs * kScalSlots);
      CR_CHECK(true_residual(P, nrhs, ninv, w.cg_x, w.cg_b, w.cg_r, rel, s, low));
      fresh = !low;
      ++nrep;
      std::memcpy(P->w.host_scal, keep.data(), keep.size() * sizeof(double));
      bool cont = false;
      for (int c = 0; c < nrhs; ++c) {
        double* sc = P->w.host_scal + c * kScalSlots;
        if (sc[S_BREAK] != 0.0) continue;
        // keep the direction only when the replacement corrects the
        // recursive residual by a small relative amount; restart it when the
        // true residual did not fall since the last replacement, or when it is
        // far above the recursive one (the Krylov recurrences drifted: with a
        // strong preconditioner and long blocks between checks the recursive
        // residual can fall orders of magnitude below the reach of the
        // low-precision operator, and beta from it would be meaningless)
        const double rec = keep[(size_t)c * kScalSlots + S_REL];
        sc[S_RESTART] = (trig[c] && (rel[c] >= last[c] || rel[c] > 4.0 * rec)) ? 1.0 : 0.0;
        last[c] = rel[c];
        refine[c] += 1;
        if (rel[c] <= tol && !low) {
          sc[S_DONE] = 1.0;
        } else if (it < o->maxiter) {
          sc[S_DONE] = 0.0;
          cont = true;
        } else {
          sc[S_DONE] = 1.0;
        }
      }
      if (!cont) break;
      // z = D^-1 r from the replaced residual, beta = <r,z>/<r,z>_prev; the
      // direction update stays pending (fused into the next operator)
      CR_CHECK(write_scalars(P, nrhs, s));
      if (pc) {
        CR_TRY(launch_pc_apply(P, nrhs, w.cg_r, w.cg_z, s, false, z32));
        CR_TRY(launch_pc_dots(P, nrhs, w.cg_r, w.cg_z, true, s, z32));
      } else {
        CR_TRY(launch_cg_replace(P, nrhs, w.cg_r, w.cg_z, s));
      }
      CR_TRY(launch_cg_scalars(P, nrhs, 3, nb, tol, 0, s));
    }
    bool any = false;
    for (int c = 0; c < nrhs; ++c) any |= P->w.host_scal[c * kScalSlots + S_DONE] == 0.0;
    if (!any || it >= o->maxiter) {
      // every column stopped: confirmed by its true residual, broken down,
      // out of iterations, or (once max_refine replacements are spent)
      // stopped on its recursive residual; report the true residual of the x
      // that is returned
      CR_CHECK(flush_x());
      if (!fresh) CR_CHECK(true_residual(P, nrhs, ninv, w.cg_x, w.cg_b, w.cg_r, rel, s));
      break;
    }
    const int n = std::min(every, o->maxiter - it);
    GraphKey key;
    key.kind = 1;
    key.nrhs = nrhs;
    key.n = n;
    key.first_update = pending ? 1 : 0;
    key.pc = pc ? 1 : 0;
    key.ninv = ninv;
    key.tol = tol;
    const bool first = pending;
    CR_CHECK(run_block(P, key, o->use_graph != 0, s, [&](hipStream_t q) -> int {
      for (int k = 0; k < n; ++k) {
        CR_CHECK(operator_core_cg(P, nrhs, k > 0 || first, ninv, w.cg_q, nb, tol, q, z32));
        CR_CHECK(pcg_update(P, nrhs, pc, nb, tol, q, cg_q32(P), z32));
      }
      return CR_OK;
    }));
    pending = true;
    fresh = false;
    it += n;
    CR_CHECK(read_scalars(P, nrhs, s));
    report_progress(P, nrhs, it, ++checks, "mixed pcg");
  }
  iters.assign(nrhs, 0);
  broke.assign(nrhs, 0);
  for (int c = 0; c < nrhs; ++c) {
    const double* sc = P->w.host_scal + c * kScalSlots;
    iters[c] = (int)sc[S_ITERS];
    broke[c] = sc[S_BREAK] != 0.0 ? 1 : 0;
  }
  return CR_OK;
}

// ====================================================== device-driven solve
// The refined PCG of solve_refined enqueued as a whole, stream-ordered: the
// decisions its host loop takes from the scalars it reads back are taken on
// the device by k_dctl (dsolve.hip) between predicated sections. One
// super-step = check, FP64 true residual (if a column asks for it), tail (z,
// <r,z> and beta from the replaced residual), block of `every` iterations.
// CR_F64 runs the same loop with the FP64 operator and replaces the residual
// only when a column claims convergence (reliable-update PCG).
struct DSolve {
  const crsht_plan* P = nullptr;
  int nrhs = 0;
  const double* ninv = nullptr;
  bool mixed = false, pc = false;
  DctlArgs a{};
  int steps = 0;   // super-steps enqueued: ceil(maxiter / every)
};

// sets the kernel predicate of the plan for the sections enqueued in its scope
struct PredScope {
  const crsht_plan* P;
  PredScope(const crsht_plan* Pc, const int* p) : P(Pc) { P->pred = p; }
  ~PredScope() { P->pred = nullptr; }
};

// r = b - A x in FP64; ||r||^2, ||b||^2 into the column scalars (no read-back)
int true_residual_dev(const crsht_plan* P, int nrhs, const double* ninv, const double2* x, const double2* b,
                      double2* r, hipStream_t s, bool low = false) {
  if (P->ncomp == 1) CR_TRY(launch_scale_alm(P, nrhs, x, P->w.bk, P->w.alm_a, s));
  {
    SplitScope sc(P, low ? CR_BF16X6 : CR_F64);
    CR_CHECK(operator_core(P, nrhs, x, P->w.alm_a, ninv, P->w.cg_q, s, low));
  }
  CR_TRY(launch_residual(P, nrhs, b, P->w.cg_q, r, s));
  CR_TRY(launch_sum_rows(P, nrhs, vec_reduce_blocks(P), s));
  return CR_OK;
}

int dsolve_setup(DSolve& d, const crsht_plan* P, const cr_problem* prob, int nrhs, const cr_opts* o) {
  if (!prob || !o) return CR_EINVAL;
  if (!prob->cl || !prob->bl || !prob->ninv) return CR_EINVAL;
  if (!(o->tol > 0.0) || o->maxiter < 1) return CR_EINVAL;
  if (o->prec != CR_F64 && o->prec != CR_MIXED) return CR_EINVAL;
  if (o->precond != CR_PC_JACOBI && o->precond != CR_PC_BLOCK) return CR_EINVAL;
  if (o->terms != CR_SUM) return CR_EINVAL;   // separate outputs: cr_solve only
  d.P = P;
  d.nrhs = nrhs;
  d.ninv = prob->ninv;
  d.mixed = o->prec == CR_MIXED;
  d.pc = o->precond == CR_PC_BLOCK;
  if (d.pc && !P->pc.built) return CR_EINVAL;
  d.a.nrhs = nrhs;
  d.a.tol = o->tol;
  d.a.itol = d.mixed ? ((o->inner_tol > 0.0 && o->inner_tol < 1.0) ? o->inner_tol : 1e-2) : 0.0;
  d.a.maxref = o->max_refine > 0 ? o->max_refine : 1000;
  d.a.maxiter = o->maxiter;
  d.a.every = o->check_every > 0 ? o->check_every : 8;
  d.a.f64 = d.mixed ? 0 : 1;
  d.steps = (o->maxiter + d.a.every - 1) / d.a.every;
  return CR_OK;
}

// check, FP64 true residual and (with tail) z, <r,z>, beta from it
int dsolve_check_replace(const DSolve& d, hipStream_t q, bool tail) {
  const crsht_plan* P = d.P;
  Workspace const& w = P->w;
  CR_TRY(launch_dctl(P, DC_CHECK, d.a, nullptr, q));
  // (mixed T iterations leave the last x += alpha p pending: applied first)
  const bool defer = d.mixed && cg_q32(P);
  {
    PredScope ps(P, w.ctl + C_SKIP_REPL);
    if (defer) CR_TRY(launch_x_flush(P, d.nrhs, q));
    CR_CHECK(true_residual_dev(P, d.nrhs, d.ninv, w.cg_x, w.cg_b, w.cg_r, q));
  }
  if (d.mixed) {
    PredScope ps(P, w.ctl + C_SKIP_REPL_LOW);
    if (defer) CR_TRY(launch_x_flush(P, d.nrhs, q));
    CR_CHECK(true_residual_dev(P, d.nrhs, d.ninv, w.cg_x, w.cg_b, w.cg_r, q, true));
  }
  CR_TRY(launch_dctl(P, DC_AFTER_REPL, d.a, nullptr, q));
  if (!tail) return CR_OK;
  PredScope ps(P, w.ctl + C_SKIP_TAIL);
  if (d.pc) {
    const bool z32 = d.mixed && cg_z32(P, d.pc);
    CR_TRY(launch_pc_apply(P, d.nrhs, w.cg_r, w.cg_z, q, false, z32));
    CR_TRY(launch_pc_dots(P, d.nrhs, w.cg_r, w.cg_z, true, q, z32));
  } else {
    CR_TRY(launch_cg_replace(P, d.nrhs, w.cg_r, w.cg_z, q));
  }
  CR_TRY(launch_cg_scalars(P, d.nrhs, 3, vec_reduce_blocks(P), d.a.tol, 0, q));
  return CR_OK;
}

// one super-step; `first`: the block starts with the pending direction update
int dsolve_step(const DSolve& d, bool first, hipStream_t q) {
  const crsht_plan* P = d.P;
  Workspace const& w = P->w;
  const int nb = vec_reduce_blocks(P);
  CR_CHECK(dsolve_check_replace(d, q, true));
  CR_TRY(launch_dctl(P, DC_PRE_BLOCK, d.a, nullptr, q));
  const bool z32 = d.mixed && cg_z32(P, d.pc);
  {
    PredScope ps(P, w.ctl + C_SKIP_ITER);
    for (int k = 0; k < d.a.every; ++k) {
      const bool upd = k > 0 || first;
      if (d.mixed) {
        CR_CHECK(operator_core_cg(P, d.nrhs, upd, d.ninv, w.cg_q, nb, d.a.tol, q, z32));
      } else {
        if (upd) CR_TRY(launch_cg_pupdate(P, d.nrhs, w.cg_z, w.cg_p, w.alm_a, q));
        CR_CHECK(operator_core(P, d.nrhs, w.cg_p, w.alm_a, d.ninv, w.cg_q, q));
        CR_TRY(launch_cg_scalars(P, d.nrhs, 1, nb, d.a.tol, 0, q));
      }
      CR_CHECK(pcg_update(P, d.nrhs, d.pc, nb, d.a.tol, q, d.mixed && cg_q32(P), z32));
    }
  }
  CR_TRY(launch_dctl(P, DC_AFTER_BLOCK, d.a, nullptr, q));
  return CR_OK;
}

// captured super-steps (first block, later blocks), kept with their key;
// returns whether they are to be replayed
int dsolve_graphs(const DSolve& d, bool use_graph, bool* graphs) {
  crsht_plan* P = const_cast<crsht_plan*>(d.P);
  *graphs = false;
  if (!use_graph || P->timing.on || !P->cap_stream) return CR_OK;
  GraphKey key;
  key.kind = d.mixed ? 3 : 4;
  key.nrhs = d.nrhs;
  key.n = d.a.every;
  key.pc = d.pc ? 1 : 0;
  key.ninv = d.ninv;
  key.tol = d.a.tol;
  key.itol = d.a.itol;
  key.maxref = d.a.maxref;
  key.maxiter = d.a.maxiter;
  key.aux_off = P->aux_off;
  if (!(P->dgraph[0] && P->dgraph[1] && P->dgraph_key == key)) {
    if (P->dgraph[0] || P->dgraph[1]) {
      // replays of the old graphs may still be queued on some stream
      CR_TRY(hipDeviceSynchronize());
      for (auto& gx : P->dgraph) {
        if (gx) (void)hipGraphExecDestroy(gx);
        gx = nullptr;
      }
    }
    P->dgraph_key = GraphKey();
    for (int f = 0; f < 2; ++f) {
      CR_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
      const int rc = dsolve_step(d, f == 1, P->cap_stream);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(P->cap_stream, &g);
      if (rc != CR_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return rc != CR_OK ? rc : CR_EDEVICE;
      }
      hipGraphExec_t ex = nullptr;
      const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) return CR_EDEVICE;
      P->dgraph[f] = ex;
    }
    P->dgraph_key = key;
  }
  *graphs = true;
  return CR_OK;
}

int dsolve_launch(const DSolve& d, int k, bool graphs, hipStream_t s) {
  if (graphs) {
    CR_TRY(hipGraphLaunch(d.P->dgraph[k > 0 ? 1 : 0], s));
    return CR_OK;
  }
  return dsolve_step(d, k > 0, s);
}

// problem set-up, right-hand side, x = 0, r = b and the start of PCG
int dsolve_prologue(const DSolve& d, const cr_problem* prob, const double* dm, const double* w0, const double* w1,
                    const double* rhs, hipStream_t s) {
  const crsht_plan* P = d.P;
  Workspace const& w = P->w;
  const size_t vbytes = (size_t)d.nrhs * vlen(P) * sizeof(double2);
  CR_CHECK(set_problem(P, prob, 1.0, s, d.nrhs));
  if (!d.pc) CR_CHECK(compute_diag(P, prob->ninv, s));
  if (rhs)
    CR_TRY(launch_project(P, d.nrhs, C2(rhs), w.cg_b, s));
  else
    CR_CHECK(assemble_rhs(P, d.nrhs, prob->ninv, dm, w0, w1, w.cg_b, s));
  CR_TRY(hipMemsetAsync(w.cg_x, 0, vbytes, s));
  CR_TRY(hipMemcpyAsync(w.cg_r, w.cg_b, vbytes, hipMemcpyDeviceToDevice, s));
  CR_CHECK(pcg_start(P, d.nrhs, w.cg_b, d.pc, s, d.mixed && cg_z32(P, d.pc)));
  CR_TRY(launch_cg_scalars(P, d.nrhs, 0, vec_reduce_blocks(P), d.a.tol, 0, s));
  CR_TRY(launch_dctl(P, DC_INIT, d.a, nullptr, s));
  return CR_OK;
}

// the last check, the FP64 true residual of the returned x (unless current),
// the statistics and x
int dsolve_epilogue(const DSolve& d, double* s_out, void* stats_dev, hipStream_t s) {
  const crsht_plan* P = d.P;
  Workspace const& w = P->w;
  CR_CHECK(dsolve_check_replace(d, s, false));
  if (d.mixed && cg_q32(P)) CR_TRY(launch_x_flush(P, d.nrhs, s));   // any pending x += alpha p
  CR_TRY(launch_dctl(P, DC_FINAL_PRE, d.a, nullptr, s));
  {
    PredScope ps(P, w.ctl + C_SKIP_FINAL);
    CR_CHECK(true_residual_dev(P, d.nrhs, d.ninv, w.cg_x, w.cg_b, w.cg_r, s));
  }
  CR_TRY(launch_dctl(P, DC_FINAL_POST, d.a, stats_dev, s));
  CR_TRY(hipMemcpyAsync(s_out, w.cg_x, (size_t)d.nrhs * vlen(P) * sizeof(double2), hipMemcpyDeviceToDevice, s));
  return CR_OK;
}

// x0 (device, nrhs columns, optional; may alias s_out): warm start. The solve
// then runs on the correction, A delta = b - A x0, to the tolerance
// tol / max_c(||b - A x0|| / ||b||) (the strictest column's), and s_out =
// x0 + delta; stats report the correction's iterations and the residual
// relative to ||b||.
int solve_core(const crsht_plan* P, const cr_problem* prob, double q, int nrhs, const double* d, const double* w0,
               const double* w1, const double* rhs, double* s_out, const cr_opts* opts, cr_stats* stats,
               hipStream_t s, const double* x0 = nullptr) {
  if (!opts || !stats || !s_out) return CR_EINVAL;
  if (!(opts->tol > 0.0) || opts->maxiter < 1) return CR_EINVAL;
  if (opts->prec != CR_F64 && opts->prec != CR_MIXED) return CR_EINVAL;
  if (opts->precond != CR_PC_JACOBI && opts->precond != CR_PC_BLOCK) return CR_EINVAL;
  const bool pc = opts->precond == CR_PC_BLOCK;
  if (pc && !P->pc.built) return CR_EINVAL;
  const int every = opts->check_every > 0 ? opts->check_every : 8;
  CR_CHECK(set_problem(P, prob, q, s, nrhs));
  if (!pc) CR_CHECK(compute_diag(P, prob->ninv, s));
  if (rhs)
    CR_TRY(launch_project(P, nrhs, C2(rhs), P->w.cg_b, s));
  else
    CR_CHECK(assemble_rhs(P, nrhs, prob->ninv, d, w0, w1, P->w.cg_b, s));
  cr_opts o = *opts;
  std::vector<double> r0(nrhs, 1.0);   // ||b - A x0|| / ||b|| per column
  const size_t vbytes = (size_t)nrhs * vlen(P) * sizeof(double2);
  if (x0) {
    CR_TRY(launch_project(P, nrhs, C2(x0), P->w.cg_x, s));
    CR_CHECK(true_residual(P, nrhs, prob->ninv, P->w.cg_x, P->w.cg_b, P->w.cg_r, r0, s));
    const double rmax = *std::max_element(r0.begin(), r0.end());
    if (rmax <= opts->tol) {   // the start already meets the tolerance
      std::vector<int> zi(nrhs, 0), zb(nrhs, 0);
      fill_stats(nrhs, opts->tol, zi, zi, r0, zb, stats);
      CR_TRY(hipMemcpyAsync(s_out, P->w.cg_x, vbytes, hipMemcpyDeviceToDevice, s));
      CR_TRY(hipStreamSynchronize(s));
      return CR_OK;
    }
    CR_TRY(hipMemcpyAsync(P->w.cg_b, P->w.cg_r, vbytes, hipMemcpyDeviceToDevice, s));
    o.tol = opts->tol / rmax * (1.0 - 1e-12);   // (so that the rescaled residuals meet tol)
  }
  std::vector<int> iters, refine, broke;
  std::vector<double> rel;
  if (o.prec == CR_MIXED) {
    CR_CHECK(solve_refined(P, nrhs, prob->ninv, &o, iters, refine, rel, broke, s, pc));
  } else {
    CR_CHECK(pcg_run(P, nrhs, prob->ninv, P->w.cg_b, o.tol, o.maxiter, every, false, true, iters, rel, broke, s,
                     o.use_graph != 0, pc));
    refine.assign(nrhs, 0);
  }
  for (int c = 0; c < nrhs; ++c) rel[c] *= r0[c];
  fill_stats(nrhs, opts->tol, iters, refine, rel, broke, stats);
  if (x0)
    CR_TRY(launch_alm_axpby((int64_t)nrhs * vlen(P), 1.0, C2(x0), 1.0, P->w.cg_x, C2(s_out), s));
  else
    CR_TRY(hipMemcpyAsync(s_out, P->w.cg_x, vbytes, hipMemcpyDeviceToDevice, s));
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

// t = a^T S^-1 a (real-field product, the problem's current S^-1) into host *t
int quad_sinv(const crsht_plan* P, const double2* a, double* t, hipStream_t s) {
  const int npart = P->w.npart;
  const int nba = std::min<int64_t>(npart, (P->g.nalm + 255) / 256);
  double* pa = P->w.partial;
  CR_TRY(hipMemsetAsync(pa, 0, 3 * (size_t)npart * sizeof(double), s));
  CR_TRY(launch_alm_wquad(P, P->w.sinv, a, pa, nba, s));
  CR_TRY(launch_sum_rows(P, 1, nba, s));
  CR_CHECK(read_scalars(P, 1, s));
  *t = P->w.host_scal[S_AUX0];
  return CR_OK;
}

// terms of ln pi into host t[3]: chi^2 of the mean field, a^T S^-1 a, f^T B^T N^-1 B f
// T+Q+U: chi^2 and the fluctuation term summed over T, Q, U (maps
// [3][npix], ninv [3][npix]); the prior with the 3x3 blocks of S^-1
int lnpi_terms_tqu(const crsht_plan* P, const double* ninv, const double* d, const double2* ahat, const double2* fhat,
                   double t[3], hipStream_t s) {
  const int npart = P->w.npart;
  const int nbp = std::min<int64_t>(npart, (P->g.npix + 255) / 256);
  const int nba = std::min<int64_t>(npart, (P->g.nalm + 255) / 256);
  const int64_t np = P->g.npix;
  double* pa = P->w.partial;
  auto sum3 = [&](int nb) -> double {
    if (launch_sum_rows(P, 1, nb, s) != hipSuccess) return NAN;
    if (read_scalars(P, 1, s) != CR_OK) return NAN;
    return P->w.host_scal[S_AUX0] + P->w.host_scal[S_AUX1] + P->w.host_scal[S_AUX2];
  };
  // chi^2: rows 0..2 = T, Q, U
  CR_TRY(hipMemsetAsync(pa, 0, 3 * (size_t)npart * sizeof(double), s));
  CR_CHECK(synth_f64(P, 1, ahat, P->w.bl_keep, P->w.map_a, s));
  for (int k = 0; k < 3; ++k)
    CR_TRY(launch_pix_wsq(P, ninv + k * np, d + k * np, P->w.map_a + k * np, pa + k * npart, nbp, s));
  t[0] = sum3(nbp);
  // prior: row 0
  CR_TRY(hipMemsetAsync(pa, 0, 3 * (size_t)npart * sizeof(double), s));
  CR_TRY(launch_alm_wquad_tqu(P, ahat, pa, nba, s));
  t[1] = sum3(nba);
  // fluctuation term: rows 0..2 = T, Q, U
  CR_TRY(hipMemsetAsync(pa, 0, 3 * (size_t)npart * sizeof(double), s));
  CR_CHECK(synth_f64(P, 1, fhat, P->w.bl_keep, P->w.map_a, s));
  for (int k = 0; k < 3; ++k)
    CR_TRY(launch_pix_wsq(P, ninv + k * np, P->w.map_a + k * np, nullptr, pa + k * npart, nbp, s));
  t[2] = sum3(nbp);
  if (!std::isfinite(t[0]) || !std::isfinite(t[1]) || !std::isfinite(t[2])) return CR_EDEVICE;
  return CR_OK;
}

int lnpi_terms(const crsht_plan* P, const double* ninv, const double* d, const double2* ahat, const double2* fhat,
               double t[3], hipStream_t s) {
  if (P->ncomp == 3) return lnpi_terms_tqu(P, ninv, d, ahat, fhat, t, s);
  const int npart = P->w.npart;
  const int nbp = std::min<int64_t>(npart, (P->g.npix + 255) / 256);
  const int nba = std::min<int64_t>(npart, (P->g.nalm + 255) / 256);
  double* pa = P->w.partial;
  CR_TRY(hipMemsetAsync(pa, 0, 3 * (size_t)npart * sizeof(double), s));
  // Y B ahat
  CR_CHECK(synth_f64(P, 1, ahat, P->w.bk, P->w.map_a, s));
  CR_TRY(launch_pix_wsq(P, ninv, d, P->w.map_a, pa, nbp, s));
  CR_TRY(launch_alm_wquad(P, P->w.sinv, ahat, pa + npart, nba, s));
  CR_CHECK(synth_f64(P, 1, fhat, P->w.bk, P->w.map_a, s));
  CR_TRY(launch_pix_wsq(P, ninv, P->w.map_a, nullptr, pa + 2 * npart, nbp, s));
  CR_TRY(launch_sum_rows(P, 1, std::max(nbp, nba), s));
  CR_CHECK(read_scalars(P, 1, s));
  t[0] = P->w.host_scal[S_AUX0];
  t[1] = P->w.host_scal[S_AUX1];
  t[2] = P->w.host_scal[S_AUX2];
  return CR_OK;
}

// lnpi_terms of n columns at once: ahat, fhat device [n][nalm]; the
// syntheses of all columns in one launch each; t host [n][3]
int lnpi_terms_batch(const crsht_plan* P, int n, const double* ninv, const double* d, const double2* ahat,
                     const double2* fhat, double* t, hipStream_t s) {
  const int npart = P->w.npart;
  const int nbp = std::min<int64_t>(npart, (P->g.npix + 255) / 256);
  const int nba = std::min<int64_t>(npart, (P->g.nalm + 255) / 256);
  const int64_t na = P->g.nalm, np = P->g.npix;
  double* pa = P->w.partial;
  CR_TRY(hipMemsetAsync(pa, 0, 4 * (size_t)n * npart * sizeof(double), s));
  CR_CHECK(synth_f64(P, n, ahat, P->w.bk, P->w.map_a, s));
  for (int c = 0; c < n; ++c) {
    double* pc = pa + (size_t)c * npart * 4;
    CR_TRY(launch_pix_wsq(P, ninv, d, P->w.map_a + c * np, pc, nbp, s));
    CR_TRY(launch_alm_wquad(P, P->w.sinv, ahat + c * na, pc + npart, nba, s));
  }
  CR_CHECK(synth_f64(P, n, fhat, P->w.bk, P->w.map_a, s));
  for (int c = 0; c < n; ++c)
    CR_TRY(launch_pix_wsq(P, ninv, P->w.map_a + c * np, nullptr, pa + (size_t)c * npart * 4 + 2 * npart, nbp, s));
  CR_TRY(launch_sum_rows(P, n, std::max(nbp, nba), s));
  CR_CHECK(read_scalars(P, n, s));
  for (int c = 0; c < n; ++c) {
    const double* sc = P->w.host_scal + c * kScalSlots;
    t[3 * c] = sc[S_AUX0];
    t[3 * c + 1] = sc[S_AUX1];
    t[3 * c + 2] = sc[S_AUX2];
  }
  return CR_OK;
}

}  // namespace

// ============================================================== transforms

extern "C" int sht_synth(const crsht_plan* P, int nrhs, const double* alm, double* map, cr_prec prec,
                         void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (!alm || !map) return CR_EINVAL;
  if (!transform_prec(prec)) return CR_EINVAL;
  SplitScope sc(P, prec);
  return synth_f64(P, nrhs, C2(alm), P->t.rec_kappa, map, S(stream), prec != CR_F64);
}

extern "C" int sht_synth_adjoint(const crsht_plan* P, int nrhs, const double* map, double* alm, cr_prec prec,
                                 void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (!alm || !map) return CR_EINVAL;
  if (!transform_prec(prec)) return CR_EINVAL;
  SplitScope sc(P, prec);
  return adjoint_f64(P, nrhs, map, C2(alm), S(stream), prec != CR_F64);
}

extern "C" int sht_analysis(const crsht_plan* P, int nrhs, const double* map, double* alm, int n_iter,
                            void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (!alm || !map || n_iter < 0) return CR_EINVAL;
  hipStream_t s = S(stream);
  const double wq = 4.0 * M_PI / (double)P->g.npix;
  const int64_t na = (int64_t)nrhs * vlen(P), np = (int64_t)nrhs * P->ncomp * P->g.npix;
  CR_CHECK(adjoint_f64(P, nrhs, map, C2(alm), s));
  CR_TRY(launch_alm_axpby(na, wq, C2(alm), 0.0, nullptr, C2(alm), s));
  for (int it = 0; it < n_iter; ++it) {
    CR_CHECK(synth_f64(P, nrhs, C2(alm), P->t.rec_kappa, P->w.map_a, s));
    CR_TRY(launch_map_axpby(np, 1.0, map, -1.0, P->w.map_a, P->w.map_a, s));
    CR_CHECK(adjoint_f64(P, nrhs, P->w.map_a, P->w.alm_b, s));
    CR_TRY(launch_alm_axpby(na, 1.0, C2(alm), wq, P->w.alm_b, C2(alm), s));
  }
  return CR_OK;
}

// ============================================================== CR system
extern "C" int cr_white(const crsht_plan* P, int nrhs, uint64_t seed, uint64_t counter, double* w0, double* w1,
                        void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (!w0 && !w1) return CR_EINVAL;
  CR_TRY(launch_white(P, nrhs * P->ncomp, seed, counter, reinterpret_cast<double2*>(w0), w1, S(stream)));
  return CR_OK;
}

extern "C" int cr_precond(const crsht_plan* P, const cr_problem* prob, double* diag, void* stream) {
  CR_CHECK(check_plan(P, 1));
  if (!diag) return CR_EINVAL;
  hipStream_t s = S(stream);
  CR_CHECK(set_problem(P, prob, 1.0, s));
  CR_CHECK(compute_diag(P, prob->ninv, s));
  CR_TRY(hipMemcpyAsync(diag, P->w.diag, vlen(P) * sizeof(double), hipMemcpyDeviceToDevice, s));
  return CR_OK;
}

extern "C" int cr_block_precond_build(crsht_plan* P, const cr_problem* prob, void* stream) {
  CR_CHECK(check_plan(P, 1));
  if (!prob || !prob->ninv) return CR_EINVAL;
  hipStream_t s = S(stream);
  CR_CHECK(set_problem(P, prob, 1.0, s));   // validates the spectrum, beam and lmin; per-l arrays
  return block_pc_build(P, prob->lmin, prob->ninv, s);
}

extern "C" int cr_block_precond_apply(const crsht_plan* P, int nrhs, const double* r, double* z, void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (!r || !z || r == z) return CR_EINVAL;
  if (!P->pc.built) return CR_EINVAL;
  CR_TRY(launch_pc_apply(P, nrhs, C2(r), C2(z), S(stream)));
  return CR_OK;
}

extern "C" int cr_rhs(const crsht_plan* P, const cr_problem* prob, int nrhs, const double* d, const double* w0,
                      const double* w1, double* b, void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (!b) return CR_EINVAL;
  hipStream_t s = S(stream);
  CR_CHECK(set_problem(P, prob, 1.0, s, nrhs));
  return assemble_rhs(P, nrhs, prob->ninv, d, w0, w1, C2(b), s);
}

extern "C" int cr_apply(const crsht_plan* P, const cr_problem* prob, int nrhs, const double* x, double* Ax,
                        cr_prec prec, void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (!x || !Ax) return CR_EINVAL;
  if (!transform_prec(prec)) return CR_EINVAL;
  hipStream_t s = S(stream);
  CR_CHECK(set_problem(P, prob, 1.0, s, nrhs));
  CR_TRY(launch_project(P, nrhs, C2(x), P->w.cg_d, s));
  if (P->ncomp == 1) CR_TRY(launch_scale_alm(P, nrhs, P->w.cg_d, P->w.bk, P->w.alm_a, s));
  SplitScope sc(P, prec);
  return operator_core(P, nrhs, P->w.cg_d, P->w.alm_a, prob->ninv, C2(Ax), s, prec != CR_F64);
}

// CR_SEPARATE: the right-hand sides of the d term and of the w0, w1 terms of
// every column, assembled as two blocks of nrhs columns and interleaved into
// s_out (mean field, fluctuation per column), solved as 2 nrhs columns with
// the amplitudes repeated; the solution overwrites its right-hand side.
int solve_separate(const crsht_plan* P, const cr_problem* prob, int nrhs, const double* d, const double* w0,
                   const double* w1, double* s_out, const cr_opts* opts, cr_stats* stats, hipStream_t s) {
  if (!prob || !opts || !stats || !s_out || !d || (!w0 && !w1)) return CR_EINVAL;
  if (2 * nrhs > P->nrhs_max) return CR_EINVAL;
  Workspace const& w = P->w;
  const size_t vb = (size_t)vlen(P) * sizeof(double2);
  CR_CHECK(set_problem(P, prob, 1.0, s, nrhs));
  CR_CHECK(assemble_rhs(P, nrhs, prob->ninv, d, nullptr, nullptr, w.cg_xacc, s));
  CR_CHECK(assemble_rhs(P, nrhs, prob->ninv, nullptr, w0, w1, w.cg_bin, s));
  CR_TRY(hipMemcpy2DAsync(s_out, 2 * vb, w.cg_xacc, vb, vb, nrhs, hipMemcpyDeviceToDevice, s));
  CR_TRY(hipMemcpy2DAsync(reinterpret_cast<char*>(s_out) + vb, 2 * vb, w.cg_bin, vb, vb, nrhs,
                          hipMemcpyDeviceToDevice, s));
  cr_problem p2 = *prob;
  std::vector<double> amp2;
  if (prob->amp) {
    amp2.resize(2 * (size_t)nrhs);
    for (int c = 0; c < nrhs; ++c) amp2[2 * c] = amp2[2 * c + 1] = prob->amp[c];
    p2.amp = amp2.data();
  }
  cr_opts o = *opts;
  o.terms = CR_SUM;
  return solve_core(P, &p2, 1.0, 2 * nrhs, nullptr, nullptr, nullptr, s_out, s_out, &o, stats, s);
}

extern "C" int cr_solve(const crsht_plan* P, const cr_problem* prob, int nrhs, const double* d, const double* w0,
                        const double* w1, const double* rhs, double* s_out, const cr_opts* opts, cr_stats* stats,
                        void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (opts && opts->terms == CR_SEPARATE) {
    if (rhs) return CR_EINVAL;
    return solve_separate(P, prob, nrhs, d, w0, w1, s_out, opts, stats, S(stream));
  }
  if (opts && opts->terms != CR_SUM) return CR_EINVAL;
  return solve_core(P, prob, 1.0, nrhs, d, w0, w1, rhs, s_out, opts, stats, S(stream));
}

extern "C" int cr_solve_async(const crsht_plan* P, const cr_problem* prob, int nrhs, const double* d,
                              const double* w0, const double* w1, const double* rhs, double* s_out,
                              const cr_opts* opts, cr_stats* stats_dev, void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (!s_out || !stats_dev) return CR_EINVAL;
  DSolve ds;
  CR_CHECK(dsolve_setup(ds, P, prob, nrhs, opts));
  hipStream_t s = S(stream);
  bool graphs = false;
  CR_CHECK(dsolve_graphs(ds, opts->use_graph != 0, &graphs));
  CR_CHECK(dsolve_prologue(ds, prob, d, w0, w1, rhs, s));
  for (int k = 0; k < ds.steps; ++k) CR_CHECK(dsolve_launch(ds, k, graphs, s));
  CR_CHECK(dsolve_epilogue(ds, s_out, stats_dev, s));
  CR_TRY(hipGetLastError());
  return CR_OK;
}

extern "C" int cr_solve_batched(const crsht_plan* const* plans, const cr_problem* probs, int nprob,
                                const double* const* d, const double* const* w0, const double* const* w1,
                                double* const* s_out, const cr_opts* opts, cr_stats* stats, void* stream) {
  if (!plans || !probs || nprob < 1 || !s_out || !opts || !stats) return CR_EINVAL;
  for (int i = 0; i < nprob; ++i) {
    CR_CHECK(check_plan(plans[i], 1));
    if (!s_out[i]) return CR_EINVAL;
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return CR_EINVAL;   // each problem needs its own workspace
  }
  int dev = -1;
  CR_TRY(hipGetDevice(&dev));
  for (int i = 0; i < nprob; ++i)
    if (plans[i]->device != dev) return CR_EINVAL;
  hipStream_t s = S(stream);
  // the problems run concurrently on their plans' streams: no forked
  // launches inside them for the duration of the call
  struct AuxOff {
    const crsht_plan* const* p;
    int n;
    ~AuxOff() {
      for (int i = 0; i < n; ++i) p[i]->aux_off = false;
    }
  } aux_guard{plans, nprob};
  for (int i = 0; i < nprob; ++i) plans[i]->aux_off = true;
  std::vector<DSolve> ds(nprob);
  std::vector<char> graphs(nprob, 0);
  for (int i = 0; i < nprob; ++i) {
    CR_CHECK(dsolve_setup(ds[i], plans[i], &probs[i], 1, opts));
    bool g = false;
    CR_CHECK(dsolve_graphs(ds[i], opts->use_graph != 0, &g));
    graphs[i] = g ? 1 : 0;
  }
  // largest problems first
  std::vector<int> order(nprob);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return plans[a]->g.npix * (int64_t)plans[a]->g.lmax > plans[b]->g.npix * (int64_t)plans[b]->g.lmax;
  });
  // every problem on its plan's stream, after the caller's stream has
  // produced the inputs
  for (int i : order) {
    const crsht_plan* P = plans[i];
    CR_TRY(hipEventRecord(P->ev_fork, s));
    CR_TRY(hipStreamWaitEvent(P->exec_stream, P->ev_fork, 0));
    *reinterpret_cast<volatile int*>(P->w.host_exited) = 0;
    CR_CHECK(dsolve_prologue(ds[i], &probs[i], d ? d[i] : nullptr, w0 ? w0[i] : nullptr, w1 ? w1[i] : nullptr,
                             nullptr, P->exec_stream));
  }
  // blocks of every problem until its solve has stopped: block r of a
  // problem is enqueued once its block r - 2 has run (two in flight) and the
  // device has not yet flagged the problem as stopped
  std::vector<char> stopped(nprob, 0);
  const int R = crsht_plan::kRoundEvents;
  for (int r = 0;; ++r) {
    bool any = false;
    for (int i : order) {
      if (stopped[i]) continue;
      const crsht_plan* P = plans[i];
      if (r >= ds[i].steps) {
        stopped[i] = 1;
        continue;
      }
      if (r >= 2) {
        CR_TRY(hipEventSynchronize(P->ev_round[(r - 2) % R]));
        if (*reinterpret_cast<volatile int*>(P->w.host_exited) != 0) {
          stopped[i] = 1;
          continue;
        }
      }
      CR_CHECK(dsolve_launch(ds[i], r, graphs[i] != 0, P->exec_stream));
      CR_TRY(hipEventRecord(P->ev_round[r % R], P->exec_stream));
      any = true;
    }
    if (!any) break;
  }
  for (int i : order) {
    const crsht_plan* P = plans[i];
    CR_CHECK(dsolve_epilogue(ds[i], s_out[i], P->w.dstats, P->exec_stream));
    CR_TRY(hipEventRecord(P->ev_join, P->exec_stream));
    CR_TRY(hipStreamWaitEvent(s, P->ev_join, 0));
  }
  CR_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < nprob; ++i)
    CR_TRY(hipMemcpy(&stats[i], plans[i]->w.dstats, sizeof(cr_stats), hipMemcpyDeviceToHost));
  return CR_OK;
}

extern "C" int cr_lnpi(const crsht_plan* P, const cr_problem* fid, double q, const double* d, const double* ahat,
                       const double* fhat, double* lnpi, void* stream) {
  CR_CHECK(check_plan(P, 1));
  if (!d || !ahat || !fhat || !lnpi) return CR_EINVAL;
  hipStream_t s = S(stream);
  CR_CHECK(set_problem(P, fid, q, s));
  double t[3];
  CR_CHECK(lnpi_terms(P, fid->ninv, d, C2(ahat), C2(fhat), t, s));
  *lnpi = -0.5 * (t[0] + t[1] + t[2]);
  return CR_OK;
}

extern "C" int sht_synth_grad(const crsht_plan* P, int nrhs, const double* map_grad, double* alm_grad,
                              cr_prec prec, void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (!map_grad || !alm_grad) return CR_EINVAL;
  if (!transform_prec(prec)) return CR_EINVAL;
  hipStream_t s = S(stream);
  {
    SplitScope sc(P, prec);
    CR_CHECK(adjoint_f64(P, nrhs, map_grad, C2(alm_grad), s, prec != CR_F64));
  }
  CR_TRY(launch_mweight(P, nrhs, C2(alm_grad), s));
  return CR_OK;
}

extern "C" int cr_grad_chi2(const crsht_plan* P, const cr_problem* prob, int nrhs, const double* d, const double* a,
                            double* grad, double* chi2, void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (!prob || !d || !a || !grad) return CR_EINVAL;
  hipStream_t s = S(stream);
  CR_CHECK(set_problem(P, prob, 1.0, s));
  const int64_t np = P->g.npix;
  const int nc = P->ncomp;
  // model map Y B a (B restricted to the kept modes) and chi^2 per column
  CR_CHECK(synth_f64(P, nrhs, C2(a), nc == 3 ? P->w.bl_keep : P->w.bk, P->w.map_a, s));
  if (chi2) {
    const int npart = P->w.npart;
    const int nbp = std::min<int64_t>(npart, (np + 255) / 256);
    for (int c = 0; c < nrhs; ++c) {
      for (int k = 0; k < 3; ++k) {   // one partial row per component (rows unused by T plans hold 0)
        const int64_t off = ((int64_t)c * nc + k) * np;
        if (k < nc)
          CR_TRY(launch_pix_wsq(P, prob->ninv + k * np, d + off, P->w.map_a + off, P->w.partial + k * npart, nbp, s));
        else
          CR_TRY(hipMemsetAsync(P->w.partial + k * npart, 0, nbp * sizeof(double), s));
      }
      CR_TRY(launch_sum_rows(P, 1, nbp, s));
      CR_CHECK(read_scalars(P, 1, s));
      const double* sc = P->w.host_scal;
      chi2[c] = sc[S_AUX0] + sc[S_AUX1] + sc[S_AUX2];
    }
  }
  // g = -2 B Y^T N^-1 (d - Y B a)
  CR_TRY(launch_pix_wres(P, nrhs, prob->ninv, d, P->w.map_a, P->w.map_a, s));
  if (nc == 3) {
    CR_TRY(launch_ring(P, 3 * nrhs, RING_ADJOINT, nullptr, P->w.map_a, nullptr, P->w.geo, false, s, tqu_cols(P)));
    CR_CHECK(tqu_from_geo(P, nrhs, P->w.bl_keep, C2(grad), s, false));
  } else {
    CR_TRY(launch_ring(P, nrhs, RING_ADJOINT, nullptr, P->w.map_a, nullptr, P->w.geo, false, s));
    CR_TRY(launch_legendre_adjoint(P, nrhs, P->w.geo, P->w.alm_b, false, s));   // raw sums (no kappa)
    CR_TRY(launch_scale_alm(P, nrhs, P->w.alm_b, P->w.bk, C2(grad), s));          // b_l kappa_lm on kept modes
  }
  CR_TRY(launch_alm_axpby((int64_t)nrhs * vlen(P), -2.0, C2(grad), 0.0, nullptr, C2(grad), s));
  CR_TRY(launch_project(P, nrhs, C2(grad), C2(grad), s));
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

extern "C" int cr_grad_lnpi(const crsht_plan* P, const cr_problem* prob, const double* d, const double* w0,
                            const double* w1, int nbins, const int* edges, const cr_opts* opts, double* grad,
                            double* lnpi, cr_stats* stats, void* stream) {
  CR_CHECK(check_plan(P, 1));
  if (prob && prob->amp) return CR_EINVAL;   // one spectrum per call
  if (!prob || !d || !edges || !opts || !grad || !lnpi || !stats) return CR_EINVAL;
  if (nbins < 1 || nbins > P->g.lmax + 1) return CR_EINVAL;
  for (int k = 0; k <= nbins; ++k) {
    if (edges[k] < 0 || edges[k] > P->g.lmax + 1) return CR_EINVAL;
    if (k > 0 && edges[k] <= edges[k - 1]) return CR_EINVAL;
  }
  hipStream_t s = S(stream);
  Workspace const& w = P->w;
  const int64_t na = P->g.nalm;
  // mean field a^ (alm_c) and fluctuation f^ (alm_d)
  CR_CHECK(solve_core(P, prob, 1.0, 1, d, nullptr, nullptr, nullptr, reinterpret_cast<double*>(w.alm_c), opts,
                      &stats[0], s));
  CR_CHECK(solve_core(P, prob, 1.0, 1, nullptr, w0, w1, nullptr, reinterpret_cast<double*>(w.alm_d), opts,
                      &stats[1], s));
  // u = M f^ = B Y^T N^-1 Y B f^ (cg_bin), then the adjoint solve lambda = A^-1 u (cg_xacc)
  CR_TRY(launch_scale_alm(P, 1, w.alm_d, w.bk, w.alm_a, s));
  CR_CHECK(operator_core(P, 1, w.alm_d, w.alm_a, prob->ninv, w.cg_bin, s, false, false));
  CR_CHECK(solve_core(P, prob, 1.0, 1, nullptr, nullptr, nullptr, reinterpret_cast<const double*>(w.cg_bin),
                      reinterpret_cast<double*>(w.cg_xacc), opts, &stats[2], s));
  // per-bin terms (problem factors sinv, sinvhalf are those of prob)
  CR_TRY(hipMemcpyAsync(w.bin_edges, edges, (size_t)(nbins + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  if (P->ncomp == 3) {
    // the 3x3 blocks: S^-1 a (cg_r), S^-1/2 w0 (cg_z), S^-1 f (cg_p), then per-bin dots
    const int64_t nv = vlen(P);
    CR_TRY(hipMemsetAsync(w.alm_b, 0, (size_t)nv * sizeof(double2), s));
    CR_TRY(launch_cg_q_tqu(P, 1, w.alm_c, w.alm_b, w.cg_r, s, true));
    CR_TRY(launch_cg_q_tqu(P, 1, w.alm_d, w.alm_b, w.cg_p, s, true));
    if (w0) CR_TRY(launch_rhs_finish_tqu(P, 1, nullptr, C2(w0), w.cg_z, s));
    CR_TRY(launch_bin_grad_dots(P, nbins, w.bin_edges, w.alm_c, w.cg_r, w0 ? w.cg_xacc : nullptr,
                                w0 ? w.cg_z : nullptr, w.cg_xacc, w.cg_p, w.bin_grad, s));
  } else {
    CR_TRY(launch_bin_grad(P, nbins, w.bin_edges, w.alm_c, w.alm_d, w.cg_xacc, w0 ? C2(w0) : nullptr, w.bin_grad,
                           s));
  }
  CR_TRY(hipMemcpyAsync(grad, w.bin_grad, (size_t)nbins * sizeof(double), hipMemcpyDeviceToHost, s));
  CR_TRY(hipStreamSynchronize(s));
  double t[3];
  CR_CHECK(lnpi_terms(P, prob->ninv, d, w.alm_c, w.alm_d, t, s));
  *lnpi = -0.5 * (t[0] + t[1] + t[2]);
  (void)na;
  return CR_OK;
}

extern "C" int joint_cl_step(const crsht_plan* P, const cr_problem* fid, const double* d, cr_chain* state,
                             const cr_draws* dr, const cr_opts* opts, cr_step_out* out, void* stream) {
  CR_CHECK(check_plan(P, 1));
  if (fid && fid->amp) return CR_EINVAL;   // one spectrum per call
  if (!fid || !d || !state || !dr || !opts || !out || !state->ahat || !state->fhat) return CR_EINVAL;
  if (!(dr->sigma_lnq > 0.0) || !(dr->u > 0.0 && dr->u < 1.0) || !std::isfinite(dr->xi)) return CR_EINVAL;
  if (!(state->q > 0.0) || !std::isfinite(state->lnpi)) return CR_EINVAL;
  if (!dr->w0 && !dr->w1) return CR_EINVAL;   // the fluctuation of an accepted move needs a random term
  hipStream_t s = S(stream);
  std::memset(out, 0, sizeof(*out));
  const double qn = state->q * std::exp(dr->sigma_lnq * dr->xi);
  out->q_new = qn;
  // 1) mean field at q', warm-started from the mean field at q
  double* ahat_n = reinterpret_cast<double*>(P->w.alm_c);
  CR_CHECK(solve_core(P, fid, qn, 1, d, nullptr, nullptr, nullptr, ahat_n, opts, &out->mean_stats, s, state->ahat));
  // 2) rescaled fluctuation sqrt(q'/q) f
  const int64_t na = vlen(P);   // coefficients of one state (3 nalm for T+Q+U)
  CR_TRY(launch_alm_axpby(na, std::sqrt(qn / state->q), C2(state->fhat), 0.0, nullptr, P->w.alm_d, s));
  // 3) ln pi(q') and ln A (problem factors are still those of q')
  double t[3];
  CR_CHECK(lnpi_terms(P, fid->ninv, d, P->w.alm_c, P->w.alm_d, t, s));
  out->lnpi_new = -0.5 * (t[0] + t[1] + t[2]);
  out->lnA = out->lnpi_new - state->lnpi + std::log(qn / state->q);
  out->accepted = std::log(dr->u) < out->lnA ? 1 : 0;
  if (!out->accepted) return CR_OK;
  // 4) accepted: fresh fluctuation at q', then ln pi of the new state
  CR_CHECK(solve_core(P, fid, qn, 1, nullptr, dr->w0, dr->w1, nullptr, state->fhat, opts, &out->fluct_stats, s));
  CR_TRY(hipMemcpyAsync(state->ahat, P->w.alm_c, na * sizeof(double2), hipMemcpyDeviceToDevice, s));
  CR_CHECK(lnpi_terms(P, fid->ninv, d, P->w.alm_c, C2(state->fhat), t, s));
  state->q = qn;
  state->lnpi = -0.5 * (t[0] + t[1] + t[2]);
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

extern "C" int joint_cl_step_batch(const crsht_plan* P, const cr_problem* fid, const double* d, int n,
                                   cr_chain* st, const double* xi, const double* u, double sigma_lnq,
                                   const double* w0, const double* w1, const cr_opts* opts, cr_step_out* out,
                                   void* stream) {
  CR_CHECK(check_plan(P, n));
  if (P->ncomp != 1) return CR_ENOTSUP;
  if (!fid || !d || !st || !xi || !u || !opts || !out || (!w0 && !w1)) return CR_EINVAL;
  if (fid->amp) return CR_EINVAL;   // the move sets the columns' amplitudes itself
  if (!(sigma_lnq > 0.0) || !std::isfinite(sigma_lnq)) return CR_EINVAL;
  for (int c = 0; c < n; ++c) {
    if (!st[c].ahat || !st[c].fhat || !(st[c].q > 0.0) || !std::isfinite(st[c].q) || !std::isfinite(st[c].lnpi))
      return CR_EINVAL;
    if (!(u[c] > 0.0 && u[c] < 1.0) || !std::isfinite(xi[c])) return CR_EINVAL;
  }
  hipStream_t s = S(stream);
  Workspace const& w = P->w;
  const int64_t na = P->g.nalm;
  const size_t cb = (size_t)na * sizeof(double2);
  std::memset(out, 0, (size_t)n * sizeof(cr_step_out));
  std::vector<double> qn(n);
  for (int c = 0; c < n; ++c) qn[c] = out[c].q_new = st[c].q * std::exp(sigma_lnq * xi[c]);
  // 1) the data term B Y^T N^-1 d of the mean-field right-hand side does not
  //    depend on the spectrum: one column, copied to every chain's
  CR_CHECK(set_problem(P, fid, 1.0, s));
  CR_CHECK(assemble_rhs(P, 1, fid->ninv, d, nullptr, nullptr, w.cg_bin, s));
  for (int c = 1; c < n; ++c)
    CR_TRY(hipMemcpyAsync(w.cg_bin + (size_t)c * na, w.cg_bin, cb, hipMemcpyDeviceToDevice, s));
  // 2) mean fields at q'_c, one column per chain, warm-started from the chains' mean fields
  for (int c = 0; c < n; ++c)
    CR_TRY(hipMemcpyAsync(w.cg_xacc + (size_t)c * na, st[c].ahat, cb, hipMemcpyDeviceToDevice, s));
  cr_problem pa = *fid;
  pa.amp = qn.data();
  std::vector<cr_stats> ms(n), fs(n);
  CR_CHECK(solve_core(P, &pa, 1.0, n, nullptr, nullptr, nullptr, reinterpret_cast<const double*>(w.cg_bin),
                      reinterpret_cast<double*>(w.cg_xacc), opts, ms.data(), s,
                      reinterpret_cast<const double*>(w.cg_xacc)));
  // 3) ln pi(q'_c) with the rescaled fluctuation, ln A, decisions. The
  //    problem factors are those of the fiducial spectrum: the prior term is
  //    divided by q'_c.
  bool any = false;
  std::vector<double> t(3 * (size_t)n);
  for (int c = 0; c < n; ++c)   // rescaled fluctuations into cg_bin (its right-hand sides are consumed)
    CR_TRY(launch_alm_axpby(na, std::sqrt(qn[c] / st[c].q), C2(st[c].fhat), 0.0, nullptr,
                            w.cg_bin + (size_t)c * na, s));
  CR_CHECK(lnpi_terms_batch(P, n, fid->ninv, d, w.cg_xacc, w.cg_bin, t.data(), s));
  for (int c = 0; c < n; ++c) {
    out[c].mean_stats = ms[c];
    out[c].lnpi_new = -0.5 * (t[3 * c] + t[3 * c + 1] / qn[c] + t[3 * c + 2]);
    out[c].lnA = out[c].lnpi_new - st[c].lnpi + std::log(qn[c] / st[c].q);
    out[c].accepted = std::log(u[c]) < out[c].lnA ? 1 : 0;
    any = any || out[c].accepted;
  }
  if (!any) return CR_OK;
  // 4) fresh fluctuations at q'_c in one solve of every column (the columns of
  //    rejected chains are computed alongside and discarded)
  CR_CHECK(solve_core(P, &pa, 1.0, n, nullptr, w0, w1, nullptr, reinterpret_cast<double*>(w.cg_bin), opts, fs.data(),
                      s));
  // 5) accepted chains take the new mean field, fluctuation, amplitude and ln
  //    pi (evaluated for every column in one batch)
  CR_CHECK(lnpi_terms_batch(P, n, fid->ninv, d, w.cg_xacc, w.cg_bin, t.data(), s));
  for (int c = 0; c < n; ++c) {
    if (!out[c].accepted) continue;
    out[c].fluct_stats = fs[c];
    CR_TRY(hipMemcpyAsync(st[c].ahat, w.cg_xacc + (size_t)c * na, cb, hipMemcpyDeviceToDevice, s));
    CR_TRY(hipMemcpyAsync(st[c].fhat, w.cg_bin + (size_t)c * na, cb, hipMemcpyDeviceToDevice, s));
    st[c].q = qn[c];
    st[c].lnpi = -0.5 * (t[3 * c] + t[3 * c + 1] / qn[c] + t[3 * c + 2]);
  }
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

// ---- HMC move of per-bin log-amplitudes at fixed whitened fluctuation
namespace {

bool valid_bins(const crsht_plan* P, int nbins, const int* edges) {
  if (nbins < 1 || nbins > P->g.lmax + 1 || !edges) return false;
  for (int k = 0; k <= nbins; ++k) {
    if (edges[k] < 0 || edges[k] > P->g.lmax + 1) return false;
    if (k > 0 && edges[k] <= edges[k - 1]) return false;
  }
  return true;
}

// per-l factor exp(c * x_k) on [edges[k], edges[k+1]), 1 elsewhere
void bin_factor(int lmax, int nbins, const int* edges, const double* x, double c, std::vector<double>& f) {
  f.assign(lmax + 1, 1.0);
  for (int k = 0; k < nbins; ++k)
    for (int l = edges[k]; l < edges[k + 1]; ++l) f[l] = std::exp(c * x[k]);
}

// ln pi at the log-amplitudes theta (C_l -> C_l exp(theta_k) per bin) with the
// fluctuation f0, given at theta0, rescaled by exp((theta - theta0)/2) per bin
// (the whitened fluctuation S^-1/2 f held fixed), and its gradient in theta:
//   d ln pi / d theta_k = 1/2 a^T S^-1_k a - 1/2 f^T M f_k,  M = B Y^T N^-1 Y B
// (the mean field a minimises chi^2 + a^T S^-1 a, so it enters only through
// the explicit S^-1; f_k changes as f_k / 2). The mean field (warm-started
// from a0, which may alias w.alm_c) goes to w.alm_c, the rescaled
// fluctuation to w.alm_d; edges are already in w.bin_edges.
int lnpi_grad_u(const crsht_plan* P, const cr_problem* fid, const double* d, int nbins, const int* edges,
                const double* theta0, const double* theta, const double* f0, const double* a0, const cr_opts* opts,
                double* lnpi, double* grad, cr_stats* st, hipStream_t s, const double* rhs_d = nullptr) {
  Workspace const& w = P->w;
  const int lmax = P->g.lmax;
  std::vector<double> fac, cl(lmax + 1), dth(nbins), lf;
  bin_factor(lmax, nbins, edges, theta, 1.0, fac);
  for (int l = 0; l <= lmax; ++l) cl[l] = fid->cl[l] * fac[l];
  cr_problem pr = *fid;
  pr.cl = cl.data();
  // the mean-field right-hand side B Y^T N^-1 d does not depend on theta: rhs_d,
  // when given, holds it (device, [nalm]) and spares its adjoint transform
  CR_CHECK(solve_core(P, &pr, 1.0, 1, rhs_d ? nullptr : d, nullptr, nullptr, rhs_d,
                      reinterpret_cast<double*>(w.alm_c), opts, st, s, a0));
  for (int k = 0; k < nbins; ++k) dth[k] = theta[k] - theta0[k];
  bin_factor(lmax, nbins, edges, dth.data(), 0.5, lf);
  CR_TRY(hipMemcpyAsync(w.lfac, lf.data(), (size_t)(lmax + 1) * sizeof(double), hipMemcpyHostToDevice, s));
  CR_TRY(launch_scale_per_l(P, C2(f0), w.lfac, w.alm_d, s));
  double t[3];
  CR_CHECK(lnpi_terms(P, fid->ninv, d, w.alm_c, w.alm_d, t, s));   // (synchronises: lf may go)
  *lnpi = -0.5 * (t[0] + t[1] + t[2]);
  CR_TRY(launch_scale_alm(P, 1, w.alm_d, w.bk, w.alm_a, s));
  CR_CHECK(operator_core(P, 1, w.alm_d, w.alm_a, fid->ninv, w.cg_bin, s, false, false));
  CR_TRY(launch_bin_grad(P, nbins, w.bin_edges, w.alm_c, w.alm_d, w.cg_bin, nullptr, w.bin_grad, s, 1));
  CR_TRY(hipMemcpyAsync(grad, w.bin_grad, (size_t)nbins * sizeof(double), hipMemcpyDeviceToHost, s));
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

}  // namespace

extern "C" int cr_lnpi_grad_fixed(const crsht_plan* P, const cr_problem* fid, const double* d, int nbins,
                                  const int* edges, const double* theta0, const double* theta, const double* f0,
                                  const double* a0, const cr_opts* opts, double* lnpi, double* grad, double* ahat,
                                  cr_stats* stats, void* stream) {
  CR_CHECK(check_plan(P, 1));
  if (fid && fid->amp) return CR_EINVAL;   // one spectrum per call
  if (P->ncomp != 1) return CR_ENOTSUP;
  if (!fid || !d || !theta0 || !theta || !f0 || !opts || !lnpi || !grad || !stats) return CR_EINVAL;
  if (!valid_bins(P, nbins, edges)) return CR_EINVAL;
  hipStream_t s = S(stream);
  CR_TRY(hipMemcpyAsync(P->w.bin_edges, edges, (size_t)(nbins + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  CR_CHECK(lnpi_grad_u(P, fid, d, nbins, edges, theta0, theta, f0, a0, opts, lnpi, grad, stats, s));
  if (ahat)
    CR_TRY(hipMemcpyAsync(ahat, P->w.alm_c, (size_t)P->g.nalm * sizeof(double2), hipMemcpyDeviceToDevice, s));
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

extern "C" int hmc_cl_step(const crsht_plan* P, const cr_problem* fid, const double* d, cr_bin_chain* st,
                           const cr_hmc_draws* dr, const cr_opts* opts, cr_hmc_out* out, void* stream) {
  CR_CHECK(check_plan(P, 1));
  if (fid && fid->amp) return CR_EINVAL;   // one spectrum per call
  if (P->ncomp != 1) return CR_ENOTSUP;
  if (!fid || !d || !st || !dr || !opts || !out || !st->theta || !st->ahat || !st->fhat || !dr->p0)
    return CR_EINVAL;
  if (!valid_bins(P, st->nbins, st->edges)) return CR_EINVAL;
  if (!(dr->eps > 0.0) || !std::isfinite(dr->eps) || dr->nleap < 1 || !(dr->u > 0.0 && dr->u < 1.0))
    return CR_EINVAL;
  if (!dr->w0 && !dr->w1) return CR_EINVAL;   // the fluctuation drawn after the move needs a random term
  const int nb = st->nbins;
  hipStream_t s = S(stream);
  Workspace const& w = P->w;
  std::memset(out, 0, sizeof(*out));
  CR_TRY(hipMemcpyAsync(w.bin_edges, st->edges, (size_t)(nb + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  // the mean-field right-hand side, the same at every point of the trajectory
  CR_CHECK(set_problem(P, fid, 1.0, s));
  CR_CHECK(assemble_rhs(P, 1, fid->ninv, d, nullptr, nullptr, w.cg_xacc, s));
  // potential U = -ln pi - sum theta (uniform prior in the amplitudes exp(theta_k)), dU = -grad - 1
  std::vector<double> th0(st->theta, st->theta + nb), th(th0), p(dr->p0, dr->p0 + nb), g(nb);
  double lp = 0.0;
  cr_stats cs;
  auto eval = [&](const double* a0) -> int {
    CR_CHECK(lnpi_grad_u(P, fid, d, nb, st->edges, th0.data(), th.data(), st->fhat, a0, opts, &lp, g.data(), &cs, s,
                         reinterpret_cast<const double*>(w.cg_xacc)));
    out->iters += cs.iters;
    out->solves += 1;
    if (cs.status != CR_OK) out->status = cs.status;
    return CR_OK;
  };
  auto U = [&]() {
    double u = -lp;
    for (int k = 0; k < nb; ++k) u -= th[k];
    return u;
  };
  auto kin = [&]() {
    double k2 = 0.0;
    for (int k = 0; k < nb; ++k) k2 += 0.5 * p[k] * p[k];
    return k2;
  };
  CR_CHECK(eval(st->ahat));
  const double H0 = U() + kin();
  // leapfrog: half step in p, nleap steps in theta, full steps in p between, half step at the end
  for (int k = 0; k < nb; ++k) p[k] += 0.5 * dr->eps * (g[k] + 1.0);
  for (int i = 0; i < dr->nleap; ++i) {
    for (int k = 0; k < nb; ++k) th[k] += dr->eps * p[k];
    CR_CHECK(eval(reinterpret_cast<const double*>(w.alm_c)));
    const double c = (i + 1 < dr->nleap) ? 1.0 : 0.5;
    for (int k = 0; k < nb; ++k) p[k] += c * dr->eps * (g[k] + 1.0);
  }
  const double H1 = U() + kin();
  out->dH = H1 - H0;
  out->lnpi_new = lp;
  out->accepted = (std::isfinite(out->dH) && std::log(dr->u) < -out->dH) ? 1 : 0;
  // then a fresh fluctuation at the amplitudes the move ends on (accepted or
  // not: a draw of the fluctuation given the amplitudes leaves the joint
  // target invariant on its own), and ln pi of the new state
  const std::vector<double>& te = out->accepted ? th : th0;
  std::vector<double> fac, cl(P->g.lmax + 1);
  bin_factor(P->g.lmax, nb, st->edges, te.data(), 1.0, fac);
  for (int l = 0; l <= P->g.lmax; ++l) cl[l] = fid->cl[l] * fac[l];
  cr_problem pr = *fid;
  pr.cl = cl.data();
  CR_CHECK(solve_core(P, &pr, 1.0, 1, nullptr, dr->w0, dr->w1, nullptr, st->fhat, opts, &out->fluct_stats, s));
  const int64_t na = P->g.nalm;
  if (out->accepted)
    CR_TRY(hipMemcpyAsync(st->ahat, w.alm_c, na * sizeof(double2), hipMemcpyDeviceToDevice, s));
  double t[3];
  CR_CHECK(lnpi_terms(P, fid->ninv, d, C2(st->ahat), C2(st->fhat), t, s));
  for (int k = 0; k < nb; ++k) st->theta[k] = te[k];
  st->lnpi = -0.5 * (t[0] + t[1] + t[2]);
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

extern "C" int gibbs_bins_step(const crsht_plan* P, const cr_problem* fid, const double* d, cr_bin_chain* st,
                               const double* g, const double* w0, const double* w1, const cr_opts* opts, double* t,
                               cr_stats* stats, void* stream) {
  CR_CHECK(check_plan(P, 1));
  if (fid && fid->amp) return CR_EINVAL;   // one spectrum per call
  if (P->ncomp != 1) return CR_ENOTSUP;
  if (!fid || !d || !st || !g || !opts || !stats || !st->theta || !st->ahat || !st->fhat || (!w0 && !w1))
    return CR_EINVAL;
  if (!valid_bins(P, st->nbins, st->edges) || st->edges[0] < fid->lmin) return CR_EINVAL;
  const int nb = st->nbins;
  for (int k = 0; k < nb; ++k)
    if (!(g[k] > 0.0) || !std::isfinite(g[k])) return CR_EINVAL;
  hipStream_t s = S(stream);
  Workspace const& w = P->w;
  const int64_t na = P->g.nalm;
  std::memset(stats, 0, 2 * sizeof(cr_stats));
  // 1) per-bin t_b = s^T S_fid^-1 s over the bin, s = ahat + fhat
  CR_CHECK(set_problem(P, fid, 1.0, s));
  CR_TRY(launch_alm_axpby(na, 1.0, C2(st->ahat), 1.0, C2(st->fhat), w.alm_d, s));
  CR_TRY(hipMemcpyAsync(w.bin_edges, st->edges, (size_t)(nb + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  CR_TRY(launch_bin_grad(P, nb, w.bin_edges, w.alm_d, w.alm_d, w.alm_d, nullptr, w.bin_grad, s, 2));
  std::vector<double> tb(nb), th(nb);
  CR_TRY(hipMemcpyAsync(tb.data(), w.bin_grad, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, s));
  CR_TRY(hipStreamSynchronize(s));
  // 2) A_b | s inverse gamma (shape k_b/2 - 1, scale t_b/2): A_b = (t_b/2) / g_b
  for (int k = 0; k < nb; ++k) {
    if (!(tb[k] > 0.0) || !std::isfinite(tb[k])) return CR_EINVAL;
    th[k] = std::log(0.5 * tb[k] / g[k]);
    if (t) t[k] = tb[k];
  }
  // 3) s | A: mean field (warm-started) and a fresh fluctuation at the new spectrum
  std::vector<double> fac, cl(P->g.lmax + 1);
  bin_factor(P->g.lmax, nb, st->edges, th.data(), 1.0, fac);
  for (int l = 0; l <= P->g.lmax; ++l) cl[l] = fid->cl[l] * fac[l];
  cr_problem pr = *fid;
  pr.cl = cl.data();
  CR_CHECK(solve_core(P, &pr, 1.0, 1, d, nullptr, nullptr, nullptr, reinterpret_cast<double*>(w.alm_c), opts,
                      &stats[0], s, st->ahat));
  CR_CHECK(solve_core(P, &pr, 1.0, 1, nullptr, w0, w1, nullptr, st->fhat, opts, &stats[1], s));
  CR_TRY(hipMemcpyAsync(st->ahat, w.alm_c, (size_t)na * sizeof(double2), hipMemcpyDeviceToDevice, s));
  double tt[3];
  CR_CHECK(lnpi_terms(P, fid->ninv, d, w.alm_c, C2(st->fhat), tt, s));
  for (int k = 0; k < nb; ++k) st->theta[k] = th[k];
  st->lnpi = -0.5 * (tt[0] + tt[1] + tt[2]);
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

extern "C" int gibbs_cl_step(const crsht_plan* P, const cr_problem* fid, const double* d, cr_chain* state, double g,
                             const double* w0, const double* w1, const cr_opts* opts, cr_gibbs_out* out,
                             void* stream) {
  CR_CHECK(check_plan(P, 1));
  if (fid && fid->amp) return CR_EINVAL;   // one spectrum per call
  if (P->ncomp != 1) return CR_ENOTSUP;
  if (!fid || !d || !state || !opts || !out || !state->ahat || !state->fhat || (!w0 && !w1)) return CR_EINVAL;
  if (!(g > 0.0) || !std::isfinite(g) || !(state->q > 0.0)) return CR_EINVAL;
  hipStream_t s = S(stream);
  std::memset(out, 0, sizeof(*out));
  const int64_t na = P->g.nalm;
  // 1) the current sky s = ahat + fhat and t = s^T S_fid^-1 s
  CR_TRY(launch_alm_axpby(na, 1.0, C2(state->ahat), 1.0, C2(state->fhat), P->w.alm_d, s));
  CR_CHECK(set_problem(P, fid, 1.0, s));
  double t = 0.0;
  CR_CHECK(quad_sinv(P, P->w.alm_d, &t, s));
  if (!(t > 0.0) || !std::isfinite(t)) return CR_EINVAL;
  // 2) q | s: inverse gamma (shape k/2 - 1, scale t/2), q' = (t/2) / g
  const double qn = 0.5 * t / g;
  out->t = t;
  out->q_new = qn;
  // 3) s | q': mean field (warm-started from the one at q) and a fresh fluctuation
  CR_CHECK(solve_core(P, fid, qn, 1, d, nullptr, nullptr, nullptr, reinterpret_cast<double*>(P->w.alm_c), opts,
                      &out->mean_stats, s, state->ahat));
  CR_CHECK(solve_core(P, fid, qn, 1, nullptr, w0, w1, nullptr, state->fhat, opts, &out->fluct_stats, s));
  CR_TRY(hipMemcpyAsync(state->ahat, P->w.alm_c, na * sizeof(double2), hipMemcpyDeviceToDevice, s));
  double tt[3];
  CR_CHECK(lnpi_terms(P, fid->ninv, d, P->w.alm_c, C2(state->fhat), tt, s));
  state->q = qn;
  state->lnpi = -0.5 * (tt[0] + tt[1] + tt[2]);
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

extern "C" int gibbs_cl_step_batch(const crsht_plan* P, const cr_problem* fid, const double* d, int n, cr_chain* st,
                                   const double* g, const double* w0, const double* w1, const cr_opts* opts,
                                   cr_gibbs_out* out, void* stream) {
  if (n < 1) return CR_EINVAL;
  CR_CHECK(check_plan(P, 2 * n));
  if (P->ncomp != 1) return CR_ENOTSUP;
  if (!fid || !d || !st || !g || !opts || !out || (!w0 && !w1)) return CR_EINVAL;
  if (fid->amp) return CR_EINVAL;   // the move sets the columns' amplitudes itself
  for (int c = 0; c < n; ++c) {
    if (!st[c].ahat || !st[c].fhat || !(st[c].q > 0.0) || !std::isfinite(st[c].q)) return CR_EINVAL;
    if (!(g[c] > 0.0) || !std::isfinite(g[c])) return CR_EINVAL;
  }
  hipStream_t s = S(stream);
  Workspace const& w = P->w;
  const int64_t na = P->g.nalm;
  const size_t cb = (size_t)na * sizeof(double2);
  std::memset(out, 0, (size_t)n * sizeof(cr_gibbs_out));
  // 1) q_c | s_c: t_c = s_c^T S_fid^-1 s_c of the current sky, q'_c = (t_c / 2) / g_c
  CR_CHECK(set_problem(P, fid, 1.0, s));
  std::vector<double> qn(2 * (size_t)n);
  for (int c = 0; c < n; ++c) {
    CR_TRY(launch_alm_axpby(na, 1.0, C2(st[c].ahat), 1.0, C2(st[c].fhat), w.alm_d, s));
    double t = 0.0;
    CR_CHECK(quad_sinv(P, w.alm_d, &t, s));
    if (!(t > 0.0) || !std::isfinite(t)) return CR_EINVAL;
    out[c].t = t;
    out[c].q_new = qn[c] = qn[n + c] = 0.5 * t / g[c];
  }
  // 2) s_c | q'_c: columns 0..n-1 the mean fields (the data term, one column
  //    copied; warm-started from the chains' mean fields), columns n..2n-1 the
  //    fluctuations from w0, w1 (cold), all at their chain's amplitude
  cr_problem pa = *fid;
  pa.amp = qn.data();
  CR_CHECK(assemble_rhs(P, 1, fid->ninv, d, nullptr, nullptr, w.cg_bin, s));
  for (int c = 1; c < n; ++c)
    CR_TRY(hipMemcpyAsync(w.cg_bin + (size_t)c * na, w.cg_bin, cb, hipMemcpyDeviceToDevice, s));
  CR_CHECK(set_problem(P, &pa, 1.0, s, n));   // columns 0..n-1 at q'_c for the S^-1/2 w0 term
  CR_CHECK(assemble_rhs(P, n, fid->ninv, nullptr, w0, w1, w.cg_bin + (size_t)n * na, s));
  for (int c = 0; c < n; ++c)
    CR_TRY(hipMemcpyAsync(w.cg_xacc + (size_t)c * na, st[c].ahat, cb, hipMemcpyDeviceToDevice, s));
  CR_TRY(hipMemsetAsync(w.cg_xacc + (size_t)n * na, 0, (size_t)n * cb, s));
  std::vector<cr_stats> ss(2 * (size_t)n);
  CR_CHECK(solve_core(P, &pa, 1.0, 2 * n, nullptr, nullptr, nullptr, reinterpret_cast<const double*>(w.cg_bin),
                      reinterpret_cast<double*>(w.cg_xacc), opts, ss.data(), s,
                      reinterpret_cast<const double*>(w.cg_xacc)));
  // 3) new states and ln pi of each (one batch)
  std::vector<double> t(3 * (size_t)n);
  CR_CHECK(lnpi_terms_batch(P, n, fid->ninv, d, w.cg_xacc, w.cg_xacc + (size_t)n * na, t.data(), s));
  for (int c = 0; c < n; ++c) {
    out[c].mean_stats = ss[c];
    out[c].fluct_stats = ss[n + c];
    CR_TRY(hipMemcpyAsync(st[c].ahat, w.cg_xacc + (size_t)c * na, cb, hipMemcpyDeviceToDevice, s));
    CR_TRY(hipMemcpyAsync(st[c].fhat, w.cg_xacc + (size_t)(n + c) * na, cb, hipMemcpyDeviceToDevice, s));
    st[c].q = qn[c];
    st[c].lnpi = -0.5 * (t[3 * c] + t[3 * c + 1] / qn[c] + t[3 * c + 2]);
  }
  CR_TRY(hipStreamSynchronize(s));
  return CR_OK;
}

// ================================================================ autotuner
namespace {

void fill_tuning(const crsht_plan* P, crsht_tuning* o) {
  std::memset(o, 0, sizeof(*o));
  o->nclasses = (int)std::min<size_t>(P->ring_cls.size(), kMaxRingClasses);
  for (int k = 0; k < 8; ++k) {
    o->fft_len[k] = k < o->nclasses ? P->ring_cls[k].L : 0;
    o->ring_div[k] = k < o->nclasses ? (k < kMaxRingClasses ? P->tune.ring_div[k] : 8) : 0;
  }
  o->f64_synth_cols = P->tune.f64_synth_cols;
  o->f64_adj_cols = P->tune.f64_adj_cols;
}

bool valid_cols(int c) { return c == 2 || c == 4 || c == 8; }

int apply_tuning(crsht_plan* P, const crsht_tuning* in) {
  if (!valid_cols(in->f64_synth_cols) || !valid_cols(in->f64_adj_cols)) return CR_EINVAL;
  Tuning t;
  const int nc = (int)std::min<size_t>(P->ring_cls.size(), kMaxRingClasses);
  for (int k = 0; k < nc; ++k) {
    const int d = in->ring_div[k];
    if (d != 8 && d != 4) return CR_EINVAL;
    if (d == 4 && P->ring_cls[k].L < 1024) return CR_EINVAL;
    t.ring_div[k] = d;
  }
  t.f64_synth_cols = in->f64_synth_cols;
  t.f64_adj_cols = in->f64_adj_cols;
  // captured graphs hold the launch shapes: drop them (after any replays)
  CR_TRY(hipDeviceSynchronize());
  if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
  P->graph_exec = nullptr;
  P->graph_key = GraphKey();
  for (auto& gx : P->dgraph) {
    if (gx) (void)hipGraphExecDestroy(gx);
    gx = nullptr;
  }
  P->dgraph_key = GraphKey();
  P->tune = t;
  return CR_OK;
}

// mean milliseconds of `reps` runs of f on s (after one untimed run)
template <class F>
int time_ms(hipStream_t s, int reps, F f, double* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  CR_TRY(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return CR_EDEVICE;
  }
  int rc = f();
  if (rc == CR_OK && hipEventRecord(a, s) != hipSuccess) rc = CR_EDEVICE;
  for (int r = 0; r < reps && rc == CR_OK; ++r) rc = f();
  if (rc == CR_OK && hipEventRecord(b, s) != hipSuccess) rc = CR_EDEVICE;
  float t = 0.f;
  if (rc == CR_OK && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&t, a, b) != hipSuccess))
    rc = CR_EDEVICE;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = (double)t / reps;
  return rc;
}

std::string tune_key(const crsht_plan* P, int nrhs, cr_prec prec) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ') c = '_';
  char buf[256];
  std::snprintf(buf, sizeof(buf), "crsht-tune-1 %s %d %d %d %d %d %d", arch.c_str(), P->g.nside, P->g.lmax,
                P->g.mmax, P->ncomp, nrhs, (int)prec);
  return buf;
}

bool cache_lookup(const char* path, const std::string& key, crsht_tuning* t) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    const size_t kl = key.size();
    if (std::strncmp(line, key.c_str(), kl) != 0 || line[kl] != ' ') continue;
    crsht_tuning c = *t;
    int* d = c.ring_div;
    if (std::sscanf(line + kl, " %d %d %d %d %d %d %d %d %d %d", &d[0], &d[1], &d[2], &d[3], &d[4], &d[5], &d[6],
                    &d[7], &c.f64_synth_cols, &c.f64_adj_cols) == 10) {
      *t = c;   // the last matching line wins
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const crsht_tuning& t) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  const int* d = t.ring_div;
  std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d\n", key.c_str(), d[0], d[1], d[2], d[3], d[4], d[5], d[6], d[7],
               t.f64_synth_cols, t.f64_adj_cols);
  std::fclose(f);
}

}  // namespace

extern "C" int crsht_get_tuning(const crsht_plan* P, crsht_tuning* out) {
  if (!P || !out) return CR_EINVAL;
  fill_tuning(P, out);
  return CR_OK;
}

extern "C" int crsht_set_tuning(crsht_plan* P, const crsht_tuning* in) {
  if (!P || !in) return CR_EINVAL;
  return apply_tuning(P, in);
}

// Measures the candidate shapes on the plan's workspace: the fused ring pass
// (N^-1 between the transforms, the form inside PCG) in the given precision,
// one class at a time (coordinate search), and the FP64 matrix-core Legendre
// synthesis and adjoint for every columns-per-launch choice.
extern "C" int crsht_autotune(crsht_plan* P, int nrhs, cr_prec prec, crsht_tuning* out, void* stream) {
  CR_CHECK(check_plan(P, nrhs));
  if (!out) return CR_EINVAL;
  if (prec != CR_F64 && prec != CR_MIXED) return CR_EINVAL;
  if (P->timing.on) return CR_EINVAL;
  hipStream_t s = S(stream);
  const bool f32 = prec == CR_MIXED;
  const std::string key = tune_key(P, nrhs, prec);
  const char* path = std::getenv("CRSHT_TUNE_CACHE");
  crsht_tuning t;
  fill_tuning(P, &t);
  if (path && *path && cache_lookup(path, key, &t)) {
    CR_CHECK(apply_tuning(P, &t));
    fill_tuning(P, out);
    out->from_cache = 1;
    return CR_OK;
  }
  // default shapes as the starting point; the inputs are the workspace's
  // contents after zero fills (the timings do not depend on the values)
  crsht_tuning cur;
  fill_tuning(P, &cur);
  for (int k = 0; k < cur.nclasses; ++k) cur.ring_div[k] = 8;
  cur.f64_synth_cols = cur.f64_adj_cols = 8;
  CR_CHECK(apply_tuning(P, &cur));
  Workspace const& w = P->w;
  const int ncomp = P->ncomp;
  const int cs = ncomp == 3 ? 9 * nrhs : nrhs, ca = ncomp == 3 ? 7 * nrhs : nrhs;   // Legendre columns
  const size_t eo_bytes = (size_t)cs * P->g.npairs * (P->g.mmax + 1) * 2 * sizeof(double2);
  const size_t geo_bytes = (size_t)ca * P->g.npairs * (P->g.mmax + 1) * 2 * sizeof(double2);
  CR_TRY(hipMemsetAsync(w.eo, 0, eo_bytes, s));
  CR_TRY(hipMemsetAsync(w.geo, 0, geo_bytes, s));
  CR_TRY(hipMemsetAsync(w.alm_a, 0, (size_t)cs * P->g.nalm * sizeof(double2), s));
  CR_TRY(hipMemsetAsync(w.map_a, 0, (size_t)ncomp * P->g.npix * sizeof(double), s));
  const double* ninv = w.map_a;
  auto ring = [&]() -> int {
    if (ncomp == 3)
      CR_TRY(launch_ring(P, 3 * nrhs, RING_FUSED, w.eo, nullptr, ninv, w.geo, f32, s, tqu_cols(P)));
    else
      CR_TRY(launch_ring(P, nrhs, RING_FUSED, w.eo, nullptr, ninv, w.geo, f32, s));
    return CR_OK;
  };
  auto syn = [&]() -> int {
    CR_TRY(launch_legendre_synth(P, cs, w.alm_a, w.eo, s));
    return CR_OK;
  };
  auto adj = [&]() -> int {
    CR_TRY(launch_legendre_adjoint(P, ca, w.geo, w.alm_b, false, s));
    return CR_OK;
  };
  const int reps = 3;
  double t_ring = 0, t_syn = 0, t_adj = 0;
  CR_CHECK(time_ms(s, reps, ring, &t_ring));
  if (cs >= 2) CR_CHECK(time_ms(s, reps, syn, &t_syn));
  if (ca >= 2) CR_CHECK(time_ms(s, reps, adj, &t_adj));
  const double t_default = t_ring + t_syn + t_adj;
  for (int k = 0; k < cur.nclasses; ++k) {
    if (P->ring_cls[k].L < 1024) continue;
    crsht_tuning c = cur;
    c.ring_div[k] = 4;
    CR_CHECK(apply_tuning(P, &c));
    double tt = 0;
    CR_CHECK(time_ms(s, reps, ring, &tt));
    if (tt < 0.97 * t_ring) {
      cur = c;
      t_ring = tt;
    }
  }
  const int cands[3] = {4, 2, 8};
  if (cs >= 2) {
    for (int v : cands) {
      if (v == cur.f64_synth_cols || v > cs) continue;
      crsht_tuning c = cur;
      c.f64_synth_cols = v;
      CR_CHECK(apply_tuning(P, &c));
      double tt = 0;
      CR_CHECK(time_ms(s, reps, syn, &tt));
      if (tt < 0.97 * t_syn) {
        cur = c;
        t_syn = tt;
      }
    }
  }
  if (ca >= 2) {
    for (int v : cands) {
      if (v == cur.f64_adj_cols || v > ca) continue;
      crsht_tuning c = cur;
      c.f64_adj_cols = v;
      CR_CHECK(apply_tuning(P, &c));
      double tt = 0;
      CR_CHECK(time_ms(s, reps, adj, &tt));
      if (tt < 0.97 * t_adj) {
        cur = c;
        t_adj = tt;
      }
    }
  }
  CR_CHECK(apply_tuning(P, &cur));
  if (path && *path) cache_store(path, key, cur);
  fill_tuning(P, out);
  out->from_cache = 0;
  out->ms_default = t_default;
  out->ms_tuned = t_ring + t_syn + t_adj;
  return CR_OK;
}
