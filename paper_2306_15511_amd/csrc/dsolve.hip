// Control of the device-driven (stream-ordered) solve: the decisions that
// the host loop of the refined PCG takes from the scalars it reads back --
// when to replace the recursive residual by the FP64 true residual, when to
// restart a column's direction, when a column or the whole solve has stopped
// -- taken by one small kernel between the enqueued sections instead, so that
// a whole solve is enqueued at once and nothing waits on the host. The
// sections are predicated by words of the control block (CtlSlot): their
// kernels return at once while the word is set.
#include <cmath>

#include "internal.h"

namespace crsht {
namespace {

constexpr int kCtlThreads = 256;

// stats in the layout of the public cr_stats
struct StatsOut {
  int status, iters, refinements;
  double rel_resid_true;
};

__device__ __forceinline__ bool block_any(bool v) { return __syncthreads_or(v ? 1 : 0) != 0; }

__global__ __launch_bounds__(kCtlThreads) void k_dctl(int mode, DctlArgs a, double* __restrict__ scal,
                                                     int* __restrict__ ctl, StatsOut* __restrict__ stats,
                                                     int* __restrict__ host_exited) {
  const int t = threadIdx.x;
  if (mode == DC_INIT) {
    if (t < kCtlSlots) ctl[t] = 0;
    for (int c = t; c < a.nrhs; c += kCtlThreads) {
      double* sc = scal + c * kScalSlots;
      sc[S_LAST] = 1.0;
      sc[S_TRUE] = 1.0;
      sc[S_REFINE] = 0.0;
      sc[S_TRIG] = 0.0;
      sc[S_RESTART] = 0.0;
    }
    return;
  }
  if (mode == DC_CHECK) {
    // a replacement is due when a column (not broken, not yet confirmed)
    // claims convergence or its recursive residual has fallen by itol since
    // its last replacement; only after the first block and within max_refine
    // An intermediate replacement -- no open column claims convergence and
    // every open column's recursive residual is at least kLowReplaceFloor --
    // uses the bf16x6 operator (mixed form only); the others FP64.
    const bool exited = ctl[C_EXITED] != 0;
    bool need = false, high = false;
    for (int c = t; c < a.nrhs; c += kCtlThreads) {
      double* sc = scal + c * kScalSlots;
      bool trig = false;
      if (!exited && sc[S_BREAK] == 0.0 && sc[S_TRUE] > a.tol) {
        trig = sc[S_DONE] != 0.0 || sc[S_REL] <= a.itol * sc[S_LAST];
        high |= sc[S_DONE] != 0.0 || sc[S_REL] < kLowReplaceFloor;
      }
      sc[S_TRIG] = trig ? 1.0 : 0.0;
      need |= trig;
    }
    need = block_any(need);
    high = block_any(high);
    if (t == 0) {
      const bool go = !exited && need && ctl[C_PENDING] != 0 && ctl[C_NREP] < a.maxref;
      const bool low = go && !high && a.f64 == 0;
      ctl[C_SKIP_REPL] = (go && !low) ? 0 : 1;
      ctl[C_SKIP_REPL_LOW] = low ? 0 : 1;
      ctl[C_LOW] = low ? 1 : 0;
      ctl[C_SKIP_TAIL] = go ? 0 : 1;
    }
    return;
  }
  if (mode == DC_AFTER_REPL) {
    if (ctl[C_SKIP_REPL] != 0 && ctl[C_SKIP_REPL_LOW] != 0) return;
    const bool low = ctl[C_LOW] != 0;   // a bf16x6 residual decides no convergence
    // the true residuals (k_sum_rows: AUX0 = ||b - Ax||^2, AUX1 = ||b||^2);
    // keep the direction only when the replacement corrects the recursive
    // residual by a small amount, restart it when the true residual did not
    // fall since the last replacement or is far above the recursive one
    const int it = ctl[C_IT];
    bool cont = false;
    for (int c = t; c < a.nrhs; c += kCtlThreads) {
      double* sc = scal + c * kScalSlots;
      const double rel = sc[S_AUX1] > 0.0 ? sqrt(sc[S_AUX0] / sc[S_AUX1]) : 0.0;
      sc[S_TRUE] = rel;
      if (sc[S_BREAK] != 0.0) continue;
      const double rec = sc[S_REL];
      sc[S_RESTART] = (sc[S_TRIG] != 0.0 && (rel >= sc[S_LAST] || rel > 4.0 * rec)) ? 1.0 : 0.0;
      sc[S_LAST] = rel;
      sc[S_REFINE] += 1.0;
      if (rel <= a.tol && !low) {
        sc[S_DONE] = 1.0;
      } else if (it < a.maxiter) {
        sc[S_DONE] = 0.0;
        cont = true;
      } else {
        sc[S_DONE] = 1.0;
      }
    }
    cont = block_any(cont);
    if (t == 0) {
      ctl[C_NREP] += 1;
      ctl[C_FRESH] = low ? 0 : 1;
      if (!cont) {
        ctl[C_EXITED] = 1;
        ctl[C_SKIP_TAIL] = 1;
      }
    }
    return;
  }
  if (mode == DC_PRE_BLOCK) {
    bool open = false;
    for (int c = t; c < a.nrhs; c += kCtlThreads) open |= scal[c * kScalSlots + S_DONE] == 0.0;
    open = block_any(open);
    if (t == 0) {
      if (ctl[C_EXITED] == 0 && (!open || ctl[C_IT] >= a.maxiter)) ctl[C_EXITED] = 1;
      ctl[C_SKIP_ITER] = ctl[C_EXITED];
      if (host_exited) *reinterpret_cast<volatile int*>(host_exited) = ctl[C_EXITED];
    }
    return;
  }
  if (mode == DC_AFTER_BLOCK) {
    if (t == 0 && ctl[C_SKIP_ITER] == 0) {
      ctl[C_IT] += a.every;
      ctl[C_PENDING] = 1;
      ctl[C_FRESH] = 0;
    }
    return;
  }
  if (mode == DC_FINAL_PRE) {
    if (t == 0) ctl[C_SKIP_FINAL] = ctl[C_FRESH];
    return;
  }
  // DC_FINAL_POST: the statistics of every column
  const bool fresh_resid = ctl[C_SKIP_FINAL] == 0;
  for (int c = t; c < a.nrhs; c += kCtlThreads) {
    double* sc = scal + c * kScalSlots;
    if (fresh_resid) sc[S_TRUE] = sc[S_AUX1] > 0.0 ? sqrt(sc[S_AUX0] / sc[S_AUX1]) : 0.0;
    const double rel = sc[S_TRUE];
    StatsOut o;
    o.iters = (int)sc[S_ITERS];
    o.refinements = a.f64 ? 0 : (int)sc[S_REFINE];
    o.rel_resid_true = rel;
    if (sc[S_BREAK] != 0.0 || !isfinite(rel))
      o.status = CR_BREAKDOWN;
    else if (rel > a.tol)
      o.status = CR_NOCONV;
    else
      o.status = CR_OK;
    if (stats) stats[c] = o;
  }
  if (t == 0 && host_exited) *reinterpret_cast<volatile int*>(host_exited) = 1;
}

}  // namespace

hipError_t launch_dctl(const crsht_plan* P, int mode, const DctlArgs& a, void* stats_dev, hipStream_t s) {
  static_assert(sizeof(StatsOut) == sizeof(cr_stats), "device stats layout");
  hipLaunchKernelGGL(k_dctl, dim3(1), dim3(kCtlThreads), 0, s, mode, a, P->w.scal, P->w.ctl,
                     reinterpret_cast<StatsOut*>(stats_dev), P->w.host_exited);
  return hipGetLastError();
}

}  // namespace crsht
