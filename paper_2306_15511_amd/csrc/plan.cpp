// Plan creation: HEALPix ring table, Legendre recurrence tables, per-ring FFT
// tables and the workspace. Host code; all tables end up in device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using crsht::Geometry;

namespace {

typedef long double ld;
typedef std::complex<ld> cld;

const ld kPi = 3.141592653589793238462643383279502884L;

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
int next_pow2(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// In-place iterative radix-2 FFT (forward: exp(-2 pi i jk / n)), long double,
// for setup tables only.
void host_fft(std::vector<cld>& a) {
  const int n = (int)a.size();
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    for (int k = 0; k < len / 2; ++k) {
      const ld ang = -2.0L * kPi * (ld)k / (ld)len;
      const cld w(cosl(ang), sinl(ang));
      for (int i = 0; i < n; i += len) {
        cld u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
    }
  }
}

template <typename T>
int dalloc(T** p, size_t count, size_t* total) {
  *p = nullptr;
  if (count == 0) count = 1;
  const size_t bytes = count * sizeof(T);
  if (hipMalloc((void**)p, bytes) != hipSuccess) {
    *p = nullptr;
    return CR_ENOMEM;
  }
  *total += bytes;
  return CR_OK;
}

template <typename T>
int upload(T** p, const std::vector<T>& h, size_t* total) {
  int rc = dalloc(p, h.size(), total);
  if (rc) return rc;
  if (hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return CR_EDEVICE;
  return CR_OK;
}

void free_plan_memory(crsht_plan* P) {
  void* ptrs[] = {P->t.pair_z, P->t.pair_nphi, P->t.pair_phi0, P->t.pair_first_n, P->t.pair_first_s,
                  P->t.pair_fft_len, P->t.pair_bs_off, P->t.pair_bk_off, P->t.bs_chirp, P->t.bs_kern,
                  P->t.twiddle, P->t.bs_chirp32, P->t.bs_kern32, P->t.twiddle32, P->t.ring_pairs, P->t.rec_alpha, P->t.rec_kappa, P->t.lmm_v, P->t.lmm_k, P->t.lst_g, P->t.pair_mtop, P->t.lst_s, P->t.mstart, P->t.ones,
                  P->t.mx_cstart, P->t.mx_tstart, P->t.mx_tile_m, P->t.mx_order, P->t.mx_ckpt, P->w.cg_xacc, P->w.cg_bin, P->w.bin_edges, P->w.bin_part, P->w.bin_grad, P->w.lfac, P->w.camp,
                  P->w.mx_ab, P->w.mx_ag, P->w.adj_part, P->w.pol,
                  P->t.idx_l, P->t.idx_m, P->w.eo, P->w.geo, P->w.alm_a, P->w.alm_b, P->w.cg_x, P->w.cg_r, P->t.idx_mv, P->w.bl_keep, P->w.sblk,
                  P->w.cg_z, P->w.cg_p, P->w.cg_q, P->w.cg_b, P->w.cg_d, P->w.alm_c, P->w.alm_d, P->w.map_a, P->w.ring_w,
                  P->w.diag, P->w.sinv, P->w.sinvhalf, P->w.bk, P->w.perl, P->w.partial, P->w.scal, P->w.ctl,
                  P->w.dstats};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (P->w.host_scal) (void)hipHostFree(P->w.host_scal);
  if (P->w.host_exited) (void)hipHostFree(P->w.host_exited);
  for (int k = 0; k < crsht_plan::kStageSlots; ++k) {
    if (P->stage_host[k]) (void)hipHostFree(P->stage_host[k]);
    if (P->stage_ev[k]) (void)hipEventDestroy(P->stage_ev[k]);
    P->stage_host[k] = nullptr;
    P->stage_ev[k] = nullptr;
  }
  for (auto& gx : P->dgraph) {
    if (gx) (void)hipGraphExecDestroy(gx);
    gx = nullptr;
  }
  crsht::block_pc_free(P->pc);
  if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
  for (int k = 0; k < crsht_plan::kAux; ++k) {
    if (P->aux_stream[k]) (void)hipStreamDestroy(P->aux_stream[k]);
    if (P->aux_join_ev[k]) (void)hipEventDestroy(P->aux_join_ev[k]);
    P->aux_stream[k] = nullptr;
    P->aux_join_ev[k] = nullptr;
  }
  if (P->aux_fork_ev) (void)hipEventDestroy(P->aux_fork_ev);
  P->aux_fork_ev = nullptr;
  if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
  if (P->exec_stream) (void)hipStreamDestroy(P->exec_stream);
  P->exec_stream = nullptr;
  hipEvent_t* evs[] = {&P->ev_fork, &P->ev_join, &P->ev_round[0], &P->ev_round[1], &P->ev_round[2]};
  for (hipEvent_t* e : evs) {
    if (*e) (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  P->graph_exec = nullptr;
  P->cap_stream = nullptr;
}

}  // namespace

static int build_plan(crsht_plan* P, int nside, int lmax, int mmax, int ncomp, int nrhs_max, size_t* total) {
  Geometry& g = P->g;
  g.nside = nside;
  g.lmax = lmax;
  g.mmax = mmax;
  g.nrings = 4 * nside - 1;
  g.npairs = 2 * nside;
  g.npix = 12LL * nside * nside;
  g.nalm = (int64_t)(mmax + 1) * (lmax + 1) - (int64_t)mmax * (mmax + 1) / 2;
  const int np = g.npairs;
  const int64_t ns = nside;

  // ---------------- ring pairs (Gorski et al. 2005, RING scheme)
  std::vector<double> pz(np), pphi0(np);
  std::vector<ld> psin(np);
  std::vector<int> pnphi(np), pfft(np);
  std::vector<int64_t> pfn(np), pfs(np), pbs(np, -1), pbk(np, -1);
  for (int p = 0; p < np; ++p) {
    const int64_t i = p + 1;  // ring number from the north pole
    ld z, s;
    int n;
    ld phi0;
    int64_t first;
    if (i < ns) {
      const ld omz = (ld)(i * i) / (ld)(3 * ns * ns);
      z = 1.0L - omz;
      s = sqrtl(omz * (2.0L - omz));
      n = (int)(4 * i);
      phi0 = kPi / (ld)(4 * i);
      first = 2 * i * (i - 1);
    } else {
      z = (ld)(4 * ns - 2 * i) / (ld)(3 * ns);
      s = sqrtl((1.0L - z) * (1.0L + z));
      n = (int)(4 * ns);
      phi0 = ((i + ns) % 2 == 1) ? 0.0L : kPi / (ld)(4 * ns);
      first = 2 * ns * (ns - 1) + 4 * ns * (i - ns);
    }
    pz[p] = (double)z;
    psin[p] = s;
    pnphi[p] = n;
    pphi0[p] = (double)phi0;
    pfn[p] = first;
    pfs[p] = g.npix - first - n;
    pfft[p] = is_pow2(n) ? n : next_pow2(2 * n - 1);
  }
  int fft_max = 2;
  for (int p = 0; p < np; ++p) fft_max = fft_max > pfft[p] ? fft_max : pfft[p];
  g.fft_max = fft_max;

  // host copies for pixel coordinates
  P->h_nphi.assign(g.nrings, 0);
  P->h_first.assign(g.nrings, 0);
  P->h_z.assign(g.nrings, 0.0);
  P->h_phi0.assign(g.nrings, 0.0);
  for (int p = 0; p < np; ++p) {
    const int rn = p, rs = g.nrings - 1 - p;
    P->h_nphi[rn] = P->h_nphi[rs] = pnphi[p];
    P->h_phi0[rn] = P->h_phi0[rs] = pphi0[p];
    P->h_first[rn] = pfn[p];
    P->h_first[rs] = pfs[p];
    P->h_z[rn] = pz[p];
    P->h_z[rs] = -pz[p];
  }

  // ---------------- Bluestein tables for rings whose length is not a power of two
  std::vector<double2> chirp, kern;
  for (int p = 0; p < np; ++p) {
    const int n = pnphi[p];
    if (is_pow2(n)) continue;
    const int L = pfft[p];
    pbs[p] = (int64_t)chirp.size();
    pbk[p] = (int64_t)kern.size();
    std::vector<cld> c(n), b(L, cld(0, 0));
    for (int j = 0; j < n; ++j) {
      const int64_t jj = ((int64_t)j * j) % (2 * (int64_t)n);
      const ld ang = -kPi * (ld)jj / (ld)n;
      c[j] = cld(cosl(ang), sinl(ang));
    }
    for (int j = 0; j < n; ++j) {
      b[j] = std::conj(c[j]);
      if (j > 0) b[L - j] = std::conj(c[j]);
    }
    host_fft(b);
    for (int j = 0; j < n; ++j) chirp.push_back(make_double2((double)c[j].real(), (double)c[j].imag()));
    for (int j = 0; j < L; ++j)
      kern.push_back(make_double2((double)(b[j].real() / (ld)L), (double)(b[j].imag() / (ld)L)));
  }
  std::vector<double2> tw(fft_max);
  for (int j = 0; j < fft_max; ++j) {
    const ld ang = -2.0L * kPi * (ld)j / (ld)fft_max;
    tw[j] = make_double2((double)cosl(ang), (double)sinl(ang));
  }

  // ---------------- Legendre recurrence tables
  std::vector<int64_t> mst(mmax + 2);
  for (int m = 0; m <= mmax + 1; ++m) mst[m] = (int64_t)m * (lmax + 1) - (int64_t)m * (m - 1) / 2;
  std::vector<double> alpha(g.nalm, 0.0), kappa(g.nalm, 0.0);
  std::vector<int> il(g.nalm), im(g.nalm);
  for (int m = 0; m <= mmax; ++m) {
    const int64_t o = mst[m];
    std::vector<ld> kap(lmax + 1 - m);
    for (int l = m; l <= lmax; ++l) {
      il[o + l - m] = l;
      im[o + l - m] = m;
      const ld L = l, M = m;
      if (l == m) {
        kap[0] = 1.0L;
      } else if (l == m + 1) {
        kap[1] = sqrtl(2.0L * M + 3.0L);
        alpha[o + 1] = 1.0;  // mu_{m+1} = 1 * z * mu_m - mu_{m-1}, with mu_{m-1} = 0
      } else {
        const ld a = sqrtl((4.0L * L * L - 1.0L) / (L * L - M * M));
        const ld b = sqrtl(((L - 1) * (L - 1) - M * M) / (4.0L * (L - 1) * (L - 1) - 1.0L));
        kap[l - m] = a * b * kap[l - m - 2];
        alpha[o + l - m] = (double)(kap[l - m - 1] / (b * kap[l - m - 2]));
      }
      kappa[o + l - m] = (double)kap[l - m];
    }
  }
  // start values lambda_mm(z_p) = v * 2^(600 k), by the product
  // lambda_mm = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1}, lambda_00 = 1/sqrt(4 pi)
  std::vector<double> lv((size_t)(mmax + 1) * np);
  std::vector<int> lk((size_t)(mmax + 1) * np);
  for (int p = 0; p < np; ++p) {
    ld mant = 1.0L / sqrtl(4.0L * kPi);
    long e2 = 0;
    const ld s = psin[p];
    for (int m = 0; m <= mmax; ++m) {
      if (m > 0) {
        mant *= -sqrtl((2.0L * m + 1.0L) / (2.0L * m)) * s;
        int ex;
        mant = frexpl(mant, &ex);
        e2 += ex;
      }
      // value = mant * 2^e2, |mant| in [0.5, 1)
      int k = 0;
      if (e2 < -100) {
        // k = floor((e2 + 100) / 600) <= -1, so that e2 - 600 k lies in [-100, 500)
        long t = e2 + 100;
        k = (int)((t - (crsht::kScaleBits - 1)) / crsht::kScaleBits);
      }
      lv[(size_t)m * np + p] = (double)ldexpl(mant, (int)(e2 - (long)crsht::kScaleBits * k));
      lk[(size_t)m * np + p] = k;
    }
  }

  // ---------------- upload
  int rc;
  if ((rc = upload(&P->t.pair_z, pz, total))) return rc;
  if ((rc = upload(&P->t.pair_nphi, pnphi, total))) return rc;
  if ((rc = upload(&P->t.pair_phi0, pphi0, total))) return rc;
  if ((rc = upload(&P->t.pair_first_n, pfn, total))) return rc;
  if ((rc = upload(&P->t.pair_first_s, pfs, total))) return rc;
  if ((rc = upload(&P->t.pair_fft_len, pfft, total))) return rc;
  if ((rc = upload(&P->t.pair_bs_off, pbs, total))) return rc;
  if ((rc = upload(&P->t.pair_bk_off, pbk, total))) return rc;
  if (chirp.empty()) chirp.push_back(make_double2(0, 0));
  if (kern.empty()) kern.push_back(make_double2(0, 0));
  if ((rc = upload(&P->t.bs_chirp, chirp, total))) return rc;
  if ((rc = upload(&P->t.bs_kern, kern, total))) return rc;
  if ((rc = upload(&P->t.twiddle, tw, total))) return rc;
  {
    auto to32 = [](const std::vector<double2>& v) {
      std::vector<float2> o(v.size());
      for (size_t i = 0; i < v.size(); ++i) o[i] = make_float2((float)v[i].x, (float)v[i].y);
      return o;
    };
    if ((rc = upload(&P->t.bs_chirp32, to32(chirp), total))) return rc;
    if ((rc = upload(&P->t.bs_kern32, to32(kern), total))) return rc;
    if ((rc = upload(&P->t.twiddle32, to32(tw), total))) return rc;
    std::vector<int> rp;
    crsht::ring_classes(pfft, P->ring_cls, rp);
    if ((rc = upload(&P->t.ring_pairs, rp, total))) return rc;
    if (crsht::ring_prepare(P) != hipSuccess) return CR_EDEVICE;
    if (crsht::legendre_prepare(P) != hipSuccess) return CR_EDEVICE;
  }
  alpha.resize(alpha.size() + 32, 0.0);   // readable past the last (l, m) by a whole chunk of 32 steps
  if ((rc = upload(&P->t.rec_alpha, alpha, total))) return rc;
  if ((rc = upload(&P->t.rec_kappa, kappa, total))) return rc;
  if ((rc = upload(&P->t.lmm_v, lv, total))) return rc;
  if ((rc = upload(&P->t.lmm_k, lk, total))) return rc;
  if ((rc = upload(&P->t.mstart, mst, total))) return rc;
  if ((rc = dalloc(&P->t.lst_g, (size_t)(mmax + 1) * np, total))) return rc;
  if ((rc = dalloc(&P->t.lst_s, (size_t)(mmax + 1) * np, total))) return rc;
  if (crsht::launch_legendre_start(P, nullptr) != hipSuccess) return CR_EDEVICE;
  if (hipDeviceSynchronize() != hipSuccess) return CR_EDEVICE;
  {
    // largest m at which each ring pair's recurrence becomes live by l = lmax
    std::vector<int> lg((size_t)(mmax + 1) * np);
    if (hipMemcpy(lg.data(), P->t.lst_g, lg.size() * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
      return CR_EDEVICE;
    std::vector<int> mtop(np, 0);
    for (int m = 0; m <= mmax; ++m)
      for (int p = 0; p < np; ++p)
        if (lg[(size_t)m * np + p] <= (lmax - m) / crsht::kStartGroup) mtop[p] = m;
    if ((rc = upload(&P->t.pair_mtop, mtop, total))) return rc;
    for (int p = 0; p < np; ++p) P->t.live_pair_m += mtop[p] + 1;
  }
  {
    std::vector<double> ones(g.nalm, 1.0);
    if ((rc = upload(&P->t.ones, ones, total))) return rc;
  }
  {
    std::vector<int64_t> cst, tst;
    std::vector<int> tm;
    std::vector<int> order;
    crsht::mixed_starts(g, cst, tst, tm, order, P->t.mx_maxq);
    if ((rc = upload(&P->t.mx_order, order, total))) return rc;
    P->t.mx_ntiles = (int64_t)tm.size();
    if ((rc = upload(&P->t.mx_cstart, cst, total))) return rc;
    if ((rc = upload(&P->t.mx_tstart, tst, total))) return rc;
    if ((rc = upload(&P->t.mx_tile_m, tm, total))) return rc;
    if ((rc = dalloc(&P->t.mx_ckpt, (size_t)P->t.mx_ntiles * np, total))) return rc;
    if (crsht::launch_checkpoints(P, nullptr) != hipSuccess) return CR_EDEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return CR_EDEVICE;
  }
  if ((rc = upload(&P->t.idx_l, il, total))) return rc;
  if ((rc = upload(&P->t.idx_m, im, total))) return rc;
  {
    std::vector<int> imv;
    for (int k = 0; k < ncomp; ++k) imv.insert(imv.end(), im.begin(), im.end());
    if ((rc = upload(&P->t.idx_mv, imv, total))) return rc;
  }

  // ---------------- workspace
  // A T+Q+U column expands to 9 scalar Legendre columns in the synthesis (T,
  // and T0..T3 of E and B) and 7 in the adjoint (T, Q, U and four weighted
  // copies of Q and U); solver vectors hold 3 blocks of nalm.
  const size_t R = (size_t)nrhs_max;
  const size_t C = (size_t)ncomp;
  const size_t ceo = ncomp == 3 ? 9 : 1, cgeo = ncomp == 3 ? 7 : 1;
  const size_t neo1 = (size_t)np * (size_t)(mmax + 1) * 2;
  const size_t na = R * (size_t)g.nalm;
  crsht::Workspace& w = P->w;
  w.npart = (mmax + 1) > 1024 ? (mmax + 1) : 1024;
  if ((rc = dalloc(&w.eo, R * ceo * neo1, total))) return rc;
  if ((rc = dalloc(&w.geo, R * cgeo * neo1, total))) return rc;
  if ((rc = dalloc(&w.alm_a, ceo * na, total))) return rc;
  if ((rc = dalloc(&w.alm_b, cgeo * na, total))) return rc;
  double2** avec[] = {&w.cg_x, &w.cg_r, &w.cg_z, &w.cg_p, &w.cg_q, &w.cg_b, &w.cg_d};
  for (double2** a : avec)
    if ((rc = dalloc(a, C * na, total))) return rc;
  if ((rc = dalloc(&w.cg_xacc, C * na, total))) return rc;
  if ((rc = dalloc(&w.cg_bin, C * na, total))) return rc;
  if (ncomp == 3) {
    // polar ring pairs (a prefix: pairs run from the north pole towards the
    // equator), whose spin-2 spectra divide Legendre sums by sin^2 theta
    int npol = 0;
    while (npol < np && (1.0 - pz[npol]) * (1.0 + pz[npol]) < crsht::kPolarSin2) ++npol;
    P->npol = npol;
    if (npol > 0 && (rc = dalloc(&w.pol, R * ceo * (size_t)npol * (size_t)(mmax + 1) * 2, total))) return rc;
  }
  {
    unsigned char *ab = nullptr, *ag = nullptr;
    if ((rc = dalloc(&ab, (size_t)crsht::mixed_ab_bytes(g), total))) return rc;
    w.mx_ab = ab;
    if ((rc = dalloc(&ag, (size_t)crsht::mixed_ag_bytes(g), total))) return rc;
    w.mx_ag = ag;
    if ((rc = dalloc(&w.adj_part, R * (size_t)P->t.mx_ntiles, total))) return rc;
  }
  if ((rc = dalloc(&w.alm_c, C * (size_t)g.nalm, total))) return rc;
  if ((rc = dalloc(&w.alm_d, C * (size_t)g.nalm, total))) return rc;
  if ((rc = dalloc(&w.map_a, R * C * (size_t)g.npix, total))) return rc;
  if ((rc = dalloc(&w.ring_w, (size_t)np, total))) return rc;
  double** dvec[] = {&w.diag, &w.sinv, &w.sinvhalf, &w.bk};
  for (double** a : dvec)
    if ((rc = dalloc(a, C * (size_t)g.nalm, total))) return rc;
  if ((rc = dalloc(&w.bl_keep, (size_t)g.nalm, total))) return rc;
  if ((rc = dalloc(&w.sblk, 8 * (size_t)(lmax + 1), total))) return rc;
  if ((rc = dalloc(&w.perl, 4 * (size_t)(lmax + 1), total))) return rc;
  if ((rc = dalloc(&w.partial, R * (size_t)w.npart * 4, total))) return rc;
  if ((rc = dalloc(&w.bin_edges, (size_t)lmax + 2, total))) return rc;
  if ((rc = dalloc(&w.bin_part, (size_t)(lmax + 1) * crsht::kBinSlices * 3, total))) return rc;
  if ((rc = dalloc(&w.bin_grad, (size_t)lmax + 1, total))) return rc;
  if ((rc = dalloc(&w.lfac, (size_t)lmax + 1, total))) return rc;
  {
    std::vector<double> ones(2 * R, 1.0);
    if ((rc = upload(reinterpret_cast<double**>(&w.camp), ones, total))) return rc;
  }
  if ((rc = dalloc(&w.scal, R * crsht::kScalSlots, total))) return rc;
  if (hipHostMalloc((void**)&w.host_scal, R * crsht::kScalSlots * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    w.host_scal = nullptr;
    return CR_ENOMEM;
  }
  if (hipMemset(w.scal, 0, R * crsht::kScalSlots * sizeof(double)) != hipSuccess) return CR_EDEVICE;
  if ((rc = dalloc(&w.ctl, (size_t)crsht::kCtlSlots, total))) return rc;
  if (hipMemset(w.ctl, 0, crsht::kCtlSlots * sizeof(int)) != hipSuccess) return CR_EDEVICE;
  // device-visible pinned word polled by the batched driver (coherent: the
  // host reads it while kernels may still write it)
  if (hipHostMalloc((void**)&w.host_exited, 64, hipHostMallocCoherent) != hipSuccess) {
    w.host_exited = nullptr;
    return CR_ENOMEM;
  }
  *w.host_exited = 1;
  // pinned staging slots for the per-call host data: column amplitudes, the
  // per-l arrays and (T+Q+U) the 3x3 spectra blocks
  P->stage_bytes = 16 * (size_t)R + 12 * sizeof(double) * (size_t)(lmax + 1) + 1024;
  for (int k = 0; k < crsht_plan::kStageSlots; ++k) {
    if (hipHostMalloc(&P->stage_host[k], P->stage_bytes, hipHostMallocDefault) != hipSuccess) {
      P->stage_host[k] = nullptr;
      return CR_ENOMEM;
    }
    if (hipEventCreateWithFlags(&P->stage_ev[k], hipEventDisableTiming) != hipSuccess) {
      P->stage_ev[k] = nullptr;
      return CR_EDEVICE;
    }
  }
  if (hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    P->cap_stream = nullptr;
    return CR_EDEVICE;
  }
  if (hipStreamCreateWithFlags(&P->exec_stream, hipStreamNonBlocking) != hipSuccess) {
    P->exec_stream = nullptr;
    return CR_EDEVICE;
  }
  hipEvent_t* evs[] = {&P->ev_fork, &P->ev_join, &P->ev_round[0], &P->ev_round[1], &P->ev_round[2]};
  for (hipEvent_t* e : evs)
    if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
      *e = nullptr;
      return CR_EDEVICE;
    }
  if (hipEventCreateWithFlags(&P->aux_fork_ev, hipEventDisableTiming) != hipSuccess) {
    P->aux_fork_ev = nullptr;
    return CR_EDEVICE;
  }
  for (int k = 0; k < crsht_plan::kAux; ++k) {
    if (hipStreamCreateWithFlags(&P->aux_stream[k], hipStreamNonBlocking) != hipSuccess) {
      P->aux_stream[k] = nullptr;
      return CR_EDEVICE;
    }
    if (hipEventCreateWithFlags(&P->aux_join_ev[k], hipEventDisableTiming) != hipSuccess) {
      P->aux_join_ev[k] = nullptr;
      return CR_EDEVICE;
    }
  }
  {
    unsigned char* ds = nullptr;
    if ((rc = dalloc(&ds, R * sizeof(cr_stats), total))) return rc;
    w.dstats = ds;
  }
  return CR_OK;
}

extern "C" int crsht_plan_create(int nside, int lmax, int mmax, int ncomp, int nrhs_max, crsht_plan** out) {
  if (!out) return CR_EINVAL;
  *out = nullptr;
  if (mmax < 0) mmax = lmax;
  if (nside < 1 || lmax < 0 || mmax > lmax || nrhs_max < 1 || nrhs_max > 4096) return CR_EINVAL;
  if (lmax > 16383) return CR_EINVAL;
  if (nside > 1024) return CR_ENOTSUP;  // FP64 adjoint: at most 8 ring pairs per thread x 256 threads
  if (ncomp != 1 && ncomp != 3) return CR_EINVAL;
  crsht_plan* P = new (std::nothrow) crsht_plan();
  if (!P) return CR_ENOMEM;
  P->ncomp = ncomp;
  P->nrhs_max = nrhs_max;
  if (hipGetDevice(&P->device) != hipSuccess) {
    delete P;
    return CR_EDEVICE;
  }
  size_t total = 0;
  int rc = build_plan(P, nside, lmax, mmax, ncomp, nrhs_max, &total);
  if (rc != CR_OK) {
    free_plan_memory(P);
    delete P;
    return rc;
  }
  P->workspace_bytes_ = (int64_t)total;
  // device address of the allocation-free call's scratch on this device
  // (once per device; a failure only disables sht_synth_noalloc)
  (void)crsht::noalloc_setup(P->device);
  *out = P;
  return CR_OK;
}

extern "C" void crsht_plan_destroy(crsht_plan* P) {
  if (!P) return;
  (void)hipDeviceSynchronize();
  free_plan_memory(P);
  delete P;
}

extern "C" const char* crsht_strerror(int status) {
  switch (status) {
    case CR_OK: return "success";
    case CR_EINVAL: return "invalid argument";
    case CR_ENOMEM: return "device allocation failed";
    case CR_EDEVICE: return "HIP runtime error";
    case CR_ENOTSUP: return "not supported by this library";
    case CR_ESCRATCH: return "the input needs more than the static scratch of the allocation-free call";
    case CR_NOCONV: return "maximum iterations reached before the tolerance";
    case CR_BREAKDOWN: return "conjugate-gradient breakdown (non-positive or non-finite curvature)";
    default: return "unknown status";
  }
}

extern "C" int crsht_plan_info(const crsht_plan* P, crsht_info* info) {
  if (!P || !info) return CR_EINVAL;
  info->nside = P->g.nside;
  info->lmax = P->g.lmax;
  info->mmax = P->g.mmax;
  info->ncomp = P->ncomp;
  info->nrhs_max = P->nrhs_max;
  info->nrings = P->g.nrings;
  info->npix = P->g.npix;
  info->nalm = P->g.nalm;
  info->workspace_bytes = P->workspace_bytes_;
  info->precond_bytes = P->pc.built ? P->pc.stored_bytes : 0;
  info->precond_blocks = P->pc.built ? P->pc.nblocks : 0;
  info->precond_half_blocks = P->pc.built ? P->pc.nhalf : 0;
  info->live_pair_m = P->t.live_pair_m;
  return CR_OK;
}

extern "C" int crsht_pixel_coords(const crsht_plan* P, double* z, double* phi) {
  if (!P || !z || !phi) return CR_EINVAL;
  const ld twopi = 2.0L * kPi;
  for (int r = 0; r < P->g.nrings; ++r) {
    const int n = P->h_nphi[r];
    const int64_t f = P->h_first[r];
    for (int j = 0; j < n; ++j) {
      z[f + j] = P->h_z[r];
      phi[f + j] = (double)((ld)P->h_phi0[r] + twopi * (ld)j / (ld)n);
    }
  }
  return CR_OK;
}
