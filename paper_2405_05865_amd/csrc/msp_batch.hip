// Host side of the batched PSD solve: validation, workspace layout, the per-system
// level-2 operator H = C^T C + lam~ W, work ordering, and the launch of k_batch_psd.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <numeric>
#include <vector>

#include "msp_batched.h"

#define BREQUIRE(cond, ...)                                            \
  do {                                                                 \
    if (!(cond)) return msp_fail(MSP_ERR_INVALID_ARG, __VA_ARGS__);    \
  } while (0)

namespace {

bool batch_log_on() {
  const char* e = getenv("MSP_LOG");
  return e && e[0] && e[0] != '0';
}

size_t esize(msp_dtype t) { return t == MSP_F64 ? 8 : (t == MSP_F32 ? 4 : 2); }
int64_t round8(int64_t v) { return (v + 7) / 8 * 8; }
bool aligned16(const void* p, int64_t ld, size_t es) {
  return ((uintptr_t)p % 16 == 0) && ((ld * (int64_t)es) % 16 == 0);
}

struct BatchLayout {
  BatchSys* dsys = nullptr;
  BatchOut* dout = nullptr;
  BatchTeam* team = nullptr;  // nsys records, zeroed before every launch
  std::vector<double*> cpart, ypart;
  std::vector<double*> H;
  std::vector<double*> vec;
  std::vector<float*> pf;
  double* gpart = nullptr;
};

// workspace: descriptors, results, per system H (s x s), 11 n-vectors + 7 s-vectors and
// an F32 direction (kcap columns each), then the Gram split partials
size_t batch_layout(WsCarver& w, int32_t nsys, const msp_system* sys, int kcap, BatchLayout* L) {
  BatchSys* dsys = w.take<BatchSys>(nsys);
  BatchOut* dout = w.take<BatchOut>(nsys);
  BatchTeam* team = w.take<BatchTeam>(nsys);
  if (L) {
    L->dsys = dsys;
    L->dout = dout;
    L->team = team;
    L->cpart.resize(nsys);
    L->ypart.resize(nsys);
    L->H.resize(nsys);
    L->vec.resize(nsys);
    L->pf.resize(nsys);
  }
  size_t gmax = 0;
  for (int32_t i = 0; i < nsys; ++i) {
    const msp_precond* P = sys[i].P;
    const int64_t n = P->n, s = P->s;
    double* H = w.take<double>(s * s);
    const size_t nch = (size_t)((n + MSP_BATCH_CHR - 1) / MSP_BATCH_CHR);
    double* cp = w.take<double>(nch * MSP_BATCH_KMAX);
    double* yp = w.take<double>(nch * MSP_BATCH_KMAX * s);
    double* v = w.take<double>((size_t)kcap * (11 * round8(n) + 7 * round8(s)));
    float* f = w.take<float>((size_t)kcap * round8(n));
    if (L) {
      L->cpart[i] = cp;
      L->ypart[i] = yp;
      L->H[i] = H;
      L->vec[i] = v;
      L->pf[i] = f;
    }
    const int sp = gram_splits(n, s);
    if (sp > 1) gmax = std::max(gmax, (size_t)sp * s * s);
  }
  double* g = w.take<double>(gmax + 1);
  if (L) L->gpart = g;
  return w.off;
}

msp_status validate_batch(int32_t nsys, const msp_system* sys, msp_dtype hi_t, msp_dtype lo_t, int64_t k,
                          const msp_solve_opts* o) {
  BREQUIRE(nsys >= 1 && sys, "need at least one system");
  BREQUIRE(k >= 1 && k <= 1024, "need 1 <= k <= 1024");
  BREQUIRE(o, "null options");
  if (!std::isfinite(o->tol) || !std::isfinite(o->inner_tol) || !std::isfinite(o->refine_inner_tol))
    return msp_fail(MSP_ERR_NONFINITE, "non-finite tolerance");
  BREQUIRE(o->tol > 0 && o->inner_tol > 0 && o->refine_inner_tol > 0, "tolerances must be > 0");
  BREQUIRE(o->max_outer >= 1 && o->max_inner >= 1 && o->max_refine >= 1, "caps must be >= 1");
  const msp_dtype yt = sys[0].P ? sys[0].P->y_t : MSP_F64;
  for (int32_t i = 0; i < nsys; ++i) {
    const msp_system& q = sys[i];
    BREQUIRE(q.P, "system %d: null handle", i);
    BREQUIRE(q.P->structure == MSP_SYM_PSD, "system %d: the batched solve needs MSP_SYM_PSD handles", i);
    BREQUIRE(q.A_hi && q.A_lo && q.B && q.X, "system %d: null pointer", i);
    BREQUIRE(q.lda >= q.P->n && q.ldb >= q.P->n && q.ldx >= q.P->n, "system %d: leading dimension < n", i);
    BREQUIRE(q.P->y_t == yt, "system %d: every handle must store Y in the same dtype", i);
    BREQUIRE(q.P->n <= (int64_t)1 << 30, "system %d: n too large", i);
  }
  if (!batch_types_supported(lo_t, hi_t, yt))
    return msp_fail(MSP_ERR_UNSUPPORTED, "batched solve supports (lo, hi, Y) = (F64, F64, F64) or "
                                         "(F32/BF16, F32/F64, F32)");
  return MSP_OK;
}

}  // namespace

extern "C" msp_status msp_solve_batched_workspace(int32_t nsys, const msp_system* sys, int64_t k,
                                                  const msp_solve_opts* opts, size_t* bytes) {
  BREQUIRE(bytes && sys && nsys >= 1 && k >= 1, "invalid arguments");
  for (int32_t i = 0; i < nsys; ++i) BREQUIRE(sys[i].P, "system %d: null handle", i);
  (void)opts;
  WsCarver w(nullptr, 0);
  batch_layout(w, nsys, sys, (int)std::min<int64_t>(k, MSP_BATCH_KMAX), nullptr);
  *bytes = w.off;
  return MSP_OK;
}

extern "C" msp_status msp_solve_batched(void* stream, int32_t nsys, const msp_system* sys, msp_dtype hi_t,
                                        msp_dtype lo_t, int64_t k, const msp_solve_opts* opts, void* ws,
                                        size_t ws_bytes, msp_solve_info* info) {
  msp_solve_opts dflt;
  msp_solve_opts_default(&dflt);
  const msp_solve_opts* o = opts ? opts : &dflt;
  msp_status vs = validate_batch(nsys, sys, hi_t, lo_t, k, o);
  if (vs != MSP_OK) return vs;
  const int kcap = (int)std::min<int64_t>(k, MSP_BATCH_KMAX);
  size_t need = 0;
  msp_solve_batched_workspace(nsys, sys, k, o, &need);
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255))
    return msp_fail(MSP_ERR_WORKSPACE, "batched workspace needs %zu bytes, 256-B aligned", need);
  hipStream_t st = (hipStream_t)stream;
  WsCarver w(ws, ws_bytes);
  BatchLayout L;
  batch_layout(w, nsys, sys, kcap, &L);
  const msp_dtype yt = sys[0].P->y_t;

  // level-2 operator of every system: H = C^T C + lam~ W (FP64)
  for (int32_t i = 0; i < nsys; ++i) {
    const msp_precond* P = sys[i].P;
    const int sp = gram_splits(P->n, P->s);
    if (yt == MSP_F64)
      MSP_CHECK_HIP(launch_gram(st, (const double*)P->Y, P->n, P->s, P->ldy, L.H[i], L.gpart, sp));
    else
      MSP_CHECK_HIP(launch_gram_f32(st, (const float*)P->Y, P->n, P->s, P->ldy, L.H[i], L.gpart, sp));
    MSP_CHECK_HIP(launch_combine_sym(st, P->s, 1.0, L.H[i], P->lt, P->Wm, 0.0, L.H[i]));
  }

  // largest systems first: the dispatcher hands them out in launch order
  std::vector<int32_t> order(nsys);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    const double wa = (double)sys[a].P->n * sys[a].P->n, wb = (double)sys[b].P->n * sys[b].P->n;
    return wa > wb;
  });

  BatchPrm prm{};
  prm.tol = o->tol;
  prm.inner_tol = o->inner_tol;
  prm.refine_tol = o->refine_inner_tol;
  prm.max_outer = o->max_outer;
  prm.max_inner = o->max_inner;
  prm.max_refine = o->max_refine;
  prm.refine = (o->refine && lo_t != MSP_F64) ? 1 : 0;
  prm.kcap = kcap;
  prm.profile = o->profile ? 1 : 0;
  prm.teams = o->batch_teams ? 1 : 0;
  prm.nsys = nsys;
  int clock_khz = 0;
  if (prm.profile) {
    int dev = 0;
    MSP_CHECK_HIP(hipGetDevice(&dev));
    MSP_CHECK_HIP(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev));
  }

  std::vector<BatchSys> hs(nsys);
  std::vector<BatchOut> ho(nsys);
  std::vector<msp_solve_info> acc(nsys);
  for (auto& a : acc) a = msp_solve_info{};
  for (int64_t j0 = 0; j0 < k; j0 += MSP_BATCH_KMAX) {
    const int kk = (int)std::min<int64_t>(MSP_BATCH_KMAX, k - j0);
    for (int32_t q = 0; q < nsys; ++q) {
      const int32_t i = order[q];
      const msp_system& u = sys[i];
      const msp_precond* P = u.P;
      BatchSys d{};
      d.A_lo = u.A_lo;
      d.A_hi = u.A_hi;
      d.lda = u.lda;
      d.Y = P->Y;
      d.ldy = P->ldy;
      d.H = L.H[i];
      d.Minv = P->Minv;
      d.B = u.B + j0 * u.ldb;
      d.ldb = u.ldb;
      d.X = u.X + j0 * u.ldx;
      d.ldx = u.ldx;
      d.vec = L.vec[i];
      d.pf = L.pf[i];
      d.n = (int32_t)P->n;
      d.s = (int32_t)P->s;
      d.ldn = (int32_t)round8(P->n);
      d.lds = (int32_t)round8(P->s);
      d.lam = P->lam;
      d.lt = P->lt;
      d.aln_lo = aligned16(u.A_lo, u.lda, esize(lo_t));
      d.aln_hi = aligned16(u.A_hi, u.lda, esize(hi_t));
      d.aln_y = aligned16(P->Y, P->ldy, esize(yt));
      d.aln_m = aligned16(P->Minv, P->s, 8) && aligned16(L.H[i], P->s, 8);
      d.team = L.team + q;  // records in launch order: helpers scan the largest systems first
      d.cpart = L.cpart[i];
      d.ypart = L.ypart[i];
      d.id = i;
      hs[q] = d;
    }
    MSP_CHECK_HIP(hipMemcpyAsync(L.dsys, hs.data(), sizeof(BatchSys) * nsys, hipMemcpyHostToDevice, st));
    MSP_CHECK_HIP(hipMemsetAsync(L.team, 0, sizeof(BatchTeam) * nsys, st));
    MSP_CHECK_HIP(launch_batch_psd(st, lo_t, hi_t, yt, L.dsys, nsys, prm, kk, L.dout));
    MSP_CHECK_HIP(hipMemcpyAsync(ho.data(), L.dout, sizeof(BatchOut) * nsys, hipMemcpyDeviceToHost, st));
    MSP_CHECK_HIP(hipStreamSynchronize(st));
    for (int32_t i = 0; i < nsys; ++i) {
      const BatchOut& r = ho[i];
      msp_solve_info& a = acc[i];
      const msp_status s = r.code == 0 ? MSP_OK
                           : r.code == 1 ? MSP_ERR_NO_CONVERGENCE
                           : r.code == 2 ? MSP_ERR_BREAKDOWN
                           : r.code == 3 ? MSP_ERR_NONFINITE
                                         : MSP_ERR_HIP;
      if (a.status == MSP_OK) a.status = s;
      a.outer_iters += r.outer;
      a.inner_iters += r.inner;
      a.refine_steps += r.refine;
      a.restarts += r.restarts;
      a.krylov_refine = prm.refine;
      a.rel_residual_max = std::max(a.rel_residual_max, r.relres);
      a.sweeps += (int64_t)r.outer + r.refine;
      if (prm.profile && clock_khz > 0) {
        // sweep_ms: the level-1 sweeps of this system; the other phases go to the log
        const double ms = 1.0 / clock_khz;
        a.sweep_ms += r.ticks[BT_SWEEP_LO] * ms;
        a.timed_sweeps += r.outer;
        if (batch_log_on())
          fprintf(stderr, "[msp] batch system %d n=%d: total %.2f ms | sweep_lo %.2f  sweep_hi %.2f  Y^T r %.2f  "
                          "level-2 %.2f  Y y %.2f | outer %d inner %d refine %d | slices helped %d self %d\n",
                  i, (int)sys[i].P->n, r.ticks[BT_TOTAL] * ms, r.ticks[BT_SWEEP_LO] * ms, r.ticks[BT_SWEEP_HI] * ms,
                  r.ticks[BT_YT] * ms, r.ticks[BT_LEVEL2] * ms, r.ticks[BT_YZ] * ms, r.outer, r.inner, r.refine,
                  r.helped, r.selfdone);
      }
    }
  }
  msp_status ret = MSP_OK;
  for (int32_t i = 0; i < nsys; ++i) {
    if (info) info[i] = acc[i];
    if (ret == MSP_OK && acc[i].status != MSP_OK) {
      ret = acc[i].status;
      msp_fail(ret, "system %d: %s (relative residual %.3e)", i,
               ret == MSP_ERR_NO_CONVERGENCE ? "tolerance not reached"
               : ret == MSP_ERR_BREAKDOWN    ? "breakdown"
               : ret == MSP_ERR_HIP          ? "a helper workgroup's sweep slice did not complete in time"
                                             : "non-finite residual",
               acc[i].rel_residual_max);
    }
  }
  return ret;
}

// ------------------------------------------------------------------------------------
// adjoints: the batched solve on G, then dlambda_i = -sum_j <dB_ij, X_ij> and dA_i
// ------------------------------------------------------------------------------------
namespace {

std::vector<msp_system> adjoint_systems(int32_t nsys, const msp_system_grad* sys) {
  std::vector<msp_system> fw(nsys);
  for (int32_t i = 0; i < nsys; ++i) {
    const msp_system_grad& g = sys[i];
    fw[i] = msp_system{g.P, g.A_hi, g.A_lo, g.lda, g.G, g.ldg, g.dB, g.lddb};
  }
  return fw;
}

}  // namespace

extern "C" msp_status msp_solve_batched_backward_workspace(int32_t nsys, const msp_system_grad* sys, int64_t k,
                                                           const msp_solve_opts* opts, size_t* bytes) {
  BREQUIRE(bytes && sys && nsys >= 1 && k >= 1, "invalid arguments");
  for (int32_t i = 0; i < nsys; ++i) BREQUIRE(sys[i].P, "system %d: null handle", i);
  const std::vector<msp_system> fw = adjoint_systems(nsys, sys);
  size_t solve = 0;
  msp_status s = msp_solve_batched_workspace(nsys, fw.data(), k, opts, &solve);
  if (s != MSP_OK) return s;
  *bytes = ((solve + 255) & ~size_t(255)) + (((size_t)nsys * k * sizeof(double) + 255) & ~size_t(255));
  return MSP_OK;
}

extern "C" msp_status msp_solve_batched_backward(void* stream, int32_t nsys, const msp_system_grad* sys,
                                                 msp_dtype hi_t, msp_dtype lo_t, int64_t k,
                                                 const msp_solve_opts* opts, void* ws, size_t ws_bytes,
                                                 double* dlambda, msp_solve_info* info) {
  BREQUIRE(nsys >= 1 && sys, "need at least one system");
  for (int32_t i = 0; i < nsys; ++i) {
    const msp_system_grad& g = sys[i];
    BREQUIRE(g.P, "system %d: null handle", i);
    BREQUIRE(g.X && g.G && g.dB, "system %d: null X, G or dB", i);
    BREQUIRE(g.ldx >= g.P->n && g.ldg >= g.P->n && g.lddb >= g.P->n, "system %d: leading dimension < n", i);
    BREQUIRE(!g.dA || g.ldda >= g.P->n, "system %d: ldda < n", i);
  }
  size_t need = 0;
  msp_status s = msp_solve_batched_backward_workspace(nsys, sys, k, opts, &need);
  if (s != MSP_OK) return s;
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255))
    return msp_fail(MSP_ERR_WORKSPACE, "batched adjoint workspace needs %zu bytes, 256-B aligned", need);
  const std::vector<msp_system> fw = adjoint_systems(nsys, sys);
  size_t solve = 0;
  msp_solve_batched_workspace(nsys, fw.data(), k, opts, &solve);
  solve = (solve + 255) & ~size_t(255);
  // dB_i = (A_i + lam_i I)^{-1} G_i
  const msp_status ret = msp_solve_batched(stream, nsys, fw.data(), hi_t, lo_t, k, opts, ws, solve, info);
  if (ret != MSP_OK && ret != MSP_ERR_NO_CONVERGENCE) return ret;
  hipStream_t st = (hipStream_t)stream;
  double* dv = (double*)((char*)ws + solve);
  for (int32_t i = 0; i < nsys; ++i) {
    const msp_system_grad& g = sys[i];
    const int64_t n = g.P->n;
    MSP_CHECK_HIP(launch_coldots(st, n, k, g.dB, g.lddb, g.X, g.ldx, dv + (size_t)i * k));
    if (g.dA) MSP_CHECK_HIP(launch_outer_neg(st, n, k, g.dB, g.lddb, g.X, g.ldx, g.dA, g.ldda));
  }
  std::vector<double> h((size_t)nsys * k);
  MSP_CHECK_HIP(hipMemcpyAsync(h.data(), dv, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
  MSP_CHECK_HIP(hipStreamSynchronize(st));
  if (dlambda)
    for (int32_t i = 0; i < nsys; ++i) {
      double t = 0.0;
      for (int64_t j = 0; j < k; ++j) t += h[(size_t)i * k + j];
      dlambda[i] = -t;
    }
  return ret;
}
