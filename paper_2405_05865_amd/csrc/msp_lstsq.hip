// Least squares min |A x - b| for a tall A (n x d, n >= d) by sketch-and-precondition with
// MSP as the inner solver (the least-squares corollary of Section 3):
//   msp_left_sketch: Psi (Definition 2.1, q rows over the n rows of A) and A~ = Psi A, a
//     q x d subspace embedding of A (the row gather of the Nystrom build, k_sketch.hip);
//   msp_lstsq: flexible PCG on A^T A x = A^T b whose preconditioner applies (A~^T A~)^{-1}
//     through msp_solve on an MSP_GENERAL handle of A~ (three levels, lam = 0), to the
//     relative accuracy opts->refine_inner_tol: a constant accuracy suffices because the
//     outer iteration is flexible and A~^T A~ is spectrally within a constant of A^T A.
// Both products with A run with FP64 arithmetic (an FP32 A is read as stored): the normal
// equations square A's condition number. The outer stop is |A^T (b - A x)| <= tol |A^T b|
// per right-hand side, on the recurrence residual and confirmed on the recomputed one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "msp_internal.h"

#define LREQUIRE(cond, ...)                                          \
  do {                                                               \
    if (!(cond)) return msp_fail(MSP_ERR_INVALID_ARG, __VA_ARGS__);  \
  } while (0)

#define LTRY(expr)                \
  do {                            \
    msp_status _s = (expr);       \
    if (_s != MSP_OK) return _s;  \
  } while (0)

namespace {

constexpr int kLsGammaMax = 32;  // nonzeros per column the index draw supports
constexpr int kLsSlot = 32;      // host-mirror slots of the outer iteration (the inner solves use 0..19)

struct LeftSketchWs {
  BucketLists b;
  void* scratch;
};

LeftSketchWs carve_left(WsCarver& w, int64_t n, int64_t q, int32_t gamma) {
  LeftSketchWs o;
  o.b.offsets = w.take<int32_t>(q + 1);
  o.b.entries = w.take<int32_t>(n * gamma);
  o.scratch = w.take<char>(bucket_scratch_bytes(n, q, gamma));
  return o;
}

struct LsWs {
  FcgState S;
  double *c, *x, *r, *ro, *z, *p, *q, *t, *tpart, *gsplit, *dots;
  size_t gsplit_n = 0;
  void* inner = nullptr;
};

LsWs carve_ls(WsCarver& w, int64_t n, int64_t d, int64_t k, size_t inner_bytes) {
  LsWs o;
  o.S = carve_fcg_state(w, d, k);
  o.c = w.take<double>(d * k);
  o.x = w.take<double>(d * k);
  o.r = w.take<double>(d * k);
  o.ro = w.take<double>(d * k);
  o.z = w.take<double>(d * k);
  o.p = w.take<double>(d * k);
  o.q = w.take<double>(d * k);
  o.t = w.take<double>(n * k);
  o.tpart = w.take<double>(std::max(gemv_t_part_doubles(n, d, k), gemm_t_part_doubles(n, d, k)));
  o.gsplit_n = k >= kGemmMinK ? gemm_split_doubles(n, k) : 0;
  o.gsplit = o.gsplit_n ? w.take<double>(o.gsplit_n) : nullptr;
  o.dots = w.take<double>(2 * k);
  o.inner = w.take<char>(inner_bytes);
  return o;
}

msp_solve_opts inner_opts(const msp_solve_opts& o) {
  msp_solve_opts io = o;
  io.normal = 1;
  io.refine = 0;
  io.tol = o.refine_inner_tol;
  io.use_graph = 0;
  io.autotune = 0;
  return io;
}

// t = A v (n x k) and out = A^T t (d x k), FP64 arithmetic on F64 or F32 storage
hipError_t normal_op(hipStream_t st, const void* A, msp_dtype a_t, int64_t n, int64_t d, int64_t lda,
                     const double* v, double* out, int64_t k, const int32_t* skip, LsWs& w) {
  hipError_t e;
  int nb = 0;
  if (k >= kGemmMinK)
    e = launch_gemm_split(st, A, a_t, a_t == MSP_F32, n, d, lda, v, d, w.t, n, k, 0.0, false, skip, nullptr, &nb,
                          w.gsplit, w.gsplit_n, 0);
  else if (a_t == MSP_F32)
    e = launch_gemv_f32_as_f64(st, (const float*)A, n, d, lda, v, d, w.t, n, k, 0.0, false, skip, nullptr, &nb);
  else
    e = launch_gemv(st, A, a_t, n, d, lda, v, d, w.t, n, k, 0.0, false, skip, nullptr, &nb);
  if (e != hipSuccess) return e;
  if (a_t == MSP_F32)
    return (k >= kGemmMinK ? launch_gemm_t_f32_as_f64 : launch_gemv_t_f32_as_f64)(st, (const float*)A, n, d, lda, w.t,
                                                                                  n, out, d, k, skip, w.tpart);
  return (k >= kGemmMinK ? launch_gemm_t : launch_gemv_t)(st, A, a_t, n, d, lda, w.t, n, out, d, k, skip, w.tpart);
}

// out = A^T B for B (n x k, ld ldb)
hipError_t transpose_op(hipStream_t st, const void* A, msp_dtype a_t, int64_t n, int64_t d, int64_t lda,
                        const double* B, int64_t ldb, double* out, int64_t k, LsWs& w) {
  if (a_t == MSP_F32)
    return (k >= kGemmMinK ? launch_gemm_t_f32_as_f64 : launch_gemv_t_f32_as_f64)(st, (const float*)A, n, d, lda, B,
                                                                                  ldb, out, d, k, nullptr, w.tpart);
  return (k >= kGemmMinK ? launch_gemm_t : launch_gemv_t)(st, A, a_t, n, d, lda, B, ldb, out, d, k, nullptr, w.tpart);
}

}  // namespace

// ====================================================================================
// msp_left_sketch
// ====================================================================================
extern "C" msp_status msp_left_sketch_workspace(int64_t n, int64_t q, int32_t gamma, size_t* bytes) {
  LREQUIRE(bytes, "null argument");
  LREQUIRE(n >= 1 && q >= 1 && gamma >= 1 && gamma <= q && gamma <= kLsGammaMax, "invalid sizes");
  WsCarver w(nullptr, 0);
  carve_left(w, n, q, gamma);
  *bytes = w.off;
  return MSP_OK;
}

extern "C" msp_status msp_left_sketch(void* stream, const void* A, msp_dtype a_t, int64_t n, int64_t d, int64_t lda,
                                      int64_t q, int32_t gamma, uint64_t seed, int32_t* Psi_rows, int8_t* Psi_signs,
                                      double* At, int64_t ldat, void* ws, size_t ws_bytes) {
  LREQUIRE(A && Psi_rows && Psi_signs && At && ws, "null pointer argument");
  LREQUIRE(a_t == MSP_F64 || a_t == MSP_F32, "A must be F64 or F32");
  LREQUIRE(n >= 1 && d >= 1 && lda >= d && q >= 1 && ldat >= d, "invalid sizes or leading dimensions");
  LREQUIRE(gamma >= 1 && gamma <= q && gamma <= kLsGammaMax, "need 1 <= gamma <= min(q, 32)");
  LREQUIRE(n * (int64_t)gamma < (int64_t(1) << 30), "n * gamma too large");
  size_t need = 0;
  LTRY(msp_left_sketch_workspace(n, q, gamma, &need));
  if (ws_bytes < need || ((uintptr_t)ws & 255))
    return msp_fail(MSP_ERR_WORKSPACE, "left-sketch workspace needs %zu bytes, 256-B aligned", need);
  hipStream_t st = (hipStream_t)stream;
  WsCarver w(ws, ws_bytes);
  LeftSketchWs o = carve_left(w, n, q, gamma);
  MSP_CHECK_HIP(launch_sketch_gen(st, seed, n, q, gamma, Psi_rows, Psi_signs));
  MSP_CHECK_HIP(build_buckets(st, Psi_rows, Psi_signs, n, q, gamma, o.b, o.scratch));
  MSP_CHECK_HIP(launch_gather_rows(st, A, a_t, lda, d, q, o.b, 1.0 / std::sqrt((double)gamma), At, ldat));
  return MSP_OK;
}

// ====================================================================================
// msp_lstsq
// ====================================================================================
extern "C" msp_status msp_lstsq_workspace(const msp_precond* P, int64_t n, int64_t k, const msp_solve_opts* opts,
                                          size_t* bytes) {
  LREQUIRE(P && bytes, "null argument");
  LREQUIRE(P->structure == MSP_GENERAL, "msp_lstsq needs an MSP_GENERAL handle of A~");
  LREQUIRE(n >= P->n && k >= 1, "need n >= d and k >= 1");
  msp_solve_opts dflt;
  msp_solve_opts_default(&dflt);
  const msp_solve_opts io = inner_opts(opts ? *opts : dflt);
  size_t inner = 0;
  LTRY(msp_solve_workspace(P, k, &io, &inner));
  WsCarver w(nullptr, 0);
  carve_ls(w, n, P->n, k, inner);
  *bytes = w.off;
  return MSP_OK;
}

extern "C" msp_status msp_lstsq(void* stream, const msp_precond* P, const double* At, int64_t ldat, const void* A,
                                msp_dtype a_t, int64_t n, int64_t lda, const double* B, int64_t ldb, int64_t k,
                                double* X, int64_t ldx, const msp_solve_opts* opts, void* ws, size_t ws_bytes,
                                msp_solve_info* info) {
  LREQUIRE(P && At && A && B && X && ws, "null pointer argument");
  LREQUIRE(P->structure == MSP_GENERAL, "msp_lstsq needs an MSP_GENERAL handle of A~");
  LREQUIRE(P->lam == 0.0, "the handle of A~ must have lambda = 0");
  LREQUIRE(a_t == MSP_F64 || a_t == MSP_F32, "A must be F64 or F32");
  const int64_t d = P->n;
  LREQUIRE(n >= d && lda >= d && ldat >= d && ldb >= n && ldx >= d && k >= 1, "invalid sizes or leading dimensions");
  msp_solve_opts dflt;
  msp_solve_opts_default(&dflt);
  const msp_solve_opts& o = opts ? *opts : dflt;
  LREQUIRE(o.tol > 0 && o.refine_inner_tol > 0 && o.max_outer >= 1, "invalid tolerances or caps");
  const msp_solve_opts io = inner_opts(o);
  size_t inner = 0, need = 0;
  LTRY(msp_solve_workspace(P, k, &io, &inner));
  LTRY(msp_lstsq_workspace(P, n, k, &o, &need));
  if (ws_bytes < need || ((uintptr_t)ws & 255))
    return msp_fail(MSP_ERR_WORKSPACE, "least-squares workspace needs %zu bytes, 256-B aligned", need);
  hipStream_t st = (hipStream_t)stream;
  WsCarver wc(ws, ws_bytes);
  LsWs w = carve_ls(wc, n, d, k, inner);
  int32_t* mirror = P->dev_view_flags + kLsSlot;
  volatile int32_t* host = P->host_flags + kLsSlot;
  msp_solve_info acc{};
  const double abytes = (double)n * (double)d * (a_t == MSP_F64 ? 8.0 : 4.0);
  MSP_CHECK_HIP(hipMemsetAsync(w.S.counter, 0, sizeof(int32_t), st));
  // the preconditioner: z = (A~^T A~)^{-1} r by the three-level MSP on A~
  auto prec = [&](const double* r, double* z) -> msp_status {
    msp_solve_info ii{};
    const msp_status s_ = msp_solve(stream, P, At, MSP_F64, At, MSP_F64, ldat, 0.0, r, d, k, z, d, &io, w.inner, inner,
                                    &ii);
    // an inner solve that stops early (cap or breakdown) still returns its iterate, which the
    // flexible outer iteration can use
    if (s_ != MSP_OK && s_ != MSP_ERR_NO_CONVERGENCE && s_ != MSP_ERR_BREAKDOWN) return s_;
    acc.inner_iters += ii.outer_iters;
    acc.level3_iters += ii.inner_iters + ii.level3_iters;
    return MSP_OK;
  };
  auto wait = [&]() -> msp_status {
    MSP_CHECK_HIP(hipStreamSynchronize(st));
    return MSP_OK;
  };
  // c = A^T b; r = c, x = 0
  MSP_CHECK_HIP(transpose_op(st, A, a_t, n, d, lda, B, ldb, w.c, k, w));
  acc.sweeps += 1;
  acc.sweep_bytes += abytes;
  MSP_CHECK_HIP(fcg_init(st, w.S, d, w.c, d, w.r, w.x, nullptr, mirror));
  LTRY(prec(w.r, w.z));
  MSP_CHECK_HIP(fcg_first_dir(st, w.S, d, w.r, w.z, w.p));
  int it = 0;
  while (true) {
    LTRY(wait());
    if (host[0] == 0) {
      // confirm on the recomputed residual c - A^T A x
      MSP_CHECK_HIP(normal_op(st, A, a_t, n, d, lda, w.x, w.q, k, nullptr, w));
      acc.sweeps += 2;
      acc.sweep_bytes += 2 * abytes;
      MSP_CHECK_HIP(launch_axpby(st, d, k, 1.0, w.c, d, -1.0, w.q, d, w.q, d, nullptr));
      MSP_CHECK_HIP(fcg_confirm(st, w.S, d, w.q, w.r, o.tol, w.dots, mirror));
      LTRY(wait());
      if (host[0] == 0 || it >= o.max_outer) break;
      acc.restarts += 1;
      LTRY(prec(w.r, w.z));
      MSP_CHECK_HIP(fcg_first_dir(st, w.S, d, w.r, w.z, w.p));
      continue;
    }
    if (it >= o.max_outer) break;
    MSP_CHECK_HIP(normal_op(st, A, a_t, n, d, lda, w.p, w.q, k, w.S.done, w));
    acc.sweeps += 2;
    acc.sweep_bytes += 2 * abytes;
    MSP_CHECK_HIP(fcg_alpha_dot(st, w.S, d, w.p, w.q));
    MSP_CHECK_HIP(fcg_update(st, w.S, d, w.x, w.r, w.ro, w.p, w.q, o.tol, o.max_outer, mirror));
    LTRY(prec(w.r, w.z));
    MSP_CHECK_HIP(fcg_direction(st, w.S, d, w.r, w.ro, w.z, w.p));
    ++it;
  }
  acc.outer_iters = host[1];
  // FP64 normal-equation residual of the returned x: |A^T (b - A x)| / |A^T b|
  MSP_CHECK_HIP(normal_op(st, A, a_t, n, d, lda, w.x, w.q, k, nullptr, w));
  MSP_CHECK_HIP(launch_axpby(st, d, k, 1.0, w.c, d, -1.0, w.q, d, w.q, d, nullptr));
  MSP_CHECK_HIP(launch_coldots(st, d, k, w.q, d, w.q, d, w.dots));
  MSP_CHECK_HIP(launch_coldots(st, d, k, w.c, d, w.c, d, w.dots + k));
  MSP_CHECK_HIP(launch_copy_block(st, d, k, w.x, d, X, ldx));
  std::vector<double> dv(2 * k);
  MSP_CHECK_HIP(hipMemcpyAsync(dv.data(), w.dots, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, st));
  LTRY(wait());
  double worst = 0.0;
  for (int64_t j = 0; j < k; ++j) {
    const double rel = dv[k + j] > 0.0 ? std::sqrt(dv[j] / dv[k + j]) : 0.0;
    worst = std::max(worst, std::isfinite(rel) ? rel : INFINITY);
  }
  acc.rel_residual_max = worst;
  acc.status = !std::isfinite(worst) ? MSP_ERR_NONFINITE : (worst <= o.tol ? MSP_OK : MSP_ERR_NO_CONVERGENCE);
  if (info) *info = acc;
  if (acc.status == MSP_ERR_NONFINITE) return msp_fail(MSP_ERR_NONFINITE, "non-finite residual");
  if (acc.status == MSP_ERR_NO_CONVERGENCE)
    return msp_fail(MSP_ERR_NO_CONVERGENCE, "tolerance not reached (relative residual %.3e)", worst);
  return MSP_OK;
}
