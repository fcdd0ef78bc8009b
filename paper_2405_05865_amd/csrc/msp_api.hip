// Host side of libmsp: argument validation, workspace layout, and the level loops of
// Multi-level Sketched Preconditioning that enqueue the kernels of k_*.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "msp_internal.h"

// ------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------
static thread_local char g_err[512] = "";

msp_status msp_fail(msp_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

msp_status msp_fail_hip(hipError_t e, const char* what, const char* file, int line) {
  snprintf(g_err, sizeof g_err, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  return MSP_ERR_HIP;
}

extern "C" const char* msp_last_error(void) { return g_err; }
extern "C" const char* msp_version(void) { return "libmsp 0.1 (gfx950)"; }

#define REQUIRE(cond, ...)                                   \
  do {                                                       \
    if (!(cond)) return msp_fail(MSP_ERR_INVALID_ARG, __VA_ARGS__); \
  } while (0)

#define TRY(expr)                         \
  do {                                    \
    msp_status _s = (expr);               \
    if (_s != MSP_OK) return _s;          \
  } while (0)


namespace {

size_t dsize(msp_dtype t) { return t == MSP_F64 ? 8 : (t == MSP_F32 ? 4 : 2); }
bool valid_dtype(int t) { return t == MSP_F64 || t == MSP_F32 || t == MSP_BF16; }
bool isfin(double v) { return std::isfinite(v); }
double wall_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kMaxGammaDraw = 32;

// MSP_LOG=1 in the environment: one progress line per refinement step, per level-1
// restart and per quadrature node, on stderr
bool log_on() {
  static int on = -1;
  if (on < 0) {
    const char* e = getenv("MSP_LOG");
    on = (e && e[0] && e[0] != '0') ? 1 : 0;
  }
  return on == 1;
}
constexpr int64_t kMaxS = 2048;    // tall-kernel register layout bound (32 columns per lane)
constexpr int64_t kMaxK = 1024;

// host mirror slots (pinned, mapped): [level*4 + 0] active count
enum { SLOT_L1 = 0, SLOT_L2 = 4, SLOT_L3 = 8, SLOT_L3B = 12, SLOT_L0 = 16 };

// ------------------------------------------------------------------------------------
// Sketch workspace layout
// ------------------------------------------------------------------------------------
struct SketchWs {
  BucketLists b;
  void* scratch;
};
SketchWs carve_sketch(WsCarver& w, int64_t n, int64_t s, int32_t gamma) {
  SketchWs o;
  o.b.offsets = w.take<int32_t>(s + 1);
  o.b.entries = w.take<int32_t>(n * gamma);
  o.scratch = w.take<char>(bucket_scratch_bytes(n, s, gamma));
  return o;
}

// ------------------------------------------------------------------------------------
// Nystrom workspace layout
// ------------------------------------------------------------------------------------
struct NysWs {
  double *Wm, *G, *Minv, *Minv2, *tmp, *small, *gpart, *scal;
  double *est_w, *est_c, *est_part;  // PSD: the lam0 estimator's W^{-1}, C^T C, Gram partials
  int32_t* status;
  int32_t* phi_rows;
  int8_t* phi_signs;
  SketchWs sk_S, sk_Phi;
};
NysWs carve_nystrom(WsCarver& w, msp_structure st, int64_t m, int64_t n, int64_t s, int64_t phi, int32_t phi_gamma) {
  NysWs o{};
  const int64_t rows = (st == MSP_SYM_PSD) ? n : m;
  o.scal = w.take<double>(16);
  o.status = w.take<int32_t>(16);
  o.G = w.take<double>(s * s);
  o.Minv = w.take<double>(s * s);
  o.tmp = w.take<double>(s * s);
  if (st == MSP_SYM_PSD) {
    o.Wm = w.take<double>(s * s);
    o.Minv2 = nullptr;
    o.est_w = w.take<double>(s * s);
    o.est_c = w.take<double>(s * s);
    o.est_part = w.take<double>((size_t)gram_splits(n, s) * s * s + 1);
  } else {
    o.Wm = nullptr;
    o.Minv2 = w.take<double>(s * s);
  }
  o.small = w.take<double>(phi * s);
  o.gpart = w.take<double>((size_t)gram_splits(phi, s) * s * s);
  o.phi_rows = w.take<int32_t>(rows * phi_gamma);
  o.phi_signs = w.take<int8_t>(rows * phi_gamma);
  o.sk_Phi = carve_sketch(w, rows, phi, phi_gamma);
  return o;
}

}  // namespace

// ====================================================================================
// msp_sketch
// ====================================================================================
// msp_sketch's scratch: the tile-major lists of S
TileLists carve_apply_lists(WsCarver& w, int64_t n, int64_t s, int32_t gamma) {
  int32_t* base = w.take<int32_t>(tile_lists_ints(n, s, gamma));
  return carve_tile_lists(base, n, s, gamma);
}

extern "C" msp_status msp_sketch_workspace(int64_t m, int64_t n, int64_t s, int32_t gamma, size_t* bytes) {
  REQUIRE(bytes, "bytes is null");
  REQUIRE(m >= 1 && n >= 1 && s >= 1 && gamma >= 1 && gamma <= s && gamma <= kMaxGammaDraw && s <= n,
          "invalid sizes m=%lld n=%lld s=%lld gamma=%d", (long long)m, (long long)n, (long long)s, gamma);
  WsCarver w(nullptr, 0);
  carve_apply_lists(w, n, s, gamma);
  *bytes = w.off;
  return MSP_OK;
}

extern "C" msp_status msp_sketch(void* stream, const void* A, msp_dtype a_t, int64_t m, int64_t n, int64_t lda,
                                 int64_t s, int32_t gamma, uint64_t seed, int32_t* S_rows, int8_t* S_signs, void* Y,
                                 msp_dtype y_t, int64_t ldy, void* ws, size_t ws_bytes) {
  REQUIRE(A && S_rows && S_signs && Y && ws, "null pointer argument");
  REQUIRE(valid_dtype(a_t) && (y_t == MSP_F64 || y_t == MSP_F32), "unsupported dtype");
  REQUIRE(!(y_t == MSP_F64 && a_t != MSP_F64), "F64 Y requires F64 A");
  REQUIRE(!(y_t == MSP_F32 && a_t == MSP_F64), "F32 Y requires F32 or BF16 A");
  REQUIRE(m >= 1 && n >= 1 && lda >= n && s >= 1 && s <= n && ldy >= s, "invalid sizes or leading dimensions");
  REQUIRE(gamma >= 1 && gamma <= s && gamma <= kMaxGammaDraw, "need 1 <= gamma <= min(s, 32)");
  REQUIRE(n * gamma < (int64_t(1) << 30), "n * gamma too large");
  REQUIRE(s <= kMaxS, "s > %lld unsupported", (long long)kMaxS);
  size_t need = 0;
  TRY(msp_sketch_workspace(m, n, s, gamma, &need));
  if (ws_bytes < need || ((uintptr_t)ws & 255)) return msp_fail(MSP_ERR_WORKSPACE, "sketch workspace needs %zu bytes, 256-B aligned", need);
  hipStream_t st = (hipStream_t)stream;
  WsCarver w(ws, ws_bytes);
  const TileLists L = carve_apply_lists(w, n, s, gamma);
  MSP_CHECK_HIP(launch_sketch_gen(st, seed, n, s, gamma, S_rows, S_signs));
  MSP_CHECK_HIP(build_tile_lists(st, S_rows, S_signs, n, s, gamma, L));
  const double scale = 1.0 / std::sqrt((double)gamma);
  MSP_CHECK_HIP(launch_sketch_apply(st, A, a_t, m, n, lda, s, L, scale, Y, y_t, ldy, sketch_rows_choice(a_t, m, n, lda, s, gamma)));
  return MSP_OK;
}

extern "C" msp_status msp_sketch_autotune(void* stream, const void* A, msp_dtype a_t, int64_t m, int64_t n,
                                          int64_t lda, int64_t s, int32_t gamma, uint64_t seed, int32_t* S_rows,
                                          int8_t* S_signs, void* Y, msp_dtype y_t, int64_t ldy, void* ws,
                                          size_t ws_bytes, int32_t* rows_per_block) {
  TRY(msp_sketch(stream, A, a_t, m, n, lda, s, gamma, seed, S_rows, S_signs, Y, y_t, ldy, ws, ws_bytes));
  hipStream_t st = (hipStream_t)stream;
  WsCarver w(ws, ws_bytes);
  const TileLists L = carve_apply_lists(w, n, s, gamma);
  int R = 0;
  MSP_CHECK_HIP(tune_sketch_apply(st, A, a_t, m, n, lda, s, gamma, L, Y, y_t, ldy, &R));
  // Y once more with the chosen shape (the timings overwrote it)
  MSP_CHECK_HIP(launch_sketch_apply(st, A, a_t, m, n, lda, s, L, 1.0 / std::sqrt((double)gamma), Y, y_t, ldy, R));
  if (rows_per_block) *rows_per_block = R;
  return MSP_OK;
}

// ====================================================================================
// msp_nystrom
// ====================================================================================
namespace {
size_t nystrom_bytes(msp_structure st, int64_t m, int64_t n, int64_t s, int64_t phi, int32_t phi_gamma,
                     int32_t gamma) {
  WsCarver w(nullptr, 0);
  NysWs o = carve_nystrom(w, st, m, n, s, phi, phi_gamma);
  (void)o;
  if (st == MSP_SYM_PSD) carve_sketch(w, n, s, gamma);  // bucket lists of S
  return w.off;
}

msp_status refactor(hipStream_t st, msp_precond* P) {
  const int64_t s = P->s;
  MSP_CHECK_HIP(hipMemsetAsync(P->status, 0, sizeof(int32_t), st));
  if (P->structure == MSP_SYM_PSD) {
    // M2 = C~^T C~ + lam~ W, then its inverse
    MSP_CHECK_HIP(launch_combine_sym(st, s, 1.0, P->G, P->lt, P->Wm, 0.0, P->Minv));
    MSP_CHECK_HIP(spd_inverse(st, s, P->Minv, P->tmp, P->shift_rel, P->scal, P->status));
  } else {
    // M3b = M3a + lam~ I
    MSP_CHECK_HIP(launch_combine_sym(st, s, 1.0, P->G, 0.0, nullptr, P->lt, P->Minv2));
    MSP_CHECK_HIP(spd_inverse(st, s, P->Minv2, P->tmp, P->shift_rel, P->scal, P->status));
  }
  int32_t h = 0;
  MSP_CHECK_HIP(hipMemcpyAsync(&h, P->status, sizeof h, hipMemcpyDeviceToHost, st));
  MSP_CHECK_HIP(hipStreamSynchronize(st));
  if (h != 0) return msp_fail(MSP_ERR_NOT_POSDEF, "inner-level preconditioner is not positive definite");
  return MSP_OK;
}
}  // namespace

namespace {
// lam0 when the caller has no tail spectrum (lambda0 < 0; reading of the lam0 of Theorem
// 4.1): (2/l) max(tr A - tr(W^+ C^T C), 0), l = s/2. tr(W^+ C^T C) is the trace of the
// Nystrom approximation C W^+ C^T of Algorithm 1; A minus it is PSD with the approximation
// of rank <= s, so the deficit is at least sum_{i>s} lambda_i, and 0 when rank(A) <= s.
// W^+ is taken as (W + mu I)^{-1}, mu = 1e-9 tr(W)/s: C (W + mu I)^{-1} C^T is still below A
// and of rank <= s, and mu keeps the directions in which a rank-deficient W is zero up to
// rounding from being amplified.
constexpr double kLambda0Shift = 1e-9;
msp_status estimate_lambda0(hipStream_t st, msp_precond* H, const NysWs& o, const void* A, msp_dtype a_t,
                            int64_t lda) {
  const int64_t n = H->n, s = H->s;
  MSP_CHECK_HIP(launch_combine_sym(st, s, 1.0, H->Wm, 0.0, nullptr, 0.0, o.est_w));
  MSP_CHECK_HIP(hipMemsetAsync(o.status, 0, sizeof(int32_t), st));
  MSP_CHECK_HIP(spd_inverse(st, s, o.est_w, o.tmp, kLambda0Shift, o.scal + 8, o.status));
  const int sp = gram_splits(n, s);
  if (H->y_t == MSP_F64)
    MSP_CHECK_HIP(launch_gram(st, (const double*)H->Y, n, s, H->ldy, o.est_c, o.est_part, sp));
  else
    MSP_CHECK_HIP(launch_gram_f32(st, (const float*)H->Y, n, s, H->ldy, o.est_c, o.est_part, sp));
  MSP_CHECK_HIP(launch_diag_sum(st, A, a_t, n, lda, o.scal));
  MSP_CHECK_HIP(launch_lambda0_est(st, o.est_w, o.est_c, s, 0.5 * (double)s, o.scal));
  double v[3] = {0, 0, 0};
  int32_t bad = 0;
  MSP_CHECK_HIP(hipMemcpyAsync(v, o.scal, sizeof v, hipMemcpyDeviceToHost, st));
  MSP_CHECK_HIP(hipMemcpyAsync(&bad, o.status, sizeof bad, hipMemcpyDeviceToHost, st));
  MSP_CHECK_HIP(hipStreamSynchronize(st));
  if (bad) return msp_fail(MSP_ERR_NOT_POSDEF, "W = S C is not positive definite (lambda0 estimator)");
  if (!isfin(v[2])) return msp_fail(MSP_ERR_NONFINITE, "lambda0 estimate not finite");
  if (!(H->lam + v[2] > 0.0))
    return msp_fail(MSP_ERR_INVALID_ARG,
                    "estimated lambda0 is 0 (the sketch recovers A exactly); pass lambda > 0 or lambda0 > 0");
  H->lam0 = v[2];
  H->lt = H->lam + v[2];
  H->trace_a = v[0];
  H->trace_nys = v[1];
  return MSP_OK;
}
}  // namespace

extern "C" msp_status msp_precond_params(const msp_precond* P, double* lambda, double* lambda0) {
  REQUIRE(P, "P is null");
  if (lambda) *lambda = P->lam;
  if (lambda0) *lambda0 = P->lam0;
  return MSP_OK;
}

extern "C" msp_status msp_nystrom_workspace(msp_structure structure, int64_t m, int64_t n, int64_t s, int64_t phi,
                                            int32_t phi_gamma, size_t* bytes) {
  REQUIRE(bytes, "bytes is null");
  REQUIRE(structure == MSP_SYM_PSD || structure == MSP_GENERAL, "bad structure");
  REQUIRE(m >= 1 && n >= 1 && s >= 1 && phi >= 1 && phi_gamma >= 1 && phi_gamma <= phi &&
              phi_gamma <= kMaxGammaDraw,
          "invalid sizes");
  *bytes = nystrom_bytes(structure, m, n, s, phi, phi_gamma, kMaxGammaDraw);
  return MSP_OK;
}

extern "C" msp_status msp_nystrom(void* stream, msp_structure structure, int64_t m, int64_t n, int64_t s,
                                  int32_t gamma, const int32_t* S_rows, const int8_t* S_signs, const void* Y,
                                  msp_dtype y_t, int64_t ldy, const void* A, msp_dtype a_t, int64_t lda,
                                  double lambda, double lambda0, int64_t phi, int32_t phi_gamma, uint64_t phi_seed,
                                  void* ws, size_t ws_bytes, msp_precond** P) {
  REQUIRE(P, "P is null");
  *P = nullptr;
  REQUIRE(structure == MSP_SYM_PSD || structure == MSP_GENERAL, "bad structure");
  REQUIRE(S_rows && S_signs && Y && ws, "null pointer argument");
  REQUIRE(y_t == MSP_F64 || y_t == MSP_F32, "Y must be F64 or F32");
  REQUIRE(m >= 1 && n >= 1 && s >= 1 && s <= n && ldy >= s && s <= kMaxS, "invalid sizes");
  REQUIRE(structure == MSP_GENERAL || m == n, "MSP_SYM_PSD needs m == n");
  REQUIRE(gamma >= 1 && gamma <= s && gamma <= kMaxGammaDraw, "invalid gamma");
  REQUIRE(phi >= 1 && phi_gamma >= 1 && phi_gamma <= phi && phi_gamma <= kMaxGammaDraw, "invalid phi/phi_gamma");
  const int64_t rows = structure == MSP_SYM_PSD ? n : m;
  REQUIRE(phi <= rows, "phi must not exceed the sketched dimension");
  REQUIRE(rows * phi_gamma < (int64_t(1) << 30) && n * gamma < (int64_t(1) << 30), "sizes too large");
  if (!isfin(lambda) || !isfin(lambda0)) return msp_fail(MSP_ERR_NONFINITE, "lambda/lambda0 not finite");
  const bool estimate = lambda0 < 0.0;
  if (estimate) {
    if (structure != MSP_SYM_PSD)
      return msp_fail(MSP_ERR_UNSUPPORTED, "the lambda0 estimator is for MSP_SYM_PSD handles; pass lambda0 >= 0");
    REQUIRE(A && valid_dtype(a_t) && lda >= n, "lambda0 < 0 (estimate) needs A (n x n, lda >= n)");
    REQUIRE(lambda >= 0.0, "need lambda >= 0");
  } else {
    REQUIRE(lambda >= 0.0 && lambda + lambda0 > 0.0, "need lambda, lambda0 >= 0 and lambda + lambda0 > 0");
  }
  const size_t need = nystrom_bytes(structure, m, n, s, phi, phi_gamma, gamma);
  if (ws_bytes < need || ((uintptr_t)ws & 255))
    return msp_fail(MSP_ERR_WORKSPACE, "nystrom workspace needs %zu bytes, 256-B aligned", need);

  hipStream_t st = (hipStream_t)stream;
  WsCarver w(ws, ws_bytes);
  NysWs o = carve_nystrom(w, structure, m, n, s, phi, phi_gamma);
  msp_precond* H = new msp_precond();
  H->structure = structure;
  H->m = m;
  H->n = n;
  H->s = s;
  H->phi = phi;
  H->gamma = gamma;
  H->phi_gamma = phi_gamma;
  H->S_rows = S_rows;
  H->S_signs = S_signs;
  H->Y = Y;
  H->y_t = y_t;
  H->ldy = ldy;
  H->lam = lambda;
  H->lam0 = lambda0;
  H->lt = lambda + lambda0;
  H->shift_rel = 1e-12;
  H->Wm = o.Wm;
  H->G = o.G;
  H->Minv = o.Minv;
  H->Minv2 = o.Minv2;
  H->tmp = o.tmp;
  H->scal = o.scal;
  H->status = o.status;
  (void)hipGetDevice(&H->device);
  if (hipHostMalloc((void**)&H->host_flags, 4096, hipHostMallocMapped) != hipSuccess) {
    delete H;
    return msp_fail(MSP_ERR_HIP, "pinned host allocation failed");
  }
  memset(H->host_flags, 0, 4096);
  if (hipHostGetDevicePointer((void**)&H->dev_view_flags, H->host_flags, 0) != hipSuccess) {
    (void)hipHostFree(H->host_flags);
    delete H;
    return msp_fail(MSP_ERR_HIP, "hipHostGetDevicePointer failed");
  }
  H->host_d = nullptr;
  H->events = new std::vector<hipEvent_t>();

  auto fail = [&](msp_status s_) {
    msp_precond_destroy(H);
    return s_;
  };
  const double sphi = 1.0 / std::sqrt((double)phi_gamma);
  if (structure == MSP_SYM_PSD) {
    // Algorithm 1: W = S C (bucket lists of S, then a row gather of C)
    SketchWs sk = carve_sketch(w, n, s, gamma);
    if (!w.ok()) return fail(msp_fail(MSP_ERR_WORKSPACE, "workspace overflow"));
    hipError_t e = build_buckets(st, S_rows, S_signs, n, s, gamma, sk.b, sk.scratch);
    if (e == hipSuccess) e = launch_gather_rows(st, Y, y_t, ldy, s, s, sk.b, 1.0 / std::sqrt((double)gamma), o.Wm, s);
    if (e == hipSuccess) e = launch_symmetrize(st, s, o.Wm);
    // Algorithm 1: C~ = Phi C, then C~^T C~
    if (e == hipSuccess) e = launch_sketch_gen(st, phi_seed, n, phi, phi_gamma, o.phi_rows, o.phi_signs);
    if (e == hipSuccess) e = build_buckets(st, o.phi_rows, o.phi_signs, n, phi, phi_gamma, o.sk_Phi.b, o.sk_Phi.scratch);
    if (e == hipSuccess) e = launch_gather_rows(st, Y, y_t, ldy, s, phi, o.sk_Phi.b, sphi, o.small, s);
    if (e == hipSuccess) e = launch_gram(st, o.small, phi, s, s, o.G, o.gpart, gram_splits(phi, s));
    if (e != hipSuccess) return fail(msp_fail_hip(e, "nystrom kernels", __FILE__, __LINE__));
    if (estimate) {
      msp_status r = estimate_lambda0(st, H, o, A, a_t, lda);
      if (r != MSP_OK) return fail(r);
    }
  } else {
    // Algorithm 3: A^ = Phi A~ over the m rows, M3a = A^^T A^
    hipError_t e = launch_sketch_gen(st, phi_seed, m, phi, phi_gamma, o.phi_rows, o.phi_signs);
    if (e == hipSuccess) e = build_buckets(st, o.phi_rows, o.phi_signs, m, phi, phi_gamma, o.sk_Phi.b, o.sk_Phi.scratch);
    if (e == hipSuccess) e = launch_gather_rows(st, Y, y_t, ldy, s, phi, o.sk_Phi.b, sphi, o.small, s);
    if (e == hipSuccess) e = launch_gram(st, o.small, phi, s, s, o.G, o.gpart, gram_splits(phi, s));
    if (e == hipSuccess) e = launch_combine_sym(st, s, 1.0, o.G, 0.0, nullptr, 0.0, o.Minv);
    if (e == hipSuccess) e = hipMemsetAsync(o.status, 0, sizeof(int32_t), st);
    if (e == hipSuccess) e = spd_inverse(st, s, o.Minv, o.tmp, H->shift_rel, o.scal, o.status);
    if (e != hipSuccess) return fail(msp_fail_hip(e, "nystrom kernels", __FILE__, __LINE__));
    int32_t h = 0;
    if (hipMemcpyAsync(&h, o.status, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(msp_fail(MSP_ERR_HIP, "sync failed"));
    if (h != 0) return fail(msp_fail(MSP_ERR_NOT_POSDEF, "M3a is not positive definite"));
  }
  msp_status r = refactor(st, H);
  if (r != MSP_OK) return fail(r);
  *P = H;
  return MSP_OK;
}

extern "C" msp_status msp_precond_destroy(msp_precond* P) {
  if (!P) return MSP_OK;
  if (P->host_flags) (void)hipHostFree(P->host_flags);
  if (P->events) {
    auto* v = (std::vector<hipEvent_t>*)P->events;
    for (hipEvent_t e : *v) (void)hipEventDestroy(e);
    delete v;
  }
  delete P;
  return MSP_OK;
}

extern "C" msp_status msp_precond_factors(void* stream, const msp_precond* P, double* W, double* Minv,
                                          double* Minv2) {
  REQUIRE(P, "P is null");
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = sizeof(double) * P->s * P->s;
  if (W && P->Wm) MSP_CHECK_HIP(hipMemcpyAsync(W, P->Wm, bytes, hipMemcpyDeviceToDevice, st));
  if (Minv) MSP_CHECK_HIP(hipMemcpyAsync(Minv, P->Minv, bytes, hipMemcpyDeviceToDevice, st));
  if (Minv2 && P->Minv2) MSP_CHECK_HIP(hipMemcpyAsync(Minv2, P->Minv2, bytes, hipMemcpyDeviceToDevice, st));
  return MSP_OK;
}

extern "C" msp_status msp_precond_set_lambda(void* stream, msp_precond* P, double lambda) {
  REQUIRE(P, "P is null");
  if (!isfin(lambda)) return msp_fail(MSP_ERR_NONFINITE, "lambda not finite");
  REQUIRE(lambda >= 0.0 && lambda + P->lam0 > 0.0, "need lambda >= 0 and lambda + lambda0 > 0");
  P->lam = lambda;
  P->lt = lambda + P->lam0;
  return refactor((hipStream_t)stream, P);
}

// ====================================================================================
// msp_solve
// ====================================================================================
extern "C" void msp_solve_opts_default(msp_solve_opts* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->max_outer = 5000;
  o->inner_tol = 1e-10;
  o->max_inner = 200;
  o->level3_tol = 1e-10;
  o->max_level3 = 200;
  o->normal = 0;
  o->refine = 0;
  o->refine_inner_tol = 1e-4;
  o->max_refine = 30;
  o->profile = 0;
  o->level2_form = 1;
  o->sym_sweep = 1;
  o->use_graph = 0;
  o->batch_teams = 1;
  o->autotune = 0;
  o->level3_kernels = 2;
}


namespace {

struct Level {
  int64_t len = 0, k = 0;
  double *x = nullptr, *r = nullptr, *ro = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  FcgState S{};
};

Level carve_level(WsCarver& w, int64_t len, int64_t k, int64_t state_len = 0) {
  Level L;
  L.len = len;
  L.k = k;
  L.x = w.take<double>(len * k);
  L.r = w.take<double>(len * k);
  L.ro = w.take<double>(len * k);
  L.z = w.take<double>(len * k);
  L.p = w.take<double>(len * k);
  L.q = w.take<double>(len * k);
  L.S = carve_fcg_state(w, std::max(len, state_len), k);
  return L;
}

// instantiated graphs of inner-step chunks, per (chunk length, operator, output): captured
// once on a private stream and replayed on the solve's stream for every SolveM1 call
struct StepGraphs {
  hipStream_t st = nullptr;   // the solve's stream (synchronised before destruction)
  hipStream_t cap = nullptr;  // capture stream
  std::map<std::tuple<int, const void*, const void*, const void*>, hipGraphExec_t> exec;
  ~StepGraphs() {
    if (!exec.empty() && st) (void)hipStreamSynchronize(st);
    for (auto& e : exec) (void)hipGraphExecDestroy(e.second);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

struct SolveCtx {
  hipStream_t st;
  const msp_precond* P;
  const msp_solve_opts* o;
  int64_t n, m, s, k;
  const void* A_sw;  // matrix swept inside MSP
  msp_dtype sw_t;
  // general path on an FP32-stored A_sw: its sweeps accumulate in FP64, since the
  // normal-equation operator A^T A squares A's condition number and FP32 sums would
  // bury its smallest directions
  bool sw64 = false;
  int sweep_nseg = 0;  // segments of the level-1 block sweep over A_sw (0: built-in rule)
  const void* A_cf;  // matrix of the confirmation / refinement residuals (FP64 arithmetic)
  msp_dtype cf_t;
  int64_t lda;
  double lam;
  double lam_sw;  // shift of the sweeps of A_sw (lam, plus delta under PSD refinement)
  Level L0, L1, L2, L3;
  double *rhs2, *wp, *pqw, *tmp_s, *relres, *dots, *gpart, *l2part, *l2pq, *l2b;
  double *rho, *tvec, *mvec, *mvec2, *nvec;  // general path: m x k (4) and n x k
  double *xh, *rh, *bn;                      // refinement
  int form = 0;                              // level2_form
  double *H2 = nullptr, *H3 = nullptr;       // explicit inner operators (s x s)
  double *B2t = nullptr, *Act = nullptr;     // general: (A^T A~)^T (s x n), A~^T (s x m)
  double* gtmp = nullptr;                    // Gram split partials
  double *Htmp = nullptr, *Hscal = nullptr;  // level2_form 2: inverse scratch
  int32_t* Hstat = nullptr;
  double* sympart = nullptr;                 // row/column partials of the lower-triangle sweep
  double* gemmpart = nullptr;                // segment partials of the level-1 block sweep
  size_t gemmpart_n = 0;
  // explicit operators with k <= kL2xMaxK: one kernel per inner step through G = H Minv
  bool use_x = false;
  L2xArgs X{};
  double* G2 = nullptr;                      // PSD: H2 M2^{-1}
  // general level 3 under level2_form 1 with k <= kL2fMaxK: two kernels per step
  bool use_f = false;
  L2fArgs F{};
  int32_t* hf;
  int32_t* df;
  int last_inner = 4, last_l3a = 4, last_l3b = 4;
  int nb_last = 0;
  msp_solve_info acc{};
  StepGraphs graphs;
  std::vector<hipEvent_t>* evpool = nullptr;
  size_t evused = 0;
};

size_t solve_layout(WsCarver& w, const msp_precond* P, int64_t k, SolveCtx* c, int form, int sym, int l3k) {
  const int64_t n = P->n, m = P->m, s = P->s;
  const int64_t mx = std::max(n, m);
  const int64_t nb_gemv = (mx + 3) / 4;  // upper bound of gemv blocks (R >= 4)
  Level L0 = carve_level(w, n, k, mx);
  Level L1 = carve_level(w, n, k, mx);
  Level L2 = carve_level(w, s, k);
  Level L3 = carve_level(w, s, k);
  double* rhs2 = w.take<double>(s * k);
  double* wp = w.take<double>(s * k);
  double* pqw = w.take<double>(s * k);
  double* tmp_s = w.take<double>(s * k);
  double* relres = w.take<double>(k);
  double* dots = w.take<double>(4 * k);
  double* gpart = w.take<double>(std::max<size_t>(nb_gemv * k, gemv_t_part_doubles(m, n, k)));
  double* l2part = w.take<double>(l2_op_part_doubles(mx, s, k));
  double* l2pq = w.take<double>(l2_op_pq_doubles(mx, k));
  double* l2b = w.take<double>(l2_bpart_doubles(s, k));
  double *rho = nullptr, *tvec = nullptr, *mvec = nullptr, *mvec2 = nullptr, *nvec = nullptr;
  if (P->structure == MSP_GENERAL) {
    rho = w.take<double>(m * k);
    tvec = w.take<double>(m * k);
    mvec = w.take<double>(m * k);
    mvec2 = w.take<double>(m * k);
    nvec = w.take<double>(n * k);
  }
  double* xh = w.take<double>(n * k);
  double* rh = w.take<double>(mx * k);
  double* bn = w.take<double>(k);
  double *H2 = nullptr, *H3 = nullptr, *B2t = nullptr, *Act = nullptr, *gtmp = nullptr;
  double *Htmp = nullptr, *Hscal = nullptr;
  int32_t* Hstat = nullptr;
  if (form == 2) {
    Htmp = w.take<double>(s * s);
    Hscal = w.take<double>(4);
    Hstat = w.take<int32_t>(4);
  }
  if (form >= 1) {
    H2 = w.take<double>(s * s);
    if (P->structure == MSP_SYM_PSD) {
      gtmp = w.take<double>((size_t)gram_splits(n, s) * s * s + 1);
    } else {
      H3 = w.take<double>(s * s);
      B2t = w.take<double>(s * n);
      Act = w.take<double>(s * m);
      gtmp = w.take<double>(gemm_t_part_doubles(m, n, s));
    }
  }
  // the one-kernel inner step (level2_form 1, block of at most kL2xMaxK columns). PSD only:
  // the step carries u = H p by the recurrence u_t = G r_t + beta u_{t-1} with G = H M^{-1},
  // which is exact in exact arithmetic but drifts from H p when H and M are as
  // ill-conditioned as the general level-3 matrices (A~^T A~ with kappa(A)^2 spread): there
  // the recurrence iterate stalls near 1e-4 relative error where direct products reach
  // 1e-7, and the outer levels take about three times the oracle's steps
  const bool use_x = form == 1 && P->structure == MSP_SYM_PSD && s >= kGemmMinK && s <= kL2xMaxS && k <= kL2xMaxK;
  L2xArgs X{};
  double* G2 = nullptr;
  if (use_x) {
    X = l2x_carve(w, s, k);
    G2 = w.take<double>(s * s);
  }
  // the general level 3 as two kernels per step (level2_form 1, at most kL2fMaxK columns)
  const bool use_f = form == 1 && P->structure == MSP_GENERAL && l3k == 2 && k <= kL2fMaxK && s <= kL2fMaxS;
  L2fArgs F{};
  if (use_f) F = l2f_carve(w, s, k);
  // the lower-triangle level-1 sweep (PSD, one right-hand side)
  double* sympart = nullptr;
  if (sym && P->structure == MSP_SYM_PSD && k == 1) sympart = w.take<double>(symv_part_doubles(n));
  double* gemmpart = nullptr;
  const size_t gemmpart_n = k >= kGemmMinK ? gemm_split_doubles(mx, k) : 0;
  if (gemmpart_n) gemmpart = w.take<double>(gemmpart_n);
  if (c) {
    c->sympart = sympart;
    c->gemmpart = gemmpart;
    c->gemmpart_n = gemmpart_n;
    c->use_x = use_x;
    c->X = X;
    c->use_f = use_f;
    c->F = F;
    c->G2 = G2;
    c->Htmp = Htmp;
    c->Hscal = Hscal;
    c->Hstat = Hstat;
    c->form = form;
    c->H2 = H2;
    c->H3 = H3;
    c->B2t = B2t;
    c->Act = Act;
    c->gtmp = gtmp;
    c->L0 = L0;
    c->L1 = L1;
    c->L2 = L2;
    c->L3 = L3;
    c->rhs2 = rhs2;
    c->wp = wp;
    c->pqw = pqw;
    c->tmp_s = tmp_s;
    c->relres = relres;
    c->dots = dots;
    c->gpart = gpart;
    c->l2part = l2part;
    c->l2pq = l2pq;
    c->l2b = l2b;
    c->rho = rho;
    c->tvec = tvec;
    c->mvec = mvec;
    c->mvec2 = mvec2;
    c->nvec = nvec;
    c->xh = xh;
    c->rh = rh;
    c->bn = bn;
  }
  return w.off;
}

inline volatile int32_t* slot(SolveCtx& c, int i) { return (volatile int32_t*)(c.hf + i); }

msp_status sync(SolveCtx& c) {
  MSP_CHECK_HIP(hipStreamSynchronize(c.st));
  return MSP_OK;
}

// profiled sweeps: an event pair around each level-1 sweep launch
msp_status ev_begin(SolveCtx& c, hipEvent_t* stop_out) {
  *stop_out = nullptr;
  if (!c.o->profile || !c.evpool) return MSP_OK;
  auto& pool = *c.evpool;
  while (pool.size() < c.evused + 2) {
    hipEvent_t e;
    MSP_CHECK_HIP(hipEventCreate(&e));
    pool.push_back(e);
  }
  MSP_CHECK_HIP(hipEventRecord(pool[c.evused], c.st));
  *stop_out = pool[c.evused + 1];
  c.evused += 2;
  return MSP_OK;
}

msp_status ev_collect(SolveCtx& c) {
  if (!c.o->profile || !c.evpool || c.evused == 0) return MSP_OK;
  MSP_CHECK_HIP(hipStreamSynchronize(c.st));
  double total = 0.0;
  for (size_t i = 0; i + 1 < c.evused; i += 2) {
    float ms = 0.f;
    MSP_CHECK_HIP(hipEventElapsedTime(&ms, (*c.evpool)[i], (*c.evpool)[i + 1]));
    total += ms;
  }
  c.acc.sweep_ms += total;
  c.acc.timed_sweeps += (int64_t)(c.evused / 2);
  c.evused = 0;
  return MSP_OK;
}

// Y = A X (+ lam X on the diagonal) for A rows x cols; fp64 forces FP64 arithmetic on
// FP32 storage (residuals); timed marks a level-1 sweep for the profile
msp_status sweep(SolveCtx& c, const void* A, msp_dtype t, int64_t rows, int64_t cols, const double* X, int64_t ldx,
                 double* Y, int64_t ldy, bool diag, const int32_t* skip, bool parts, bool fp64, bool timed) {
  int nb = 0;
  hipEvent_t stop = nullptr;
  if (timed) TRY(ev_begin(c, &stop));
  hipError_t e;
  const double lam = (A == c.A_sw) ? c.lam_sw : c.lam;
  fp64 = fp64 || (c.sw64 && A == c.A_sw);
  // the level-1 operator of a symmetric A from its lower triangle
  const bool sym = c.sympart && A == c.A_sw && !fp64 && rows == cols && symv_supported(A, t, c.lda, c.k);
  if (sym)
    e = launch_symv(c.st, A, t, rows, c.lda, X, Y, lam, diag, skip, c.sympart, parts ? c.gpart : nullptr, &nb);
  else if (c.k >= kGemmMinK)
    e = launch_gemm_split(c.st, A, t, fp64 && t == MSP_F32, rows, cols, c.lda, X, ldx, Y, ldy, c.k, lam, diag, skip,
                          parts ? c.gpart : nullptr, &nb, c.gemmpart, c.gemmpart_n, A == c.A_sw ? c.sweep_nseg : 0);
  else if (fp64 && t == MSP_F32)
    e = launch_gemv_f32_as_f64(c.st, (const float*)A, rows, cols, c.lda, X, ldx, Y, ldy, c.k, lam, diag, skip,
                               parts ? c.gpart : nullptr, &nb);
  else
    e = launch_gemv(c.st, A, t, rows, cols, c.lda, X, ldx, Y, ldy, c.k, lam, diag, skip, parts ? c.gpart : nullptr,
                    &nb);
  MSP_CHECK_HIP(e);
  if (stop) MSP_CHECK_HIP(hipEventRecord(stop, c.st));
  c.nb_last = nb;
  c.acc.sweeps += 1;
  c.acc.sweep_bytes += (sym ? 0.5 * (double)rows * (double)(rows + 1) : (double)rows * (double)cols) * (double)dsize(t);
  return MSP_OK;
}

// Y = A^T X for A rows x cols (X length rows, Y length cols)
msp_status sweep_t(SolveCtx& c, const void* A, msp_dtype t, int64_t rows, int64_t cols, const double* X, int64_t ldx,
                   double* Y, int64_t ldy, const int32_t* skip) {
  if (c.sw64 && A == c.A_sw && t == MSP_F32)
    MSP_CHECK_HIP((c.k >= kGemmMinK ? launch_gemm_t_f32_as_f64 : launch_gemv_t_f32_as_f64)(
        c.st, (const float*)A, rows, cols, c.lda, X, ldx, Y, ldy, c.k, skip, c.gpart));
  else if (c.k >= kGemmMinK)
    MSP_CHECK_HIP(launch_gemm_t(c.st, A, t, rows, cols, c.lda, X, ldx, Y, ldy, c.k, skip, c.gpart));
  else
    MSP_CHECK_HIP(launch_gemv_t(c.st, A, t, rows, cols, c.lda, X, ldx, Y, ldy, c.k, skip, c.gpart));
  c.acc.sweeps += 1;
  c.acc.sweep_bytes += (double)rows * (double)cols * (double)dsize(t);
  return MSP_OK;
}

// Y = A^T X in FP64 arithmetic whatever A's storage (the residuals of the normal equations)
hipError_t sweep_t64(SolveCtx& c, const void* A, msp_dtype t, int64_t rows, int64_t cols, const double* X,
                     int64_t ldx, double* Y, int64_t ldy) {
  if (t == MSP_F32)
    return (c.k >= kGemmMinK ? launch_gemm_t_f32_as_f64 : launch_gemv_t_f32_as_f64)(
        c.st, (const float*)A, rows, cols, c.lda, X, ldx, Y, ldy, c.k, nullptr, c.gpart);
  return (c.k >= kGemmMinK ? launch_gemm_t : launch_gemv_t)(c.st, A, t, rows, cols, c.lda, X, ldx, Y, ldy, c.k,
                                                            nullptr, c.gpart);
}

L2Step l2step_for(SolveCtx& c, Level& L, const double* Minv, const double* W, double wscale, double sigma,
                  double tol, int max_iter, int slotid, const int32_t* parent_done) {
  L2Step a;
  a.s = c.s;
  a.k = c.k;
  a.nbC = l2_blocks(std::max(c.n, c.m));
  a.part = c.l2part;
  a.pqpart = c.l2pq;
  a.wp = W ? c.wp : nullptr;
  a.pqw = W ? c.pqw : nullptr;
  a.wscale = wscale;
  a.sigma = sigma;
  a.y = L.x;
  a.r = L.r;
  a.ro = L.ro;
  a.z = L.z;
  a.p = L.p;
  a.q = L.q;
  a.Minv = Minv;
  a.S = L.S;
  a.bpart = c.l2b;
  a.tol = tol;
  a.max_iter = max_iter;
  a.mirror = c.df + slotid;
  a.parent_done = parent_done;
  a.gscratch = c.gemmpart;
  a.gscratch_n = c.gemmpart_n;
  return a;
}

// iterations of an inner FCG on the sketch: chunk = predicted count, then pairs
// M != null: the operator is the explicit s x s matrix M (a.nbC = 0, wscale = 1)
// the first P steps of an inner solve on the explicit operator M as one graph (use_graph);
// keyed by the step count, M, the preconditioner and the solution vector, which fix every
// kernel argument of the steps within one solve
msp_status l2_graph(SolveCtx& c, const L2Step& a, const double* M, int P, hipGraphExec_t* out) {
  const auto key = std::make_tuple(P | (1 << 24), (const void*)M, (const void*)a.Minv, (const void*)a.y);
  auto it = c.graphs.exec.find(key);
  if (it != c.graphs.exec.end()) {
    *out = it->second;
    return MSP_OK;
  }
  c.graphs.st = c.st;
  if (!c.graphs.cap) MSP_CHECK_HIP(hipStreamCreateWithFlags(&c.graphs.cap, hipStreamNonBlocking));
  MSP_CHECK_HIP(hipStreamBeginCapture(c.graphs.cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < P && e == hipSuccess; ++i) {
    e = l2_op_matrix(c.graphs.cap, M, c.s, a.p, c.k, a.S.done, a.wp, a.pqw, a.gscratch, a.gscratch_n);
    if (e == hipSuccess) e = l2_step(c.graphs.cap, a, i + 1 == P);  // the host reads after the graph
  }
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c.graphs.cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    MSP_CHECK_HIP(e != hipSuccess ? e : e2);
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  MSP_CHECK_HIP(e);
  c.graphs.exec[key] = ex;
  *out = ex;
  return MSP_OK;
}

msp_status run_l2(SolveCtx& c, const L2Step& a_in, const double* W, int slotid, int* last, int64_t* counter,
                  const double* M = nullptr) {
  const msp_precond* P = c.P;
  const int64_t rows = P->structure == MSP_SYM_PSD ? c.n : c.m;
  L2Step a = a_in;
  // an explicit operator on the matrix cores leaves <p, M p> to the step (no pqw)
  if (M && a.gscratch && c.k >= kGemmMinK) a.pqw = nullptr;
  int issued = 0;
  int chunk = std::max(1, *last);
  const int cap = a.max_iter;
  if (c.o->use_graph && M && chunk <= cap) {  // the predicted chunk as one graph launch
    hipGraphExec_t ex = nullptr;
    TRY(l2_graph(c, a, M, chunk, &ex));
    MSP_CHECK_HIP(hipGraphLaunch(ex, c.st));
    issued = chunk;
    TRY(sync(c));
    if (*slot(c, slotid) == 0 || issued >= cap) {
      const int taken = *slot(c, slotid + 1);
      *counter += taken;
      if (taken > 0) *last = taken;
      return MSP_OK;
    }
    chunk = 2;
  }
  while (true) {
    for (int i = 0; i < chunk && issued < cap; ++i, ++issued) {
      if (M)
        MSP_CHECK_HIP(l2_op_matrix(c.st, M, c.s, a.p, c.k, a.S.done, a.wp, a.pqw, a.gscratch, a.gscratch_n));
      else
        MSP_CHECK_HIP(l2_op(c.st, P->Y, P->y_t, rows, c.s, P->ldy, a.p, c.s, c.k, a.S.done, a.part, a.pqpart, W,
                            a.wp, a.pqw, false));
      // the host mirror is read after the chunk: only its last step publishes it
      MSP_CHECK_HIP(l2_step(c.st, a, i + 1 == chunk || issued + 1 >= cap));
    }
    TRY(sync(c));
    if (*slot(c, slotid) == 0 || issued >= cap) break;
    chunk = 2;
  }
  const int taken = *slot(c, slotid + 1);
  *counter += taken;
  if (taken > 0) *last = taken;
  return MSP_OK;
}

// the first P steps as one graph (use_graph): steps 0..P-1 with their parities
msp_status step_graph(SolveCtx& c, const L2xArgs& x, int P, hipGraphExec_t* out) {
  const auto key = std::make_tuple(P, (const void*)x.G, (const void*)x.y, (const void*)x.mirror);
  auto it = c.graphs.exec.find(key);
  if (it != c.graphs.exec.end()) {
    *out = it->second;
    return MSP_OK;
  }
  c.graphs.st = c.st;
  if (!c.graphs.cap) MSP_CHECK_HIP(hipStreamCreateWithFlags(&c.graphs.cap, hipStreamNonBlocking));
  MSP_CHECK_HIP(hipStreamBeginCapture(c.graphs.cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < P && e == hipSuccess; ++i) e = l2x_step(c.graphs.cap, x, i & 1, i == 0 ? 1 : 0);
  if (e == hipSuccess) e = l2x_publish(c.graphs.cap, x, P & 1);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c.graphs.cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    MSP_CHECK_HIP(e != hipSuccess ? e : e2);
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  MSP_CHECK_HIP(e);
  c.graphs.exec[key] = ex;
  *out = ex;
  return MSP_OK;
}

// inner FCG with one kernel per step (explicit operator): the right-hand side is in
// X.r[0] and X.y is zero. Issues the predicted count plus one step (a finished column
// costs a launch that only carries its state), then pairs until every column is done.
msp_status run_l2x(SolveCtx& c, const L2xArgs& x, int slotid, int* last, int64_t* counter) {
  MSP_CHECK_HIP(l2x_start(c.st, x));
  int issued = 0;
  int chunk = std::max(1, *last + 1);
  const int cap = x.max_iter;
  if (c.o->use_graph && chunk <= cap) {  // the predicted chunk as one graph launch
    hipGraphExec_t ex = nullptr;
    TRY(step_graph(c, x, chunk, &ex));
    MSP_CHECK_HIP(hipGraphLaunch(ex, c.st));
    issued = chunk;
    TRY(sync(c));
    if (*slot(c, slotid) == 0 || issued >= cap) {
      const int taken = *slot(c, slotid + 1);
      *counter += taken;
      if (taken > 0) *last = taken;
      return MSP_OK;
    }
    chunk = 2;
  }
  while (true) {
    for (int i = 0; i < chunk && issued < cap; ++i, ++issued)
      MSP_CHECK_HIP(l2x_step(c.st, x, issued & 1, issued == 0 ? 1 : 0));
    MSP_CHECK_HIP(l2x_publish(c.st, x, issued & 1));
    TRY(sync(c));
    if (*slot(c, slotid) == 0 || issued >= cap) break;
    chunk = 2;
  }
  const int taken = *slot(c, slotid + 1);
  *counter += taken;
  if (taken > 0) *last = taken;
  return MSP_OK;
}

// the first P steps of a two-kernel solve as one graph (use_graph), keyed like l2_graph
msp_status l2f_graph(SolveCtx& c, const L2fArgs& f, int P, hipGraphExec_t* out) {
  const auto key = std::make_tuple(P | (2 << 24), (const void*)f.H, (const void*)f.Minv, (const void*)f.y);
  auto it = c.graphs.exec.find(key);
  if (it != c.graphs.exec.end()) {
    *out = it->second;
    return MSP_OK;
  }
  c.graphs.st = c.st;
  if (!c.graphs.cap) MSP_CHECK_HIP(hipStreamCreateWithFlags(&c.graphs.cap, hipStreamNonBlocking));
  MSP_CHECK_HIP(hipStreamBeginCapture(c.graphs.cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < P && e == hipSuccess; ++i) {
    e = l2f_op(c.graphs.cap, f, i, i == 0 ? 1 : 0);
    if (e == hipSuccess) e = l2f_prec(c.graphs.cap, f, i);
  }
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c.graphs.cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    MSP_CHECK_HIP(e != hipSuccess ? e : e2);
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  MSP_CHECK_HIP(e);
  c.graphs.exec[key] = ex;
  *out = ex;
  return MSP_OK;
}

// inner FCG with two kernels per step (explicit operator, direct products) from the
// l2_init state. The decision on step t's residual is taken by the operator kernel of
// step t + 1, so the predicted count plus one step is issued first (the last step's
// kernels only carry the finished state), then pairs until every column is done.
msp_status run_l2f(SolveCtx& c, const L2fArgs& f, int slotid, int* last, int64_t* counter) {
  const int cap = f.max_iter + 1;  // the decision of the capped step needs one more launch
  const int chunk = std::min(cap, std::max(1, *last + 1));
  int issued = 0;
  if (c.o->use_graph) {  // the predicted chunk as one graph launch
    hipGraphExec_t ex = nullptr;
    TRY(l2f_graph(c, f, chunk, &ex));
    MSP_CHECK_HIP(hipGraphLaunch(ex, c.st));
    issued = chunk;
  }
  int want = chunk;
  while (true) {
    for (; issued < want && issued < cap; ++issued) {
      MSP_CHECK_HIP(l2f_op(c.st, f, issued, issued == 0 ? 1 : 0));
      MSP_CHECK_HIP(l2f_prec(c.st, f, issued));
    }
    TRY(sync(c));
    if (*slot(c, slotid) == 0 || issued >= cap) break;
    want = issued + 2;
  }
  const int taken = *slot(c, slotid + 1);
  *counter += taken;
  if (taken > 0) *last = taken;
  return MSP_OK;
}

// out[:, j] = M v_j for an FP64 rows x cols row-major M (block product for k >= 8)
msp_status dense_mv(SolveCtx& c, const double* M, int64_t rows, int64_t cols, const double* v, int64_t ldv,
                    double* out, int64_t ldo, const int32_t* skip) {
  int nb = 0;
  if (c.k >= kGemmMinK && c.gemmpart) {
    // short reduction segments pay for these few-row matrices; shortest while cache-resident
    const int min_seg = (double)rows * (double)cols * 8.0 <= 64.0 * (1 << 20) ? kSegSmall : kSegWide;
    MSP_CHECK_HIP(launch_gemm_seg(c.st, M, rows, cols, v, ldv, out, ldo, c.k, skip, c.gemmpart, c.gemmpart_n,
                                  min_seg));
  } else if (c.k >= kGemmMinK)
    MSP_CHECK_HIP(launch_gemm(c.st, M, MSP_F64, false, rows, cols, cols, v, ldv, out, ldo, c.k, 0.0, false, skip,
                              nullptr, &nb));
  else
    MSP_CHECK_HIP(launch_gemv(c.st, M, MSP_F64, rows, cols, cols, v, ldv, out, ldo, c.k, 0.0, false, skip, nullptr,
                              &nb));
  return MSP_OK;
}

// out[:, j] = M^T v_j for an FP64 rows x cols row-major M
msp_status dense_mv_t(SolveCtx& c, const double* M, int64_t rows, int64_t cols, const double* v, int64_t ldv,
                      double* out, int64_t ldo, const int32_t* skip) {
  MSP_CHECK_HIP((c.k >= kGemmMinK ? launch_gemm_t : launch_gemv_t)(c.st, M, MSP_F64, rows, cols, cols, v, ldv, out,
                                                                    ldo, c.k, skip, c.gpart));
  return MSP_OK;
}

// level2_form 1: the inner operators through matrices formed once per solve.
// PSD: H2 = C^T C + lam~ W. General: A~^T (transposed copy), B^T = (A^T A~)^T by one
// block product over A with s right-hand sides and H3 = A~^T A~ (level 3); level 2 is
// applied through B. Form 2 also forms H2 = B^T B + lam~ H3 (PSD: C^T C + lam~ W) and
// inverts it.
msp_status invert_h2(SolveCtx& c) {
  if (c.form != 2) return MSP_OK;
  // the one-level preconditioner: SolveM1 exactly, through (H2 + mu I)^{-1}
  MSP_CHECK_HIP(hipMemsetAsync(c.Hstat, 0, sizeof(int32_t), c.st));
  MSP_CHECK_HIP(spd_inverse(c.st, c.s, c.H2, c.Htmp, c.P->shift_rel, c.Hscal, c.Hstat));
  int32_t bad = 0;
  MSP_CHECK_HIP(hipMemcpyAsync(&bad, c.Hstat, sizeof(int32_t), hipMemcpyDeviceToHost, c.st));
  MSP_CHECK_HIP(hipStreamSynchronize(c.st));
  if (bad) return msp_fail(MSP_ERR_NOT_POSDEF, "the level-2 matrix is not positive definite");
  return MSP_OK;
}

// G = H Minv in row-major order for symmetric H and Minv: the block product Minv H
// stores column j of Minv H, which is row j of (Minv H)^T = H Minv
msp_status form_g(SolveCtx& c, const double* H, const double* Minv, double* G) {
  int nb = 0;
  MSP_CHECK_HIP(launch_gemm(c.st, Minv, MSP_F64, false, c.s, c.s, c.s, H, c.s, G, c.s, c.s, 0.0, false, nullptr,
                            nullptr, &nb));
  return MSP_OK;
}

msp_status build_explicit(SolveCtx& c) {
  if (c.form == 0) return MSP_OK;
  const msp_precond* P = c.P;
  const int64_t n = c.n, m = c.m, s = c.s;
  if (P->structure == MSP_SYM_PSD) {
    const int sp = gram_splits(n, s);
    if (P->y_t == MSP_F64)
      MSP_CHECK_HIP(launch_gram(c.st, (const double*)P->Y, n, s, P->ldy, c.H2, c.gtmp, sp));
    else
      MSP_CHECK_HIP(launch_gram_f32(c.st, (const float*)P->Y, n, s, P->ldy, c.H2, c.gtmp, sp));
    MSP_CHECK_HIP(launch_combine_sym(c.st, s, 1.0, c.H2, P->lt, P->Wm, 0.0, c.H2));
    if (c.use_x) TRY(form_g(c, c.H2, P->Minv, c.G2));
    return invert_h2(c);
  }
  int nb = 0;
  MSP_CHECK_HIP(launch_transpose_f64(c.st, P->Y, P->y_t, m, s, P->ldy, c.Act, m));
  // B^T rows: (A^T A~)[:, j] = A^T (A~ e_j), the block transposed product with s columns
  if (s >= kGemmMinK && c.sw64)
    MSP_CHECK_HIP(launch_gemm_t_f32_as_f64(c.st, (const float*)c.A_sw, m, n, c.lda, c.Act, m, c.B2t, n, s, nullptr,
                                           c.gtmp));
  else if (s >= kGemmMinK)
    MSP_CHECK_HIP(launch_gemm_t(c.st, c.A_sw, c.sw_t, m, n, c.lda, c.Act, m, c.B2t, n, s, nullptr, c.gtmp));
  else
    MSP_CHECK_HIP(launch_gemv_t(c.st, c.A_sw, c.sw_t, m, n, c.lda, c.Act, m, c.B2t, n, s, nullptr, c.gpart));
  MSP_CHECK_HIP(launch_gemm(c.st, c.Act, MSP_F64, false, s, m, m, c.Act, m, c.H3, s, s, 0.0, false, nullptr, nullptr,
                            &nb));
  MSP_CHECK_HIP(launch_combine_sym(c.st, s, 1.0, c.H3, 0.0, nullptr, 0.0, c.H3));
  if (c.form == 2) {  // the one-level variant needs the level-2 matrix itself
    MSP_CHECK_HIP(launch_gemm(c.st, c.B2t, MSP_F64, false, s, n, n, c.B2t, n, c.H2, s, s, 0.0, false, nullptr,
                              nullptr, &nb));
    MSP_CHECK_HIP(launch_combine_sym(c.st, s, 1.0, c.H2, P->lt, c.H3, 0.0, c.H2));
  }
  return invert_h2(c);
}

// ---------------------------------- PSD (Algorithms 1-2) ----------------------------
// z = (r - C y^) / lam~ with y^ from level-2 FCG on (C^T C + lam~ W) y = C^T r, M2^{-1}
msp_status psd_solve_m1(SolveCtx& c, const double* r, double* z) {
  const msp_precond* P = c.P;
  const int64_t s = c.s, n = c.n, k = c.k;
  const int32_t* pdone = c.L1.S.done;
  L2Step a = l2step_for(c, c.L2, P->Minv, P->Wm, P->lt, 0.0, c.o->inner_tol, c.o->max_inner, SLOT_L2, pdone);
  MSP_CHECK_HIP(l2_op(c.st, P->Y, P->y_t, n, s, P->ldy, r, n, k, pdone, a.part, nullptr, nullptr, nullptr, nullptr,
                      true));
  if (c.form == 2) {  // y = (C^T C + lam~ W)^{-1} C^T r exactly
    MSP_CHECK_HIP(l2_reduce_to(c.st, a, c.rhs2, pdone));
    MSP_CHECK_HIP(launch_small_mv(c.st, s, c.H2, c.rhs2, k, pdone, c.L2.x));
    MSP_CHECK_HIP(
        launch_y_z(c.st, P->Y, P->y_t, n, s, P->ldy, c.L2.x, k, 1.0 / P->lt, r, n, -1.0 / P->lt, pdone, z, n));
    TRY(sync(c));  // the level-1 mirror is read by the caller after SolveM1
    return MSP_OK;
  }
  if (c.use_x) {  // one kernel per step on H = C^T C + lam~ W through G2 = H M2^{-1}
    L2xArgs x = c.X;
    x.Minv = P->Minv;
    x.G = c.G2;
    x.y = c.L2.x;
    x.tol = c.o->inner_tol;
    x.max_iter = c.o->max_inner;
    x.mirror = c.df + SLOT_L2;
    x.parent_done = pdone;
    a.r = x.r[0];
    MSP_CHECK_HIP(l2_rhs(c.st, a));
    TRY(run_l2x(c, x, SLOT_L2, &c.last_inner, &c.acc.inner_iters));
    MSP_CHECK_HIP(
        launch_y_z(c.st, P->Y, P->y_t, n, s, P->ldy, c.L2.x, k, 1.0 / P->lt, r, n, -1.0 / P->lt, pdone, z, n));
    return MSP_OK;
  }
  MSP_CHECK_HIP(l2_init(c.st, a));
  if (c.form == 1) {
    L2Step b = a;  // steps on H = C^T C + lam~ W
    b.nbC = 0;
    b.wscale = 1.0;
    b.wp = c.wp;
    b.pqw = c.pqw;
    TRY(run_l2(c, b, nullptr, SLOT_L2, &c.last_inner, &c.acc.inner_iters, c.H2));
  } else {
    TRY(run_l2(c, a, P->Wm, SLOT_L2, &c.last_inner, &c.acc.inner_iters));
  }
  MSP_CHECK_HIP(launch_y_z(c.st, P->Y, P->y_t, n, s, P->ldy, c.L2.x, k, 1.0 / P->lt, r, n, -1.0 / P->lt, pdone, z, n));
  return MSP_OK;
}

// The level-1 iteration of Algorithm 1: FCG on (A_sw + lam I) X = B, confirmed on A_cf. X -> L1.x
msp_status psd_core(SolveCtx& c, const double* B, int64_t ldb, double tol, int max_outer) {
  Level& L = c.L1;
  const int64_t n = c.n, k = c.k;
  MSP_CHECK_HIP(fcg_init(c.st, L.S, n, B, ldb, L.r, L.x, nullptr, c.df + SLOT_L1));
  TRY(psd_solve_m1(c, L.r, L.z));
  MSP_CHECK_HIP(fcg_first_dir(c.st, L.S, n, L.r, L.z, L.p));
  int it = 0;
  while (true) {
    // the level-1 mirror is current: psd_solve_m1 synchronised after the update
    if (*slot(c, SLOT_L1) == 0) {
      TRY(sweep(c, c.A_cf, c.cf_t, n, n, L.x, n, L.q, n, true, nullptr, false, true, false));
      MSP_CHECK_HIP(launch_axpby(c.st, n, k, 1.0, B, ldb, -1.0, L.q, n, L.q, n, nullptr));
      MSP_CHECK_HIP(fcg_confirm(c.st, L.S, n, L.q, L.r, tol, c.relres, c.df + SLOT_L1));
      TRY(sync(c));
      if (*slot(c, SLOT_L1) == 0) break;
      c.acc.restarts += 1;
      TRY(psd_solve_m1(c, L.r, L.z));
      MSP_CHECK_HIP(fcg_first_dir(c.st, L.S, n, L.r, L.z, L.p));
      continue;
    }
    if (it >= max_outer) break;
    TRY(sweep(c, c.A_sw, c.sw_t, n, n, L.p, n, L.q, n, true, L.S.done, true, false, true));
    MSP_CHECK_HIP(fcg_update(c.st, L.S, n, L.x, L.r, L.ro, L.p, L.q, tol, max_outer, c.df + SLOT_L1, c.gpart,
                             c.nb_last));
    TRY(psd_solve_m1(c, L.r, L.z));
    MSP_CHECK_HIP(fcg_direction(c.st, L.S, n, L.r, L.ro, L.z, L.p));
    ++it;
  }
  c.acc.outer_iters += (int32_t)*slot(c, SLOT_L1 + 1);
  return MSP_OK;
}

// -------------------------------- general (Algorithms 3-5) --------------------------
// level 3 (Algorithm 5): (A~^T A~ + sigma I) u = rhs by FCG with Minv; result -> out
msp_status gen_level3(SolveCtx& c, const double* rhs, double* out, double sigma, const double* Minv,
                      const int32_t* parent_done, int* last) {
  L2Step a = l2step_for(c, c.L3, Minv, nullptr, 0.0, sigma, c.o->level3_tol, c.o->max_level3, SLOT_L3, parent_done);
  a.rhs = rhs;
  if (c.form == 1) {  // (A~^T A~ + sigma I) through the explicit A~^T A~
    a.nbC = 0;
    a.wscale = 1.0;
    a.wp = c.wp;
    a.pqw = c.pqw;
  }
  MSP_CHECK_HIP(l2_init(c.st, a));
  if (c.use_f) {
    L2fArgs f = c.F;
    f.H = c.H3;
    f.Minv = Minv;
    f.sigma = sigma;
    f.S = c.L3.S;
    f.y = c.L3.x;
    f.r[0] = c.L3.r;
    f.r[1] = c.L3.ro;
    f.p[0] = c.L3.p;
    f.tol = c.o->level3_tol;
    f.max_iter = c.o->max_level3;
    f.mirror = c.df + SLOT_L3;
    TRY(run_l2f(c, f, SLOT_L3, last, &c.acc.level3_iters));
  } else {
    TRY(run_l2(c, a, nullptr, SLOT_L3, last, &c.acc.level3_iters, c.form == 1 ? c.H3 : nullptr));
  }
  MSP_CHECK_HIP(launch_copy_block(c.st, c.s, c.k, c.L3.x, c.s, out, c.s));
  return MSP_OK;
}

// SolveM2 (Algorithm 5) in the product form z = W^{-1} ((W + lam~ I)^{-1} r)
msp_status gen_solve_m2(SolveCtx& c, const double* r, double* z, const int32_t* parent_done) {
  const msp_precond* P = c.P;
  TRY(gen_level3(c, r, c.tmp_s, P->lt, P->Minv2, parent_done, &c.last_l3b));
  TRY(gen_level3(c, c.tmp_s, z, 0.0, P->Minv, parent_done, &c.last_l3a));
  return MSP_OK;
}

// q2 = A~^T A A^T A~ p2 + lam~ A~^T A~ p2   (the operator of Algorithm 4)
msp_status gen_op2(SolveCtx& c, const double* p2, double* q2, const int32_t* skip) {
  const msp_precond* P = c.P;
  const int64_t m = c.m, n = c.n, s = c.s, k = c.k;
  if (c.form == 1) {
    // B^T (B p2) + lam~ A~^T A~ p2 with B = A^T A~ formed once (two passes over B). The
    // product B^T B itself is not formed: its condition number is the fourth power of
    // A's singular-value spread and FP64 would lose the small directions.
    TRY(dense_mv_t(c, c.B2t, s, n, p2, s, c.nvec, n, skip));
    TRY(dense_mv(c, c.B2t, s, n, c.nvec, n, q2, s, skip));
    TRY(dense_mv(c, c.H3, s, s, p2, s, c.tmp_s, s, skip));
    MSP_CHECK_HIP(launch_axpby(c.st, s, k, 1.0, q2, s, P->lt, c.tmp_s, s, q2, s, skip));
    return MSP_OK;
  }
  MSP_CHECK_HIP(launch_y_z(c.st, P->Y, P->y_t, m, s, P->ldy, p2, k, 0.0, nullptr, 0, 1.0, skip, c.mvec, m));
  TRY(sweep_t(c, c.A_sw, c.sw_t, m, n, c.mvec, m, c.nvec, n, skip));
  TRY(sweep(c, c.A_sw, c.sw_t, m, n, c.nvec, n, c.mvec2, m, false, skip, false, false, false));
  MSP_CHECK_HIP(launch_axpby(c.st, m, k, 1.0, c.mvec2, m, P->lt, c.mvec, m, c.mvec2, m, skip));
  L2Step a = l2step_for(c, c.L2, nullptr, nullptr, 0.0, 0.0, 0.0, 1, SLOT_L2, nullptr);
  MSP_CHECK_HIP(l2_op(c.st, P->Y, P->y_t, m, s, P->ldy, c.mvec2, m, k, skip, a.part, nullptr, nullptr, nullptr,
                      nullptr, true));
  MSP_CHECK_HIP(l2_reduce_to(c.st, a, q2, skip));
  return MSP_OK;
}

// SolveM1 (Algorithm 4): y^ from level-2 FCG on (A~^T A A^T A~ + lam~ A~^T A~) y = A~^T A r
// preconditioned by SolveM2, then w^ = (r - A^T A~ y^) / lam~
msp_status gen_solve_m1(SolveCtx& c, const double* r, double* z) {
  const msp_precond* P = c.P;
  Level& L = c.L2;
  const int64_t m = c.m, n = c.n, s = c.s, k = c.k;
  const int32_t* pdone = c.L1.S.done;
  if (c.form == 1) {  // A~^T A r = B^T r with B = A^T A~ (s x n rows of B^T)
    TRY(dense_mv(c, c.B2t, s, n, r, n, c.rhs2, s, pdone));
  } else {
    TRY(sweep(c, c.A_sw, c.sw_t, m, n, r, n, c.mvec, m, false, pdone, false, false, false));
    L2Step a = l2step_for(c, L, nullptr, nullptr, 0.0, 0.0, 0.0, 1, SLOT_L2, nullptr);
    MSP_CHECK_HIP(l2_op(c.st, P->Y, P->y_t, m, s, P->ldy, c.mvec, m, k, pdone, a.part, nullptr, nullptr, nullptr,
                        nullptr, true));
    MSP_CHECK_HIP(l2_reduce_to(c.st, a, c.rhs2, pdone));
  }
  if (c.form == 2) {  // y = (B^T B + lam~ A~^T A~)^{-1} A~^T A r exactly: no level 2 or 3
    MSP_CHECK_HIP(launch_small_mv(c.st, s, c.H2, c.rhs2, k, pdone, L.x));
    TRY(dense_mv_t(c, c.B2t, s, n, L.x, s, c.nvec, n, pdone));
    MSP_CHECK_HIP(launch_axpby(c.st, n, k, 1.0 / P->lt, r, n, -1.0 / P->lt, c.nvec, n, z, n, pdone));
    return MSP_OK;
  }
  MSP_CHECK_HIP(fcg_init(c.st, L.S, s, c.rhs2, s, L.r, L.x, pdone, c.df + SLOT_L2));
  TRY(gen_solve_m2(c, L.r, L.z, L.S.done));
  MSP_CHECK_HIP(fcg_first_dir(c.st, L.S, s, L.r, L.z, L.p));
  for (int it = 0; it < c.o->max_inner; ++it) {
    TRY(sync(c));
    if (*slot(c, SLOT_L2) == 0) break;
    TRY(gen_op2(c, L.p, L.q, L.S.done));
    MSP_CHECK_HIP(fcg_alpha_dot(c.st, L.S, s, L.p, L.q));
    MSP_CHECK_HIP(fcg_update(c.st, L.S, s, L.x, L.r, L.ro, L.p, L.q, c.o->inner_tol, c.o->max_inner, c.df + SLOT_L2));
    TRY(gen_solve_m2(c, L.r, L.z, L.S.done));
    MSP_CHECK_HIP(fcg_direction(c.st, L.S, s, L.r, L.ro, L.z, L.p));
  }
  TRY(sync(c));
  c.acc.inner_iters += *slot(c, SLOT_L2 + 1);
  // w^ = (r - A^T (A~ y^)) / lam~
  if (c.form == 1) {  // A^T A~ y = B y
    TRY(dense_mv_t(c, c.B2t, s, n, L.x, s, c.nvec, n, pdone));
  } else {
    MSP_CHECK_HIP(launch_y_z(c.st, P->Y, P->y_t, m, s, P->ldy, L.x, k, 0.0, nullptr, 0, 1.0, pdone, c.mvec, m));
    TRY(sweep_t(c, c.A_sw, c.sw_t, m, n, c.mvec, m, c.nvec, n, pdone));
  }
  MSP_CHECK_HIP(launch_axpby(c.st, n, k, 1.0 / P->lt, r, n, -1.0 / P->lt, c.nvec, n, z, n, pdone));
  return MSP_OK;
}

// q = A^T (A p) + lam p ; t = A p kept for the rho recurrence
msp_status gen_op1(SolveCtx& c, const double* p, double* q, double* t, const int32_t* skip) {
  const int64_t m = c.m, n = c.n, k = c.k;
  TRY(sweep(c, c.A_sw, c.sw_t, m, n, p, n, t, m, false, skip, false, false, true));
  TRY(sweep_t(c, c.A_sw, c.sw_t, m, n, t, m, q, n, skip));
  if (c.lam != 0.0) MSP_CHECK_HIP(launch_axpby(c.st, n, k, 1.0, q, n, c.lam, p, n, q, n, skip));
  return MSP_OK;
}

// The level-1 iteration of Algorithm 3. normal == 0: A x = B (B m x k) with the stop on |B - A x|;
// normal != 0: (A^T A + lam I) x = B (B n x k). X -> L1.x
msp_status gen_core(SolveCtx& c, const double* B, int64_t ldb, double tol, int max_outer, bool normal) {
  Level& L = c.L1;
  const int64_t m = c.m, n = c.n, k = c.k;
  if (normal) {
    MSP_CHECK_HIP(fcg_init(c.st, L.S, n, B, ldb, L.r, L.x, nullptr, c.df + SLOT_L1));
  } else {
    MSP_CHECK_HIP(fcg_init(c.st, L.S, m, B, ldb, c.rho, nullptr, nullptr, c.df + SLOT_L1));
    MSP_CHECK_HIP(launch_axpby(c.st, n, k, 0.0, L.x, n, 0.0, nullptr, 0, L.x, n, nullptr));
    TRY(sweep_t(c, c.A_sw, c.sw_t, m, n, c.rho, m, L.r, n, nullptr));
  }
  TRY(gen_solve_m1(c, L.r, L.z));
  MSP_CHECK_HIP(fcg_first_dir(c.st, L.S, n, L.r, L.z, L.p));
  int it = 0;
  while (true) {
    TRY(sync(c));
    if (*slot(c, SLOT_L1) == 0) {
      if (normal) {
        // rtrue = B - (A^T A + lam I) x
        TRY(sweep(c, c.A_cf, c.cf_t, m, n, L.x, n, c.tvec, m, false, nullptr, false, true, false));
        MSP_CHECK_HIP(sweep_t64(c, c.A_cf, c.cf_t, m, n, c.tvec, m, L.q, n));
        if (c.lam != 0.0) MSP_CHECK_HIP(launch_axpby(c.st, n, k, 1.0, L.q, n, c.lam, L.x, n, L.q, n, nullptr));
        MSP_CHECK_HIP(launch_axpby(c.st, n, k, 1.0, B, ldb, -1.0, L.q, n, L.q, n, nullptr));
        MSP_CHECK_HIP(fcg_confirm(c.st, L.S, n, L.q, L.r, tol, c.relres, c.df + SLOT_L1));
      } else {
        TRY(sweep(c, c.A_cf, c.cf_t, m, n, L.x, n, c.tvec, m, false, nullptr, false, true, false));
        MSP_CHECK_HIP(launch_axpby(c.st, m, k, 1.0, B, ldb, -1.0, c.tvec, m, c.tvec, m, nullptr));
        MSP_CHECK_HIP(fcg_confirm(c.st, L.S, m, c.tvec, c.rho, tol, c.relres, c.df + SLOT_L1));
      }
      TRY(sync(c));
      if (*slot(c, SLOT_L1) == 0) break;
      c.acc.restarts += 1;
      if (!normal) TRY(sweep_t(c, c.A_sw, c.sw_t, m, n, c.rho, m, L.r, n, L.S.done));
      TRY(gen_solve_m1(c, L.r, L.z));
      MSP_CHECK_HIP(fcg_first_dir(c.st, L.S, n, L.r, L.z, L.p));
      continue;
    }
    if (it >= max_outer) break;
    TRY(gen_op1(c, L.p, L.q, c.tvec, L.S.done));
    MSP_CHECK_HIP(fcg_alpha_dot(c.st, L.S, n, L.p, L.q));
    if (normal) {
      MSP_CHECK_HIP(fcg_update(c.st, L.S, n, L.x, L.r, L.ro, L.p, L.q, tol, max_outer, c.df + SLOT_L1));
    } else {
      MSP_CHECK_HIP(fcg_update_nodecide(c.st, L.S, n, L.x, L.r, L.ro, L.p, L.q));
      MSP_CHECK_HIP(fcg_rho_update(c.st, L.S, m, c.rho, c.tvec, tol, max_outer, c.df + SLOT_L1));
    }
    TRY(gen_solve_m1(c, L.r, L.z));
    MSP_CHECK_HIP(fcg_direction(c.st, L.S, n, L.r, L.ro, L.z, L.p));
    ++it;
    if (log_on() && it % 25 == 0)
      fprintf(stderr, "[msp] level 1: %d steps, %lld level-2, %lld level-3 so far\n", it,
              (long long)c.acc.inner_iters, (long long)c.acc.level3_iters);
  }
  c.acc.outer_iters += (int32_t)*slot(c, SLOT_L1 + 1);
  return MSP_OK;
}

msp_status core(SolveCtx& c, const double* B, int64_t ldb, double tol, int max_outer) {
  if (c.P->structure == MSP_SYM_PSD) return psd_core(c, B, ldb, tol, max_outer);
  return gen_core(c, B, ldb, tol, max_outer, c.o->normal != 0);
}

// ------------------------------- FP64 iterative refinement --------------------------
// residual of the user's system with A_hi in FP64: rh = B - op_hi(xh)
msp_status hi_residual(SolveCtx& c, const void* A_hi, msp_dtype hi_t, const double* B, int64_t ldb, double* out) {
  const int64_t n = c.n, m = c.m, k = c.k;
  const bool psd = c.P->structure == MSP_SYM_PSD;
  if (psd) {
    TRY(sweep(c, A_hi, hi_t, n, n, c.xh, n, out, n, true, nullptr, false, true, false));
    MSP_CHECK_HIP(launch_axpby(c.st, n, k, 1.0, B, ldb, -1.0, out, n, out, n, nullptr));
  } else if (!c.o->normal) {
    TRY(sweep(c, A_hi, hi_t, m, n, c.xh, n, out, m, false, nullptr, false, true, false));
    MSP_CHECK_HIP(launch_axpby(c.st, m, k, 1.0, B, ldb, -1.0, out, m, out, m, nullptr));
  } else {
    TRY(sweep(c, A_hi, hi_t, m, n, c.xh, n, c.tvec, m, false, nullptr, false, true, false));
    MSP_CHECK_HIP(sweep_t64(c, A_hi, hi_t, m, n, c.tvec, m, out, n));
    if (c.lam != 0.0) MSP_CHECK_HIP(launch_axpby(c.st, n, k, 1.0, out, n, c.lam, c.xh, n, out, n, nullptr));
    MSP_CHECK_HIP(launch_axpby(c.st, n, k, 1.0, B, ldb, -1.0, out, n, out, n, nullptr));
  }
  return MSP_OK;
}

// per-column |v| / |B| -> host
msp_status rel_norms(SolveCtx& c, const double* v, int64_t len, std::vector<double>& out) {
  std::vector<double> num(c.k), den(c.k);
  MSP_CHECK_HIP(launch_coldots(c.st, len, c.k, v, len, v, len, c.dots));
  MSP_CHECK_HIP(hipMemcpyAsync(num.data(), c.dots, sizeof(double) * c.k, hipMemcpyDeviceToHost, c.st));
  MSP_CHECK_HIP(hipMemcpyAsync(den.data(), c.bn, sizeof(double) * c.k, hipMemcpyDeviceToHost, c.st));
  MSP_CHECK_HIP(hipStreamSynchronize(c.st));
  out.resize(c.k);
  for (int64_t j = 0; j < c.k; ++j) out[j] = den[j] > 0 ? std::sqrt(num[j] / den[j]) : 0.0;
  return MSP_OK;
}

// x += MSP_lo(b - A_hi x) until |b - A_hi x| <= tol |b|. A step "stalls" when it fails to
// halve some unconverged column's residual. After two stalled steps: PSD switches to Krylov
// refinement; general tightens the inner tolerance by 100x (not below kInnerFloor), and
// gives up (MSP_ERR_NO_CONVERGENCE, best iterate) when the step after a tightening stalls
// too, when the floor is reached, or at once for the one-level form, which has no inner
// level a tighter tolerance could improve. The level-1 steps of all inner solves together
// are capped by max_outer.
constexpr double kInnerFloor = 1e-12;

msp_status refine(SolveCtx& c, const void* A_hi, msp_dtype hi_t, const double* B, int64_t ldb, double tol,
                  std::vector<double>& rel) {
  const int64_t n = c.n, k = c.k;
  const bool psd = c.P->structure == MSP_SYM_PSD;
  const int64_t blen = (!psd && !c.o->normal) ? c.m : n;
  const int budget = c.o->max_outer;
  const int used0 = c.acc.outer_iters;
  auto left = [&]() { return budget - (c.acc.outer_iters - used0); };
  MSP_CHECK_HIP(launch_coldots(c.st, blen, k, B, ldb, B, ldb, c.bn));
  MSP_CHECK_HIP(launch_axpby(c.st, n, k, 0.0, c.xh, n, 0.0, nullptr, 0, c.xh, n, nullptr));
  MSP_CHECK_HIP(launch_copy_block(c.st, blen, k, B, ldb, c.rh, blen));
  double inner = c.o->refine_inner_tol;
  std::vector<double> prev(k, 1.0), best_rel;
  std::vector<int> slow(k, 0);
  double best = INFINITY;
  bool krylov = false, tightened = false, give_up = false;
  for (int step = 0; step < c.o->max_refine && left() > 0; ++step) {
    TRY(core(c, c.rh, blen, inner, left()));
    MSP_CHECK_HIP(launch_axpby(c.st, n, k, 1.0, c.xh, n, 1.0, c.L1.x, n, c.xh, n, nullptr));
    TRY(hi_residual(c, A_hi, hi_t, B, ldb, c.rh));
    TRY(rel_norms(c, c.rh, blen, rel));
    c.acc.refine_steps += 1;
    double worst = 0.0;
    for (double v : rel) worst = std::max(worst, v);
    if (log_on())
      fprintf(stderr, "[msp] refine step %d: max rel residual %.3e (inner tol %.1e, %d level-1 steps left)\n",
              step + 1, worst, inner, left());
    if (!psd && worst < best) {  // the general path keeps its best iterate for a give-up
      best = worst;
      best_rel = rel;
      MSP_CHECK_HIP(launch_copy_block(c.st, n, k, c.xh, n, c.L0.x, n));
    }
    bool all = true, stalled = false, halved = true;
    for (int64_t j = 0; j < k; ++j) {
      if (rel[j] > tol) all = false;
      const bool slow_step = rel[j] > 0.5 * prev[j];
      slow[j] = slow_step ? slow[j] + 1 : 0;
      if (slow_step && rel[j] > tol) halved = false;
      if (slow[j] >= 2 && rel[j] > tol) stalled = true;
      prev[j] = rel[j];
    }
    if (all) return MSP_OK;
    if (psd) {
      if (stalled) {
        krylov = true;
        break;
      }
      continue;
    }
    if (tightened) {
      if (!halved) {  // the tighter inner solve did not help either
        give_up = true;
        break;
      }
      tightened = false;
    }
    if (stalled) {
      if (c.form == 2 || inner <= kInnerFloor) {
        give_up = true;
        break;
      }
      inner = std::max(inner * 1e-2, kInnerFloor);  // ask the inner solve for more accuracy
      tightened = true;
      std::fill(slow.begin(), slow.end(), 0);
    }
  }
  if (!krylov) {
    if (!psd && (give_up || left() <= 0) && best < INFINITY) {
      double worst = 0.0;
      for (double v : rel) worst = std::max(worst, v);
      if (best < worst) {  // return the best iterate seen, with its residual
        MSP_CHECK_HIP(launch_copy_block(c.st, n, k, c.L0.x, n, c.xh, n));
        rel = best_rel;
      }
    }
    if (give_up && log_on()) fprintf(stderr, "[msp] refinement stalled: giving up\n");
    return MSP_OK;  // the caller reports MSP_ERR_NO_CONVERGENCE from the residuals
  }
  if (left() <= 0) return MSP_OK;
  // Krylov refinement: FCG in FP64 on (A_hi + lam I) e = rh, preconditioned by MSP_lo
  c.acc.krylov_refine = 1;
  Level& L = c.L0;
  MSP_CHECK_HIP(fcg_init(c.st, L.S, n, c.rh, n, L.r, L.x, nullptr, c.df + SLOT_L0));
  TRY(core(c, L.r, n, inner, left()));
  MSP_CHECK_HIP(launch_copy_block(c.st, n, k, c.L1.x, n, L.z, n));
  MSP_CHECK_HIP(fcg_first_dir(c.st, L.S, n, L.r, L.z, L.p));
  // target: |rh - A e| <= tol |B| / |rh| relative to the current residual
  double worst = 0.0;
  for (double v : rel) worst = std::max(worst, v);
  const double ktol = worst > 0 ? tol / worst : tol;
  for (int it = 0; it < c.o->max_outer && left() > 0; ++it) {
    TRY(sync(c));
    if (*slot(c, SLOT_L0) == 0) break;
    TRY(sweep(c, A_hi, hi_t, n, n, L.p, n, L.q, n, true, L.S.done, true, true, false));
    MSP_CHECK_HIP(fcg_update(c.st, L.S, n, L.x, L.r, L.ro, L.p, L.q, ktol, c.o->max_outer, c.df + SLOT_L0, c.gpart,
                             c.nb_last));
    TRY(core(c, L.r, n, inner, left()));
    MSP_CHECK_HIP(launch_copy_block(c.st, n, k, c.L1.x, n, L.z, n));
    MSP_CHECK_HIP(fcg_direction(c.st, L.S, n, L.r, L.ro, L.z, L.p));
  }
  MSP_CHECK_HIP(launch_axpby(c.st, n, k, 1.0, c.xh, n, 1.0, L.x, n, c.xh, n, nullptr));
  TRY(hi_residual(c, A_hi, hi_t, B, ldb, c.rh));
  TRY(rel_norms(c, c.rh, n, rel));
  return MSP_OK;
}

msp_status validate_solve(const msp_precond* P, const void* A_hi, msp_dtype hi_t, const void* A_lo, msp_dtype lo_t,
                          int64_t lda, double lambda, const double* B, int64_t ldb, int64_t k, double* X, int64_t ldx,
                          const msp_solve_opts* o) {
  REQUIRE(P, "P is null");
  REQUIRE(A_hi && A_lo && B && X && o, "null pointer argument");
  REQUIRE(valid_dtype(hi_t) && valid_dtype(lo_t), "bad dtype");
  REQUIRE(hi_t != MSP_BF16, "A_hi must be F64 or F32");
  REQUIRE(lda >= P->n, "lda < n");
  REQUIRE(k >= 1 && k <= kMaxK, "need 1 <= k <= %lld", (long long)kMaxK);
  const int64_t blen = (P->structure == MSP_GENERAL && !o->normal) ? P->m : P->n;
  REQUIRE(ldb >= blen && ldx >= P->n, "leading dimension too small");
  if (!isfin(o->tol) || !isfin(o->inner_tol) || !isfin(o->level3_tol) || !isfin(o->refine_inner_tol))
    return msp_fail(MSP_ERR_NONFINITE, "non-finite tolerance");
  REQUIRE(o->tol > 0 && o->inner_tol > 0 && o->level3_tol > 0 && o->refine_inner_tol > 0, "tolerances must be > 0");
  REQUIRE(o->max_outer >= 1 && o->max_inner >= 1 && o->max_level3 >= 1 && o->max_refine >= 1, "caps must be >= 1");
  if (!isfin(lambda)) return msp_fail(MSP_ERR_NONFINITE, "lambda not finite");
  REQUIRE(lambda >= 0.0, "need lambda >= 0");
  REQUIRE(!(P->structure == MSP_GENERAL && !o->normal && lambda != 0.0),
          "A x = b needs lambda = 0 (use normal = 1 for (A^T A + lam I) x = c)");
  return MSP_OK;
}

// segments of the level-1 block sweep over A_sw (k >= 8): the autotuner's choice, timed on
// this matrix into scratch vectors, or the built-in rule's
msp_status choose_segments(SolveCtx& c) {
  if (c.k < kGemmMinK || !c.gemmpart) return MSP_OK;
  const bool psd = c.P->structure == MSP_SYM_PSD;
  const int64_t rows = psd ? c.n : c.m, cols = c.n;
  const bool f64 = c.sw64;
  if (c.o->autotune) {
    // X = zeros (n x k), Y = a level-1 scratch of rows x k; both are rewritten before use
    double* Xs = c.L1.p;
    double* Ys = psd ? c.L1.q : c.tvec;
    MSP_CHECK_HIP(hipMemsetAsync(Xs, 0, sizeof(double) * (size_t)cols * (size_t)c.k, c.st));
    int nseg = 0;
    MSP_CHECK_HIP(tune_block_sweep(c.st, c.A_sw, c.sw_t, f64, rows, cols, c.lda, Xs, cols, Ys, rows, c.k, c.gemmpart,
                                   c.gemmpart_n, &nseg));
    c.sweep_nseg = nseg;
  } else {
    c.sweep_nseg = 0;
  }
  c.acc.sweep_segments =
      c.sweep_nseg > 0 ? c.sweep_nseg : gemm_split_default(rows, cols, c.k, c.sw_t, f64, c.gemmpart_n);
  return MSP_OK;
}

// the whole solve into X; status from the residuals
msp_status solve_into(SolveCtx& c, const void* A_hi, msp_dtype hi_t, const double* B, int64_t ldb, double* X,
                      int64_t ldx, msp_solve_info* info) {
  const msp_solve_opts* o = c.o;
  msp_status st = MSP_OK;
  std::vector<double> rel;
  const bool do_refine = o->refine && (c.sw_t != MSP_F64);
  TRY(choose_segments(c));
  TRY(build_explicit(c));
  if (do_refine) {
    c.A_cf = c.A_sw;  // the inner solves confirm on the matrix they sweep
    c.cf_t = c.sw_t;
    if (c.P->structure == MSP_SYM_PSD && c.A_sw != A_hi) {
      // inner operator A_lo + (lam + delta) I with delta = u_lo ||A_hi||_inf >= ||A_lo - A_hi||_2
      // (elementwise rounding of a symmetric matrix): it dominates A_hi + lam I, so the
      // low-precision MSP stays a positive definite preconditioner of the FP64 refinement
      MSP_CHECK_HIP(launch_row_abs_max(c.st, A_hi, hi_t, c.n, c.n, c.lda, c.L0.q, c.n * c.k, c.relres));
      double ninf = 0.0;
      MSP_CHECK_HIP(hipMemcpyAsync(&ninf, c.relres, sizeof(double), hipMemcpyDeviceToHost, c.st));
      MSP_CHECK_HIP(hipStreamSynchronize(c.st));
      const double u_lo = c.sw_t == MSP_BF16 ? 0x1p-8 : 0x1p-24;
      c.lam_sw = c.lam + u_lo * ninf;
    }
    TRY(refine(c, A_hi, hi_t, B, ldb, o->tol, rel));
    MSP_CHECK_HIP(launch_copy_block(c.st, c.n, c.k, c.xh, c.n, X, ldx));
  } else {
    TRY(core(c, B, ldb, o->tol, o->max_outer));
    MSP_CHECK_HIP(launch_copy_block(c.st, c.n, c.k, c.L1.x, c.n, X, ldx));
    // FP64 residual of the returned solution on A_hi
    const bool psd = c.P->structure == MSP_SYM_PSD;
    const int64_t blen = (!psd && !o->normal) ? c.m : c.n;
    MSP_CHECK_HIP(launch_coldots(c.st, blen, c.k, B, ldb, B, ldb, c.bn));
    MSP_CHECK_HIP(launch_copy_block(c.st, c.n, c.k, c.L1.x, c.n, c.xh, c.n));
    TRY(hi_residual(c, A_hi, hi_t, B, ldb, c.rh));
    TRY(rel_norms(c, c.rh, blen, rel));
  }
  TRY(ev_collect(c));
  std::vector<int32_t> done(c.k);
  MSP_CHECK_HIP(hipMemcpyAsync(done.data(), c.L1.S.done, sizeof(int32_t) * c.k, hipMemcpyDeviceToHost, c.st));
  MSP_CHECK_HIP(hipStreamSynchronize(c.st));
  double worst = 0.0;
  for (int64_t j = 0; j < c.k; ++j) {
    worst = std::max(worst, rel[j]);
    if (!std::isfinite(rel[j])) st = MSP_ERR_NONFINITE;
  }
  if (st == MSP_OK && worst > o->tol) {
    st = MSP_ERR_NO_CONVERGENCE;
    if (!do_refine)
      for (int64_t j = 0; j < c.k; ++j)
        if (done[j] == 2) st = MSP_ERR_BREAKDOWN;
  }
  c.acc.rel_residual_max = worst;
  c.acc.status = st;
  if (info) *info = c.acc;
  if (st == MSP_ERR_NO_CONVERGENCE) msp_fail(st, "tolerance not reached (relative residual %.3e)", worst);
  if (st == MSP_ERR_BREAKDOWN) msp_fail(st, "breakdown: p^T A p <= 0");
  if (st == MSP_ERR_NONFINITE) msp_fail(st, "non-finite residual");
  return st;
}

msp_status make_ctx(SolveCtx& c, void* stream, const msp_precond* P, const void* A_hi, msp_dtype hi_t,
                    const void* A_lo, msp_dtype lo_t, int64_t lda, double lambda, int64_t k, const msp_solve_opts* o,
                    void* ws, size_t ws_bytes) {
  c.st = (hipStream_t)stream;
  c.P = P;
  c.o = o;
  c.n = P->n;
  c.m = P->m;
  c.s = P->s;
  c.k = k;
  c.A_sw = A_lo;
  c.sw_t = lo_t;
  c.sw64 = P->structure == MSP_GENERAL && lo_t == MSP_F32;
  c.A_cf = A_hi;
  c.cf_t = hi_t;
  c.lda = lda;
  c.lam = lambda;  // the preconditioner keeps the handle's lam~ = lam_P + lam0
  c.lam_sw = lambda;
  c.hf = P->host_flags;
  c.df = P->dev_view_flags;
  c.evpool = (std::vector<hipEvent_t>*)P->events;
  WsCarver w(ws, ws_bytes);
  solve_layout(w, P, k, &c, o->level2_form, o->sym_sweep, o->level3_kernels);
  if (!w.ok()) return msp_fail(MSP_ERR_WORKSPACE, "workspace overflow");
  // the explicit general operators need the block transposed product (s >= 8)
  if (P->structure == MSP_GENERAL && P->s < kGemmMinK) c.form = 0;
  for (Level* L : {&c.L0, &c.L1, &c.L2, &c.L3}) MSP_CHECK_HIP(hipMemsetAsync(L->S.counter, 0, sizeof(int32_t), c.st));
  MSP_CHECK_HIP(hipMemsetAsync(c.l2b, 0, sizeof(double) * l2_bpart_doubles(c.s, k), c.st));
  return MSP_OK;
}

}  // namespace

extern "C" msp_status msp_solve_workspace(const msp_precond* P, int64_t k, const msp_solve_opts* opts,
                                          size_t* bytes) {
  REQUIRE(P && bytes, "null argument");
  REQUIRE(k >= 1 && k <= kMaxK, "need 1 <= k <= %lld", (long long)kMaxK);
  msp_solve_opts dflt;
  msp_solve_opts_default(&dflt);
  const msp_solve_opts* o = opts ? opts : &dflt;
  REQUIRE(o->level2_form >= 0 && o->level2_form <= 2, "level2_form must be 0, 1 or 2");
  REQUIRE(o->level3_kernels == 0 || o->level3_kernels == 2, "level3_kernels must be 0 or 2");
  WsCarver w(nullptr, 0);
  solve_layout(w, P, k, nullptr, o->level2_form, o->sym_sweep, o->level3_kernels);
  *bytes = w.off;
  return MSP_OK;
}

extern "C" msp_status msp_solve(void* stream, const msp_precond* P, const void* A_hi, msp_dtype hi_t,
                                const void* A_lo, msp_dtype lo_t, int64_t lda, double lambda, const double* B,
                                int64_t ldb, int64_t k, double* X, int64_t ldx, const msp_solve_opts* opts, void* ws,
                                size_t ws_bytes, msp_solve_info* info) {
  const double t0 = wall_seconds();
  msp_solve_opts dflt;
  msp_solve_opts_default(&dflt);
  const msp_solve_opts* o = opts ? opts : &dflt;
  TRY(validate_solve(P, A_hi, hi_t, A_lo, lo_t, lda, lambda, B, ldb, k, X, ldx, o));
  REQUIRE(ws, "workspace is null");
  size_t need = 0;
  TRY(msp_solve_workspace(P, k, o, &need));
  if (ws_bytes < need || ((uintptr_t)ws & 255))
    return msp_fail(MSP_ERR_WORKSPACE, "solve workspace needs %zu bytes, 256-B aligned", need);
  SolveCtx c;
  TRY(make_ctx(c, stream, P, A_hi, hi_t, A_lo, lo_t, lda, lambda, k, o, ws, ws_bytes));
  const msp_status st = solve_into(c, A_hi, hi_t, B, ldb, X, ldx, info);
  if (info) info->seconds = wall_seconds() - t0;
  return st;
}

extern "C" msp_status msp_solve_backward(void* stream, const msp_precond* P, const void* A_hi, msp_dtype hi_t,
                                         const void* A_lo, msp_dtype lo_t, int64_t lda, double lambda, const double* X,
                                         int64_t ldx, const double* G, int64_t ldg, int64_t k, double* dB,
                                         int64_t lddb, double* dlambda, double* dA, int64_t ldda,
                                         const msp_solve_opts* opts, void* ws, size_t ws_bytes, msp_solve_info* info) {
  const double t0 = wall_seconds();
  msp_solve_opts dflt;
  msp_solve_opts_default(&dflt);
  const msp_solve_opts* o = opts ? opts : &dflt;
  REQUIRE(P, "P is null");
  if (P->structure != MSP_SYM_PSD)
    return msp_fail(MSP_ERR_UNSUPPORTED, "the adjoint needs A^{-T}; only symmetric (MSP_SYM_PSD) handles");
  REQUIRE(X && G && dB, "null pointer argument");
  REQUIRE(ldx >= P->n && ldg >= P->n && lddb >= P->n, "leading dimension too small");
  REQUIRE(!dA || ldda >= P->n, "ldda < n");
  TRY(validate_solve(P, A_hi, hi_t, A_lo, lo_t, lda, lambda, G, ldg, k, dB, lddb, o));
  size_t need = 0;
  TRY(msp_solve_workspace(P, k, o, &need));
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255))
    return msp_fail(MSP_ERR_WORKSPACE, "solve workspace needs %zu bytes, 256-B aligned", need);
  SolveCtx c;
  TRY(make_ctx(c, stream, P, A_hi, hi_t, A_lo, lo_t, lda, lambda, k, o, ws, ws_bytes));
  // dB = (A + lam I)^{-T} G = (A + lam I)^{-1} G for symmetric A, same handle
  msp_status st = solve_into(c, A_hi, hi_t, G, ldg, dB, lddb, info);
  if (st != MSP_OK && st != MSP_ERR_NO_CONVERGENCE) return st;
  if (dlambda) {
    std::vector<double> d(k);
    MSP_CHECK_HIP(launch_coldots(c.st, c.n, k, dB, lddb, X, ldx, c.dots));
    MSP_CHECK_HIP(hipMemcpyAsync(d.data(), c.dots, sizeof(double) * k, hipMemcpyDeviceToHost, c.st));
    MSP_CHECK_HIP(hipStreamSynchronize(c.st));
    double acc = 0.0;
    for (double v : d) acc += v;
    *dlambda = -acc;
  }
  if (dA) {
    MSP_CHECK_HIP(launch_outer_neg(c.st, c.n, k, dB, lddb, X, ldx, dA, ldda));
    MSP_CHECK_HIP(hipStreamSynchronize(c.st));
  }
  if (info) info->seconds = wall_seconds() - t0;
  return st;
}

// ====================================================================================
// msp_schatten
// ====================================================================================
namespace {
size_t schatten_extra(const msp_precond* P, int64_t N) {
  // X, A G, A X and the generated probes (n x N each), the A^T partials of the power
  // iteration, probe dots
  return ((size_t)4 * P->n * N + gemv_t_part_doubles(P->n, P->n, 1) + 4 * N + 4096) * sizeof(double);
}
}  // namespace

extern "C" msp_status msp_schatten_workspace(const msp_precond* P, int64_t nprobes, const msp_solve_opts* opts,
                                             size_t* bytes) {
  REQUIRE(P && bytes, "null argument");
  size_t solve = 0;
  TRY(msp_solve_workspace(P, nprobes, opts, &solve));
  *bytes = ((solve + 255) & ~size_t(255)) + schatten_extra(P, nprobes);
  return MSP_OK;
}

extern "C" msp_status msp_gaussian_probes(void* stream, int64_t n, int64_t N, uint64_t seed, double* G,
                                          int64_t ldg) {
  REQUIRE(G, "G is null");
  REQUIRE(n >= 1 && N >= 1 && ldg >= n, "need n, N >= 1 and ldg >= n");
  MSP_CHECK_HIP(launch_probes((hipStream_t)stream, seed, n, N, G, ldg));
  return MSP_OK;
}

namespace {

// The ridge values of the trace driver (Section 3.2): per probe g_k and node t,
// T_k = <A g_k, A x_k> and D_k = t <g_k, x_k> with x_k = (A^T A + t I)^{-1} g_k solved by the
// three-level MSP of the handle (lam~ = t + lam0), so that T_k = |g_k|^2 - D_k.
struct TraceRun {
  hipStream_t st = nullptr;
  void* stream = nullptr;
  msp_precond* P = nullptr;
  const void *A_hi = nullptr, *A_lo = nullptr;
  msp_dtype hi_t = MSP_F64, lo_t = MSP_F64;
  int64_t lda = 0, n = 0, N = 0, ldg = 0;
  const double* G = nullptr;
  msp_solve_opts o{};
  void* ws = nullptr;
  size_t solve_bytes = 0;
  double *X = nullptr, *AG = nullptr, *AX = nullptr, *gtp = nullptr, *dv = nullptr;
  std::vector<double> gg;  // |g_k|^2
  msp_solve_info acc{};
  bool unconverged = false;
  int nodes = 0;
};

void trace_add_info(TraceRun& R, const msp_solve_info& i) {
  R.acc.outer_iters += i.outer_iters;
  R.acc.inner_iters += i.inner_iters;
  R.acc.level3_iters += i.level3_iters;
  R.acc.refine_steps += i.refine_steps;
  R.acc.sweeps += i.sweeps;
  R.acc.sweep_bytes += i.sweep_bytes;
  R.acc.rel_residual_max = std::max(R.acc.rel_residual_max, i.rel_residual_max);
  R.acc.sweep_segments = i.sweep_segments;
}

// workspace carving, probes (given or drawn from probe_seed), |g|^2
msp_status trace_setup(TraceRun& R, void* stream, msp_precond* P, const void* A_hi, msp_dtype hi_t, const void* A_lo,
                       msp_dtype lo_t, int64_t lda, const double* G, int64_t ldg, int64_t N, uint64_t probe_seed,
                       const msp_solve_opts& o, void* ws, size_t ws_bytes) {
  REQUIRE(N >= 1 && (!G || ldg >= P->n), "bad probe block");
  REQUIRE(P->m == P->n, "square A only");
  size_t need = 0;
  TRY(msp_schatten_workspace(P, N, &o, &need));
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255))
    return msp_fail(MSP_ERR_WORKSPACE, "trace workspace needs %zu bytes, 256-B aligned", need);
  R.stream = stream;
  R.st = (hipStream_t)stream;
  R.P = P;
  R.A_hi = A_hi;
  R.hi_t = hi_t;
  R.A_lo = A_lo;
  R.lo_t = lo_t;
  R.lda = lda;
  R.n = P->n;
  R.N = N;
  R.o = o;
  R.ws = ws;
  TRY(msp_solve_workspace(P, N, &o, &R.solve_bytes));
  R.solve_bytes = (R.solve_bytes + 255) & ~size_t(255);
  const int64_t n = R.n;
  R.X = (double*)((char*)ws + R.solve_bytes);
  R.AG = R.X + n * N;
  R.AX = R.AG + n * N;
  double* Gw = R.AX + n * N;
  R.gtp = Gw + n * N;
  R.dv = R.gtp + gemv_t_part_doubles(n, n, 1);
  if (!G) {  // probes from probe_seed (the generator of msp_gaussian_probes)
    MSP_CHECK_HIP(launch_probes(R.st, probe_seed, n, N, Gw, n));
    G = Gw;
    ldg = n;
  }
  R.G = G;
  R.ldg = ldg;
  R.gg.assign(N, 0.0);
  MSP_CHECK_HIP(launch_coldots(R.st, n, N, G, ldg, G, ldg, R.dv));
  MSP_CHECK_HIP(hipMemcpyAsync(R.gg.data(), R.dv, sizeof(double) * N, hipMemcpyDeviceToHost, R.st));
  MSP_CHECK_HIP(hipStreamSynchronize(R.st));
  return MSP_OK;
}

// A g for every probe, once (before the first node)
msp_status trace_ag(TraceRun& R) {
  int nb = 0;
  MSP_CHECK_HIP(R.N >= kGemmMinK ? launch_gemm(R.st, R.A_hi, R.hi_t, false, R.n, R.n, R.lda, R.G, R.ldg, R.AG, R.n, R.N,
                                               0.0, false, nullptr, nullptr, &nb)
                                 : launch_gemv(R.st, R.A_hi, R.hi_t, R.n, R.n, R.lda, R.G, R.ldg, R.AG, R.n, R.N, 0.0,
                                               false, nullptr, nullptr, &nb));
  return MSP_OK;
}

// |A| by power iteration on A^T A from the first probe (30 steps, 1% margin)
msp_status trace_sigma_max(TraceRun& R, double* smax) {
  const int64_t n = R.n;
  double* v = R.X;
  MSP_CHECK_HIP(launch_copy_block(R.st, n, 1, R.G, R.ldg, v, n));
  double s2 = 0.0;
  std::vector<double> nn(1);
  for (int it = 0; it < 30; ++it) {
    MSP_CHECK_HIP(launch_coldots(R.st, n, 1, v, n, v, n, R.dv));
    MSP_CHECK_HIP(hipMemcpyAsync(nn.data(), R.dv, sizeof(double), hipMemcpyDeviceToHost, R.st));
    MSP_CHECK_HIP(hipStreamSynchronize(R.st));
    const double nv = std::sqrt(nn[0]);
    if (nv == 0.0) break;
    MSP_CHECK_HIP(launch_axpby(R.st, n, 1, 1.0 / nv, v, n, 0.0, nullptr, 0, v, n, nullptr));
    int nb = 0;
    MSP_CHECK_HIP(launch_gemv(R.st, R.A_hi, R.hi_t, n, n, R.lda, v, n, R.AX, n, 1, 0.0, false, nullptr, nullptr, &nb));
    MSP_CHECK_HIP(launch_gemv_t(R.st, R.A_hi, R.hi_t, n, n, R.lda, R.AX, n, v, n, 1, nullptr, R.gtp));
    MSP_CHECK_HIP(launch_coldots(R.st, n, 1, v, n, v, n, R.dv));
    MSP_CHECK_HIP(hipMemcpyAsync(nn.data(), R.dv, sizeof(double), hipMemcpyDeviceToHost, R.st));
    MSP_CHECK_HIP(hipStreamSynchronize(R.st));
    s2 = std::sqrt(nn[0]);  // |A^T A v| with |v| = 1
  }
  *smax = std::sqrt(std::max(s2, 1e-300)) * 1.01;
  return MSP_OK;
}

// one node: T[k] = <A g_k, A x_k>, D[k] = t <g_k, x_k>
msp_status trace_node(TraceRun& R, double t, int index, int count, std::vector<double>& T, std::vector<double>& D) {
  const int64_t n = R.n, N = R.N;
  TRY(msp_precond_set_lambda(R.stream, R.P, t));
  msp_solve_info i{};
  msp_status s_ = msp_solve(R.stream, R.P, R.A_hi, R.hi_t, R.A_lo, R.lo_t, R.lda, t, R.G, R.ldg, N, R.X, n, &R.o, R.ws,
                            R.solve_bytes, &i);
  if (s_ != MSP_OK && s_ != MSP_ERR_NO_CONVERGENCE) return s_;
  if (s_ != MSP_OK) R.unconverged = true;
  trace_add_info(R, i);
  R.nodes += 1;
  if (log_on())
    fprintf(stderr, "[msp] trace node %d%s%d t=%.3e outer=%d inner=%lld level3=%lld relres=%.2e\n", index + 1,
            count > 0 ? "/" : " ", count > 0 ? count : 0, t, i.outer_iters, (long long)i.inner_iters,
            (long long)i.level3_iters, i.rel_residual_max);
  int nb = 0;
  MSP_CHECK_HIP(N >= kGemmMinK ? launch_gemm(R.st, R.A_hi, R.hi_t, false, n, n, R.lda, R.X, n, R.AX, n, N, 0.0, false,
                                             nullptr, nullptr, &nb)
                               : launch_gemv(R.st, R.A_hi, R.hi_t, n, n, R.lda, R.X, n, R.AX, n, N, 0.0, false, nullptr,
                                             nullptr, &nb));
  MSP_CHECK_HIP(launch_coldots(R.st, n, N, R.AG, n, R.AX, n, R.dv));
  MSP_CHECK_HIP(launch_coldots(R.st, n, N, R.G, R.ldg, R.X, n, R.dv + N));
  T.resize(N);
  D.resize(N);
  MSP_CHECK_HIP(hipMemcpyAsync(T.data(), R.dv, sizeof(double) * N, hipMemcpyDeviceToHost, R.st));
  MSP_CHECK_HIP(hipMemcpyAsync(D.data(), R.dv + N, sizeof(double) * N, hipMemcpyDeviceToHost, R.st));
  MSP_CHECK_HIP(hipStreamSynchronize(R.st));
  for (int64_t k = 0; k < N; ++k) D[k] *= t;
  return MSP_OK;
}

// sum over the grid nodes below u_j (u_j - h, u_j - 2h, ...) of h sin(pi p/2)/pi e^{(p/2) u}
double lower_tail_weight(double p, double h, double u_j) {
  const double c = h * std::sin(M_PI * p / 2.0) / M_PI;
  return c * std::exp(0.5 * p * (u_j - h)) / (1.0 - std::exp(-0.5 * p * h));
}

// u_hi from |A|: above it the integrand's tail is eps_q of the top singular value's share
double upper_end(double smax, double p, double eps_q) {
  return 2.0 * std::log(smax) + (2.0 / (2.0 - p)) * std::log(1.0 / eps_q);
}

void finish_stats(const std::vector<double>& per, double* estimate, double* std_err) {
  const int64_t N = (int64_t)per.size();
  double mean = 0.0;
  for (double v : per) mean += v;
  mean /= (double)N;
  double var = 0.0;
  for (double v : per) var += (v - mean) * (v - mean);
  *estimate = mean;
  if (std_err) *std_err = N > 1 ? std::sqrt(var / (double)(N - 1) / (double)N) : NAN;
}

msp_status trace_finish(TraceRun& R, double t0, msp_solve_info* info) {
  R.acc.status = R.unconverged ? MSP_ERR_NO_CONVERGENCE : MSP_OK;
  R.acc.seconds = wall_seconds() - t0;
  R.acc.trace_nodes = R.nodes;
  if (info) *info = R.acc;
  if (R.unconverged) return msp_fail(MSP_ERR_NO_CONVERGENCE, "a ridge solve stopped at its iteration cap");
  return MSP_OK;
}

constexpr int kMaxTraceNodes = 400;
constexpr double kTraceEps = 1e-4;

}  // namespace

extern "C" msp_status msp_schatten(void* stream, msp_trace_kind kind, msp_precond* P, const void* A_hi,
                                   msp_dtype hi_t, const void* A_lo, msp_dtype lo_t, int64_t lda, double p,
                                   const double* G, int64_t ldg, int64_t N, uint64_t probe_seed, double h,
                                   double u_lo, double u_hi, const msp_solve_opts* opts, void* ws, size_t ws_bytes,
                                   double* estimate, double* std_err, msp_solve_info* info) {
  const double t0 = wall_seconds();
  msp_solve_opts dflt;
  msp_solve_opts_default(&dflt);
  msp_solve_opts o = opts ? *opts : dflt;
  REQUIRE(P && estimate, "null argument");
  REQUIRE(kind == MSP_TRACE_SCHATTEN_P || kind == MSP_TRACE_EFFDIM, "bad kind");
  if (!isfin(p)) return msp_fail(MSP_ERR_NONFINITE, "p not finite");
  if (kind == MSP_TRACE_EFFDIM) {
    REQUIRE(P->structure == MSP_SYM_PSD, "effective dimension needs an MSP_SYM_PSD handle");
    REQUIRE(p > 0.0, "lam > 0");
  } else {
    REQUIRE(P->structure == MSP_GENERAL, "Schatten-p needs an MSP_GENERAL handle");
    REQUIRE(p > 0.0 && p < 2.0, "need 0 < p < 2");
    REQUIRE(h > 0.0 && isfin(h), "need h > 0");
    REQUIRE(!isfin(u_lo) || !isfin(u_hi) || u_hi >= u_lo, "u_hi < u_lo");
  }
  TraceRun R;
  TRY(trace_setup(R, stream, P, A_hi, hi_t, A_lo, lo_t, lda, G, ldg, N, probe_seed, o, ws, ws_bytes));
  const int64_t n = R.n;
  std::vector<double> per(N, 0.0);
  if (kind == MSP_TRACE_EFFDIM) {
    if (P->lam != p) TRY(msp_precond_set_lambda(stream, P, p));
    msp_solve_info i{};
    msp_status s_ = msp_solve(stream, P, A_hi, hi_t, A_lo, lo_t, lda, p, R.G, R.ldg, N, R.X, n, &R.o, ws,
                              R.solve_bytes, &i);
    if (s_ != MSP_OK && s_ != MSP_ERR_NO_CONVERGENCE) return s_;
    if (s_ != MSP_OK) R.unconverged = true;
    trace_add_info(R, i);
    R.nodes = 1;
    // per probe: g^T g - lam g^T x
    MSP_CHECK_HIP(launch_coldots(R.st, n, N, R.G, R.ldg, R.X, n, R.dv));
    std::vector<double> gx(N);
    MSP_CHECK_HIP(hipMemcpyAsync(gx.data(), R.dv, sizeof(double) * N, hipMemcpyDeviceToHost, R.st));
    MSP_CHECK_HIP(hipStreamSynchronize(R.st));
    for (int64_t j = 0; j < N; ++j) per[j] = R.gg[j] - p * gx[j];
    finish_stats(per, estimate, std_err);
    return trace_finish(R, t0, info);
  }
  R.o.normal = 1;
  if (!isfin(u_hi)) {  // the upper end from a power-iteration estimate of |A|
    double smax = 0.0;
    TRY(trace_sigma_max(R, &smax));
    u_hi = upper_end(smax, p, kTraceEps);
  }
  TRY(trace_ag(R));
  const double c = h * std::sin(M_PI * p / 2.0) / M_PI;
  const double lam_save = P->lam;
  std::vector<double> T, D;
  auto restore = [&](msp_status s) {
    (void)msp_precond_set_lambda(stream, P, lam_save);
    return s;
  };
  if (isfin(u_lo)) {  // the fixed grid u_lo, u_lo + h, ... <= u_hi
    const int count = (int)std::floor((u_hi - u_lo) / h + 1e-9) + 1;
    for (int jn = 0; jn < count; ++jn) {
      const double u = u_lo + h * jn;
      msp_status s_ = trace_node(R, std::exp(u), jn, count, T, D);
      if (s_ != MSP_OK) return restore(s_);
      const double w = c * std::exp(0.5 * p * u);
      for (int64_t j = 0; j < N; ++j) per[j] += w * T[j];
    }
  } else {
    // nodes u_hi, u_hi - h, ... with the lower tail replaced by its t -> 0 limit |g|^2: the
    // deficit t <g, x> is nondecreasing in t, so after node j that replacement is off by at
    // most D_j times the tail weight per probe; stop when the mean of that bound is at most
    // kTraceEps of the estimate
    std::vector<double> acc(N, 0.0);
    for (int jn = 0; jn < kMaxTraceNodes; ++jn) {
      const double u = u_hi - h * jn;
      msp_status s_ = trace_node(R, std::exp(u), jn, 0, T, D);
      if (s_ != MSP_OK) return restore(s_);
      const double w = c * std::exp(0.5 * p * u);
      const double wb = lower_tail_weight(p, h, u);
      double dm = 0.0, em = 0.0;
      for (int64_t j = 0; j < N; ++j) {
        acc[j] += w * T[j];
        per[j] = acc[j] + wb * R.gg[j];
        dm += std::fabs(D[j]);
        em += per[j];
      }
      dm /= (double)N;
      em /= (double)N;
      if (dm * wb <= kTraceEps * std::fabs(em)) break;
    }
  }
  TRY(msp_precond_set_lambda(stream, P, lam_save));
  finish_stats(per, estimate, std_err);
  return trace_finish(R, t0, info);
}

extern "C" msp_status msp_orlicz(void* stream, msp_precond* P, const void* A_hi, msp_dtype hi_t, const void* A_lo,
                                 msp_dtype lo_t, int64_t lda, const double* coefs, const double* powers,
                                 int64_t nterms, const double* G, int64_t ldg, int64_t N, uint64_t probe_seed,
                                 double h, double u_hi, double eps_q, const msp_solve_opts* opts, void* ws,
                                 size_t ws_bytes, double* estimate, double* std_err, double* sums,
                                 msp_solve_info* info) {
  const double t0 = wall_seconds();
  msp_solve_opts dflt;
  msp_solve_opts_default(&dflt);
  msp_solve_opts o = opts ? *opts : dflt;
  REQUIRE(P && estimate && coefs && powers, "null argument");
  REQUIRE(P->structure == MSP_GENERAL, "the Orlicz norm needs an MSP_GENERAL handle");
  REQUIRE(nterms >= 1 && nterms <= 16, "need 1 <= nterms <= 16");
  for (int64_t q = 0; q < nterms; ++q) {
    REQUIRE(isfin(coefs[q]) && coefs[q] > 0.0, "coefficients must be finite and > 0");
    REQUIRE(isfin(powers[q]) && powers[q] > 0.0 && powers[q] < 2.0, "powers must lie in (0, 2)");
  }
  REQUIRE(h > 0.0 && isfin(h), "need h > 0");
  if (!isfin(eps_q)) eps_q = kTraceEps;
  REQUIRE(eps_q > 0.0 && eps_q < 1.0, "need 0 < eps_q < 1");
  TraceRun R;
  TRY(trace_setup(R, stream, P, A_hi, hi_t, A_lo, lo_t, lda, G, ldg, N, probe_seed, o, ws, ws_bytes));
  R.o.normal = 1;
  double pmax = 0.0;
  for (int64_t q = 0; q < nterms; ++q) pmax = std::max(pmax, powers[q]);
  if (!isfin(u_hi)) {
    double smax = 0.0;
    TRY(trace_sigma_max(R, &smax));
    u_hi = upper_end(smax, pmax, eps_q);
  }
  TRY(trace_ag(R));
  const double lam_save = P->lam;
  std::vector<double> T, D;
  std::vector<std::vector<double>> acc(nterms, std::vector<double>(N, 0.0)), per(nterms, std::vector<double>(N, 0.0));
  for (int jn = 0; jn < kMaxTraceNodes; ++jn) {
    const double u = u_hi - h * jn;
    msp_status s_ = trace_node(R, std::exp(u), jn, 0, T, D);
    if (s_ != MSP_OK) {
      (void)msp_precond_set_lambda(stream, P, lam_save);
      return s_;
    }
    double dm = 0.0;
    for (int64_t j = 0; j < N; ++j) dm += std::fabs(D[j]);
    dm /= (double)N;
    bool done = true;
    for (int64_t q = 0; q < nterms; ++q) {
      const double pq = powers[q];
      const double w = h * std::sin(M_PI * pq / 2.0) / M_PI * std::exp(0.5 * pq * u);
      const double wb = lower_tail_weight(pq, h, u);
      double em = 0.0;
      for (int64_t j = 0; j < N; ++j) {
        acc[q][j] += w * T[j];
        per[q][j] = acc[q][j] + wb * R.gg[j];
        em += per[q][j];
      }
      em /= (double)N;
      if (dm * wb > eps_q * std::fabs(em)) done = false;
    }
    if (done) break;
  }
  TRY(msp_precond_set_lambda(stream, P, lam_save));
  // the Schatten sums, then the root r of sum_q c_q r^{-p_q} S_q = 1 by bisection on ln r
  std::vector<double> S(nterms, 0.0);
  for (int64_t q = 0; q < nterms; ++q) {
    for (int64_t j = 0; j < N; ++j) S[q] += per[q][j];
    S[q] /= (double)N;
    if (!(S[q] > 0.0)) return msp_fail(MSP_ERR_NONFINITE, "a Schatten sum estimate is not positive");
  }
  if (sums)
    for (int64_t q = 0; q < nterms; ++q) sums[q] = S[q];
  auto phi = [&](double lr) {
    double v = 0.0;
    for (int64_t q = 0; q < nterms; ++q) v += coefs[q] * S[q] * std::exp(-powers[q] * lr);
    return v - 1.0;
  };
  double lo = -1.0, hi = 1.0;
  while (phi(lo) < 0.0) lo -= 2.0 * (hi - lo);
  while (phi(hi) > 0.0) hi += 2.0 * (hi - lo);
  for (int it = 0; it < 400; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (phi(mid) > 0.0) lo = mid;
    else hi = mid;
    if (hi - lo <= 1e-15 * std::max(1.0, std::fabs(mid))) break;
  }
  const double r = std::exp(0.5 * (lo + hi));
  *estimate = r;
  if (std_err) {  // delta method: per-probe values of the left side, divided by its slope in r
    std::vector<double> vals(N, 0.0);
    double dphi = 0.0;
    for (int64_t q = 0; q < nterms; ++q) {
      const double f = coefs[q] * std::pow(r, -powers[q]);
      for (int64_t j = 0; j < N; ++j) vals[j] += f * per[q][j];
      dphi += -powers[q] * f / r * S[q];
    }
    double m = 0.0, se = 0.0;
    finish_stats(vals, &m, &se);
    *std_err = se / std::fabs(dphi);
  }
  return trace_finish(R, t0, info);
}
