// Host side of libmsp: argument validation, workspace layout, and the level loops of
// Multi-level Sketched Preconditioning that enqueue the kernels of k_*.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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

hipError_t launch_gemv_f32_as_f64(hipStream_t st, const float* A, int64_t rows, int64_t cols, int64_t lda,
                                  const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k, double lam,
                                  bool diag_shift, const int32_t* skip, double* dot_part, int* nblocks);

namespace {

size_t dsize(msp_dtype t) { return t == MSP_F64 ? 8 : (t == MSP_F32 ? 4 : 2); }
bool valid_dtype(int t) { return t == MSP_F64 || t == MSP_F32 || t == MSP_BF16; }
bool isfin(double v) { return std::isfinite(v); }

constexpr int kMaxGammaDraw = 32;
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
extern "C" msp_status msp_sketch_workspace(int64_t m, int64_t n, int64_t s, int32_t gamma, size_t* bytes) {
  REQUIRE(bytes, "bytes is null");
  REQUIRE(m >= 1 && n >= 1 && s >= 1 && gamma >= 1 && gamma <= s && gamma <= kMaxGammaDraw && s <= n,
          "invalid sizes m=%lld n=%lld s=%lld gamma=%d", (long long)m, (long long)n, (long long)s, gamma);
  WsCarver w(nullptr, 0);
  carve_sketch(w, n, s, gamma);
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
  SketchWs k = carve_sketch(w, n, s, gamma);
  MSP_CHECK_HIP(launch_sketch_gen(st, seed, n, s, gamma, S_rows, S_signs));
  MSP_CHECK_HIP(build_buckets(st, S_rows, S_signs, n, s, gamma, k.b, k.scratch));
  const double scale = 1.0 / std::sqrt((double)gamma);
  MSP_CHECK_HIP(launch_sketch_apply(st, A, a_t, m, n, lda, s, k.b, scale, Y, y_t, ldy));
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
                                  msp_dtype y_t, int64_t ldy, double lambda, double lambda0, int64_t phi,
                                  int32_t phi_gamma, uint64_t phi_seed, void* ws, size_t ws_bytes, msp_precond** P) {
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
  REQUIRE(lambda >= 0.0 && lambda0 >= 0.0 && lambda + lambda0 > 0.0, "need lambda, lambda0 >= 0 and lambda + lambda0 > 0");
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
    // Algorithm 1 line 3: W = S C (bucket lists of S, then a row gather of C)
    SketchWs sk = carve_sketch(w, n, s, gamma);
    if (!w.ok()) return fail(msp_fail(MSP_ERR_WORKSPACE, "workspace overflow"));
    hipError_t e = build_buckets(st, S_rows, S_signs, n, s, gamma, sk.b, sk.scratch);
    if (e == hipSuccess) e = launch_gather_rows(st, Y, y_t, ldy, s, s, sk.b, 1.0 / std::sqrt((double)gamma), o.Wm, s);
    if (e == hipSuccess) e = launch_symmetrize(st, s, o.Wm);
    // line 4: C~ = Phi C, then C~^T C~
    if (e == hipSuccess) e = launch_sketch_gen(st, phi_seed, n, phi, phi_gamma, o.phi_rows, o.phi_signs);
    if (e == hipSuccess) e = build_buckets(st, o.phi_rows, o.phi_signs, n, phi, phi_gamma, o.sk_Phi.b, o.sk_Phi.scratch);
    if (e == hipSuccess) e = launch_gather_rows(st, Y, y_t, ldy, s, phi, o.sk_Phi.b, sphi, o.small, s);
    if (e == hipSuccess) e = launch_gram(st, o.small, phi, s, s, o.G, o.gpart, gram_splits(phi, s));
    if (e != hipSuccess) return fail(msp_fail_hip(e, "nystrom kernels", __FILE__, __LINE__));
  } else {
    // Algorithm 3 lines 4-5: A^ = Phi A~ over the m rows, M3a = A^^T A^
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
  o->refine_inner_tol = 1e-6;
  o->max_refine = 30;
  o->profile = 0;
}

namespace {

struct Level {
  int64_t len = 0, k = 0;
  double *x = nullptr, *r = nullptr, *ro = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  FcgState S{};
};

Level carve_level(WsCarver& w, int64_t len, int64_t k) {
  Level L;
  L.len = len;
  L.k = k;
  L.x = w.take<double>(len * k);
  L.r = w.take<double>(len * k);
  L.ro = w.take<double>(len * k);
  L.z = w.take<double>(len * k);
  L.p = w.take<double>(len * k);
  L.q = w.take<double>(len * k);
  L.S = carve_fcg_state(w, len, k);
  return L;
}

struct SolveCtx {
  hipStream_t st;
  const msp_precond* P;
  const msp_solve_opts* o;
  int64_t n, m, s, k;
  // sweep matrix (inside MSP) and confirmation matrix (FP64 residuals)
  const void* A_sw;
  msp_dtype sw_t;
  const void* A_cf;
  msp_dtype cf_t;
  int64_t lda;
  double lam;
  Level L1, L2, L3;
  double *tpart, *rhs2, *wp, *relres, *gpart;
  double *l2part, *l2pq, *pqw, *l2b;
  int nb_last = 0;  // blocks of the last level-1 sweep (its <p, q> partials)
  double *mvec, *mvec2, *nvec;  // general path: m x k, m x k, n x k
  int32_t* hf;                  // host mirror (pinned)
  int32_t* df;                  // device view of the host mirror
  int last_inner = 4;
  int last_l3 = 4;
  msp_solve_info acc{};
  std::vector<hipEvent_t>* evpool = nullptr;
  size_t evused = 0;
};

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

size_t solve_layout(WsCarver& w, const msp_precond* P, int64_t k, SolveCtx* c) {
  const int64_t n = P->n, m = P->m, s = P->s;
  const int64_t nb_gemv = (std::max(n, m) + 3) / 4;  // upper bound of gemv blocks (R >= 4)
  Level L1 = carve_level(w, n, k);
  Level L2 = carve_level(w, s, k);
  Level L3 = carve_level(w, s, k);
  double* tpart = w.take<double>((size_t)tall_blocks(std::max(n, m)) * s * k);
  double* rhs2 = w.take<double>(s * k);
  double* wp = w.take<double>(s * k);
  double* relres = w.take<double>(k);
  double* gpart = w.take<double>(std::max<size_t>(nb_gemv * k, gemv_t_part_doubles(m, n, k)));
  double* l2part = w.take<double>(l2_op_part_doubles(std::max(n, m), s, k));
  double* l2pq = w.take<double>(l2_op_pq_doubles(std::max(n, m), k));
  double* pqw = w.take<double>(s * k);
  double* l2b = w.take<double>(l2_bpart_doubles(s, k));
  double *mvec = nullptr, *mvec2 = nullptr, *nvec = nullptr;
  if (P->structure == MSP_GENERAL) {
    mvec = w.take<double>(m * k);
    mvec2 = w.take<double>(m * k);
    nvec = w.take<double>(n * k);
  }
  if (c) {
    c->L1 = L1;
    c->L2 = L2;
    c->L3 = L3;
    c->tpart = tpart;
    c->rhs2 = rhs2;
    c->wp = wp;
    c->relres = relres;
    c->gpart = gpart;
    c->mvec = mvec;
    c->mvec2 = mvec2;
    c->nvec = nvec;
    c->l2part = l2part;
    c->l2pq = l2pq;
    c->pqw = pqw;
    c->l2b = l2b;
  }
  return w.off;
}

inline volatile int32_t* slot(SolveCtx& c, int i) { return (volatile int32_t*)(c.hf + i); }

msp_status sync(SolveCtx& c) {
  MSP_CHECK_HIP(hipStreamSynchronize(c.st));
  return MSP_OK;
}

// q = (A + lam I) p with per-block <p, q> partials; alpha for level 1. fp64: FP64
// arithmetic also for FP32 storage (the refinement residual).
msp_status psd_op1(SolveCtx& c, const void* A, msp_dtype t, const double* p, double* q, const int32_t* skip,
                   bool with_alpha, bool fp64 = false) {
  int nb = 0;
  hipError_t e;
  hipEvent_t stop = nullptr;
  if (with_alpha) TRY(ev_begin(c, &stop));
  if (fp64 && t == MSP_F32)
    e = launch_gemv_f32_as_f64(c.st, (const float*)A, c.n, c.n, c.lda, p, c.n, q, c.n, c.k, c.lam, true, skip,
                               with_alpha ? c.gpart : nullptr, &nb);
  else
    e = launch_gemv(c.st, A, t, c.n, c.n, c.lda, p, c.n, q, c.n, c.k, c.lam, true, skip,
                    with_alpha ? c.gpart : nullptr, &nb);
  MSP_CHECK_HIP(e);
  if (stop) MSP_CHECK_HIP(hipEventRecord(stop, c.st));
  c.nb_last = nb;
  c.acc.sweeps += 1;
  c.acc.sweep_bytes += (double)c.n * (double)c.n * (double)dsize(t);
  return MSP_OK;
}

// ---- level 2 of the PSD method (Algorithm 2) --------------------------------------
// z = (r - C y^) / lam~ with y^ from level-2 FCG on (C^T C + lam~ W) y = C^T r, M2^{-1}
msp_status psd_solve_m1(SolveCtx& c, const double* r, double* z) {
  const msp_precond* P = c.P;
  Level& L = c.L2;
  const int64_t s = c.s, n = c.n, k = c.k;
  const int32_t* pdone = c.L1.S.done;
  L2Step a;
  a.s = s;
  a.k = k;
  a.nbC = l2_blocks(n);
  a.part = c.l2part;
  a.pqpart = c.l2pq;
  a.wp = c.wp;
  a.pqw = c.pqw;
  a.wscale = P->lt;
  a.sigma = 0.0;
  a.y = L.x;
  a.r = L.r;
  a.ro = L.ro;
  a.z = L.z;
  a.p = L.p;
  a.q = L.q;
  a.Minv = P->Minv;
  a.S = L.S;
  a.bpart = c.l2b;
  a.tol = c.o->inner_tol;
  a.max_iter = c.o->max_inner;
  a.mirror = c.df + SLOT_L2;
  a.parent_done = pdone;
  // right-hand side C^T r, then z = M2^{-1} r2, p = z
  MSP_CHECK_HIP(l2_op(c.st, P->Y, P->y_t, n, s, P->ldy, r, n, k, pdone, a.part, nullptr, nullptr, nullptr, nullptr,
                      true));
  MSP_CHECK_HIP(l2_init(c.st, a));
  int issued = 0;
  int chunk = std::max(1, c.last_inner);
  const int cap = c.o->max_inner;
  while (true) {
    for (int i = 0; i < chunk && issued < cap; ++i, ++issued) {
      MSP_CHECK_HIP(l2_op(c.st, P->Y, P->y_t, n, s, P->ldy, L.p, s, k, L.S.done, a.part, a.pqpart, P->Wm, a.wp,
                          a.pqw, false));
      MSP_CHECK_HIP(l2_step(c.st, a));
    }
    TRY(sync(c));
    if (*slot(c, SLOT_L2) == 0 || issued >= cap) break;
    chunk = 2;
  }
  const int taken = *slot(c, SLOT_L2 + 1);
  c.acc.inner_iters += taken;
  if (taken > 0) c.last_inner = taken;
  // w^ = (r - C y^) / lam~
  MSP_CHECK_HIP(launch_y_z(c.st, P->Y, P->y_t, n, s, P->ldy, L.x, k, 1.0 / P->lt, r, n, -1.0 / P->lt, pdone, z, n));
  return MSP_OK;
}

// ---- level 1 of the PSD method (Algorithm 1 line 5) --------------------------------
// Solves (A_sw + lam I) X = B to tolerance tol, confirmed with A_cf. Result in L1.x.
msp_status psd_core(SolveCtx& c, const double* B, int64_t ldb, double tol, int max_outer) {
  Level& L = c.L1;
  const int64_t n = c.n, k = c.k;
  MSP_CHECK_HIP(fcg_init(c.st, L.S, n, B, ldb, L.r, L.x, nullptr, c.df + SLOT_L1));
  TRY(psd_solve_m1(c, L.r, L.z));
  MSP_CHECK_HIP(fcg_first_dir(c.st, L.S, n, L.r, L.z, L.p));
  int it = 0;
  while (true) {
    // the host mirror of level 1 is current here: psd_solve_m1 synchronised after the update
    if (*slot(c, SLOT_L1) == 0) {
      // confirm every column that converged on its recurrence residual
      TRY(psd_op1(c, c.A_cf, c.cf_t, L.x, L.q, nullptr, false, true));
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
    TRY(psd_op1(c, c.A_sw, c.sw_t, L.p, L.q, L.S.done, true));
    MSP_CHECK_HIP(fcg_update(c.st, L.S, n, L.x, L.r, L.ro, L.p, L.q, tol, max_outer, c.df + SLOT_L1, c.gpart,
                             c.nb_last));
    TRY(psd_solve_m1(c, L.r, L.z));
    MSP_CHECK_HIP(fcg_direction(c.st, L.S, n, L.r, L.ro, L.z, L.p));
    ++it;
  }
  c.acc.outer_iters = std::max(c.acc.outer_iters, (int32_t)*slot(c, SLOT_L1 + 1));
  return MSP_OK;
}

msp_status finish_info(SolveCtx& c, msp_solve_info* info, msp_status st) {
  // per-column status and residuals
  std::vector<int32_t> done(c.k);
  std::vector<double> rel(c.k);
  MSP_CHECK_HIP(hipMemcpyAsync(done.data(), c.L1.S.done, sizeof(int32_t) * c.k, hipMemcpyDeviceToHost, c.st));
  MSP_CHECK_HIP(hipMemcpyAsync(rel.data(), c.relres, sizeof(double) * c.k, hipMemcpyDeviceToHost, c.st));
  MSP_CHECK_HIP(hipStreamSynchronize(c.st));
  double worst = 0.0;
  msp_status out = st;
  for (int64_t j = 0; j < c.k; ++j) {
    worst = std::max(worst, rel[j]);
    if (out == MSP_OK) {
      if (done[j] == 2) out = MSP_ERR_BREAKDOWN;
      else if (done[j] == 3 || done[j] == 0) out = MSP_ERR_NO_CONVERGENCE;
      else if (!std::isfinite(rel[j])) out = MSP_ERR_NONFINITE;
    }
  }
  c.acc.rel_residual_max = worst;
  c.acc.status = out;
  if (info) *info = c.acc;
  if (out != MSP_OK && out != st) {
    if (out == MSP_ERR_NO_CONVERGENCE) msp_fail(out, "iteration cap reached before the tolerance");
    if (out == MSP_ERR_BREAKDOWN) msp_fail(out, "breakdown: p^T A p <= 0");
    if (out == MSP_ERR_NONFINITE) msp_fail(out, "non-finite residual");
  }
  return out;
}

}  // namespace

extern "C" msp_status msp_solve_workspace(const msp_precond* P, int64_t k, const msp_solve_opts* opts,
                                          size_t* bytes) {
  REQUIRE(P && bytes, "null argument");
  REQUIRE(k >= 1 && k <= kMaxK, "need 1 <= k <= %lld", (long long)kMaxK);
  (void)opts;
  WsCarver w(nullptr, 0);
  solve_layout(w, P, k, nullptr);
  *bytes = w.off;
  return MSP_OK;
}

namespace {
msp_status validate_solve(const msp_precond* P, const void* A_hi, msp_dtype hi_t, const void* A_lo, msp_dtype lo_t,
                          int64_t lda, const double* B, int64_t ldb, int64_t k, double* X, int64_t ldx,
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
  return MSP_OK;
}
}  // namespace

extern "C" msp_status msp_solve(void* stream, const msp_precond* P, const void* A_hi, msp_dtype hi_t,
                                const void* A_lo, msp_dtype lo_t, int64_t lda, const double* B, int64_t ldb,
                                int64_t k, double* X, int64_t ldx, const msp_solve_opts* opts, void* ws,
                                size_t ws_bytes, msp_solve_info* info) {
  msp_solve_opts dflt;
  msp_solve_opts_default(&dflt);
  const msp_solve_opts* o = opts ? opts : &dflt;
  TRY(validate_solve(P, A_hi, hi_t, A_lo, lo_t, lda, B, ldb, k, X, ldx, o));
  REQUIRE(ws, "workspace is null");
  size_t need = 0;
  TRY(msp_solve_workspace(P, k, o, &need));
  if (ws_bytes < need || ((uintptr_t)ws & 255))
    return msp_fail(MSP_ERR_WORKSPACE, "solve workspace needs %zu bytes, 256-B aligned", need);
  if (P->structure != MSP_SYM_PSD) return msp_fail(MSP_ERR_UNSUPPORTED, "general structure not in this build yet");

  SolveCtx c;
  c.st = (hipStream_t)stream;
  c.P = P;
  c.o = o;
  c.n = P->n;
  c.m = P->m;
  c.s = P->s;
  c.k = k;
  c.A_sw = A_lo;
  c.sw_t = lo_t;
  c.A_cf = A_hi;
  c.cf_t = hi_t;
  c.lda = lda;
  c.lam = P->lam;
  c.hf = P->host_flags;
  c.df = P->dev_view_flags;
  WsCarver w(ws, ws_bytes);
  solve_layout(w, P, k, &c);
  // the last-block tickets start at zero
  for (Level* L : {&c.L1, &c.L2, &c.L3}) MSP_CHECK_HIP(hipMemsetAsync(L->S.counter, 0, sizeof(int32_t), c.st));
  MSP_CHECK_HIP(hipMemsetAsync(c.l2b, 0, sizeof(double) * l2_bpart_doubles(c.s, k), c.st));


  c.evpool = (std::vector<hipEvent_t>*)P->events;
  msp_status st = psd_core(c, B, ldb, o->tol, o->max_outer);
  if (st != MSP_OK) return st;
  TRY(ev_collect(c));
  MSP_CHECK_HIP(launch_copy_block(c.st, c.n, k, c.L1.x, c.n, X, ldx));
  return finish_info(c, info, MSP_OK);
}

extern "C" msp_status msp_solve_backward(void*, const msp_precond*, const void*, msp_dtype, const void*, msp_dtype,
                                         int64_t, const double*, int64_t, const double*, int64_t, int64_t, double*,
                                         int64_t, double*, double*, int64_t, const msp_solve_opts*, void*, size_t,
                                         msp_solve_info*) {
  return msp_fail(MSP_ERR_UNSUPPORTED, "not in this build yet");
}

extern "C" msp_status msp_schatten_workspace(const msp_precond*, int64_t, const msp_solve_opts*, size_t*) {
  return msp_fail(MSP_ERR_UNSUPPORTED, "not in this build yet");
}

extern "C" msp_status msp_schatten(void*, msp_trace_kind, msp_precond*, const void*, msp_dtype, const void*, msp_dtype,
                                   int64_t, double, const double*, int64_t, int64_t, double, double, double,
                                   const msp_solve_opts*, void*, size_t, double*, double*, msp_solve_info*) {
  return msp_fail(MSP_ERR_UNSUPPORTED, "not in this build yet");
}
