// The Ky Fan k-norm ||A||_(k) = sum_{i<=k} sigma_i(A) (Section 3.2 names Ky Fan norms beside
// the Orlicz norms as reachable by the spectral-sum machinery). A sum of the top k singular
// values needs the top of the spectrum itself, which ridge solves (A^T A + t I)^{-1} do not
// isolate; it comes from the top singular subspace:
//   Z_0 = Omega (b >= k Gaussian vectors of msp_gaussian_probes), Q_0 = orth(Z_0),
//   Q_i = orth(A^T A Q_{i-1}) for i = 1..q, and the Rayleigh-Ritz values of A on Q_q,
//   the square roots of the eigenvalues of (A Q_q)^T (A Q_q).
// orth(Z) = Z V Lambda^{-1/2} from the eigenpairs of Z^T Z (directions with eigenvalue at most
// 1e-13 of the largest become zero columns). The products with A are the block sweeps of the
// solver (matrix cores for b >= 8, FP64 arithmetic on an F64 or F32 A); the b x b eigenproblems
// (b <= 64) run in one workgroup by cyclic Jacobi rotations (Golub and Van Loan, the
// symmetric Schur step of Section 8.5) in a parallel (round-robin) ordering, in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <mutex>
#include <vector>

#include "msp_internal.h"

#define KREQUIRE(cond, ...)                                          \
  do {                                                               \
    if (!(cond)) return msp_fail(MSP_ERR_INVALID_ARG, __VA_ARGS__);  \
  } while (0)

namespace {

constexpr int JT = 256;          // threads of the Jacobi workgroup
constexpr int kMaxB = 64;        // block size limit (the b x b matrices live in LDS)
constexpr int kJacobiSweeps = 40;
constexpr double kDrop = 1e-13;  // orth: eigenvalues at most this fraction of the largest are dropped

// player at position pos of round r in the circle method over bb (even) players: position 0
// keeps player 0, the others rotate; pair m of a round is (position m, position bb - 1 - m)
__device__ __forceinline__ int rr_player(int pos, int r, int bb) {
  return pos == 0 ? 0 : 1 + ((pos - 1 + r) % (bb - 1));
}

// eigenvalues lam[0..b) and eigenvectors V (column j = eigenvector j, row-major b x b) of the
// symmetric part of G (row-major b x b)
__global__ void __launch_bounds__(JT) k_jacobi_eig(const double* __restrict__ G, int b, double* __restrict__ lam,
                                                  double* __restrict__ V) {
  extern __shared__ double sm[];  // a and v, b x (b + 1) each
  __shared__ double cs[kMaxB / 2], sn[kMaxB / 2];
  __shared__ int pp[kMaxB / 2], qq[kMaxB / 2];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const int ld = b + 1;
  double* a = sm;
  double* v = sm + (size_t)b * ld;
  for (int idx = tid; idx < b * b; idx += JT) {
    const int i = idx / b, j = idx - i * b;
    a[i * ld + j] = 0.5 * (G[i * b + j] + G[j * b + i]);
    v[i * ld + j] = i == j ? 1.0 : 0.0;
  }
  const int bb = b + (b & 1);  // an odd size gets a phantom index that pairs with nothing
  const int np = bb / 2;
  __syncthreads();
  // threshold Jacobi: a pair whose |a_pq| is at most 1e-16 sqrt(|a_pp a_qq|) is left as it
  // is; the sweeps end after one that rotates no pair
  for (int sweep = 0; sweep < kJacobiSweeps && b > 1; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < bb - 1; ++r) {
      if (tid < np) {
        int p = rr_player(tid, r, bb), q = rr_player(bb - 1 - tid, r, bb);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        double c = 1.0, s = 0.0;
        if (q < b) {
          const double apq = a[p * ld + q];
          if (fabs(apq) > 1e-16 * sqrt(fabs(a[p * ld + p] * a[q * ld + q]))) {
            rotated = 1;  // every writer stores 1: no ordering needed
            const double tau = (a[q * ld + q] - a[p * ld + p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(fma(tau, tau, 1.0)));
            c = 1.0 / sqrt(fma(t, t, 1.0));
            s = t * c;
          }
        }
        pp[tid] = p;
        qq[tid] = q;
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      // rows p, q of a: a <- J^T a (disjoint pairs)
      for (int idx = tid; idx < np * b; idx += JT) {
        const int m = idx / b, j = idx - m * b;
        const int p = pp[m], q = qq[m];
        if (q >= b) continue;
        const double c = cs[m], s = sn[m];
        const double ap = a[p * ld + j], aq = a[q * ld + j];
        a[p * ld + j] = c * ap - s * aq;
        a[q * ld + j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns p, q of a and v: a <- a J, v <- v J
      for (int idx = tid; idx < np * b; idx += JT) {
        const int m = idx / b, i = idx - m * b;
        const int p = pp[m], q = qq[m];
        if (q >= b) continue;
        const double c = cs[m], s = sn[m];
        const double ap = a[i * ld + p], aq = a[i * ld + q];
        a[i * ld + p] = c * ap - s * aq;
        a[i * ld + q] = s * ap + c * aq;
        const double vp = v[i * ld + p], vq = v[i * ld + q];
        v[i * ld + p] = c * vp - s * vq;
        v[i * ld + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    if (!rotated) break;  // uniform: read after the round's last barrier
    __syncthreads();      // every thread has read it before thread 0 clears it
  }
  for (int i = tid; i < b; i += JT) lam[i] = a[i * ld + i];
  for (int idx = tid; idx < b * b; idx += JT) {
    const int i = idx / b, j = idx - i * b;
    V[i * b + j] = v[i * ld + j];
  }
}

// Q[c][i] = sum_j Z[j][i] V[j][c] / sqrt(lam[c]) (0 for dropped directions); Z and Q hold b
// vectors of length n; a block takes 32 consecutive i for every c
constexpr int OT = 256;
constexpr int OR = 32;
__global__ void __launch_bounds__(OT) k_orth_apply(const double* __restrict__ Z, int64_t n, int b,
                                                  const double* __restrict__ V, const double* __restrict__ lam,
                                                  double* __restrict__ Q) {
  __shared__ double zs[kMaxB][OR + 1];
  __shared__ double vs[kMaxB][kMaxB + 1];
  __shared__ double sc[kMaxB];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * OR;
  double lmax = 0.0;
  for (int j = 0; j < b; ++j) lmax = fmax(lmax, lam[j]);
  for (int c = tid; c < b; c += OT) sc[c] = lam[c] > kDrop * lmax ? 1.0 / sqrt(lam[c]) : 0.0;
  for (int idx = tid; idx < b * b; idx += OT) vs[idx / b][idx % b] = V[idx];
  for (int idx = tid; idx < b * OR; idx += OT) {
    const int j = idx / OR, ii = idx % OR;
    const int64_t i = i0 + ii;
    zs[j][ii] = i < n ? Z[(int64_t)j * n + i] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < b * OR; idx += OT) {
    const int c = idx / OR, ii = idx % OR;
    const int64_t i = i0 + ii;
    if (i >= n) continue;
    double t = 0.0;
    for (int j = 0; j < b; ++j) t = fma(zs[j][ii], vs[j][c], t);
    Q[(int64_t)c * n + i] = t * sc[c];
  }
}

size_t jacobi_lds(int b) { return 2 * (size_t)b * (size_t)(b + 1) * sizeof(double); }

std::once_flag g_jacobi_once;
hipError_t g_jacobi_err = hipSuccess;

hipError_t launch_jacobi(hipStream_t st, const double* G, int b, double* lam, double* V) {
  std::call_once(g_jacobi_once, [] {
    g_jacobi_err = hipFuncSetAttribute((const void*)k_jacobi_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)jacobi_lds(kMaxB));
  });
  if (g_jacobi_err != hipSuccess) return g_jacobi_err;
  hipLaunchKernelGGL(k_jacobi_eig, dim3(1), dim3(JT), jacobi_lds(b), st, G, b, lam, V);
  return hipGetLastError();
}

struct KyWs {
  double *Z, *Q, *T, *G, *V, *lam, *part;
};

KyWs kyfan_layout(WsCarver& w, int64_t m, int64_t n, int64_t b) {
  KyWs k{};
  k.Z = w.take<double>(b * n);
  k.Q = w.take<double>(b * n);
  k.T = w.take<double>(b * m);
  k.G = w.take<double>(b * b);
  k.V = w.take<double>(b * b);
  k.lam = w.take<double>(b);
  k.part = w.take<double>(std::max(gemv_t_part_doubles(m, n, b), gemv_t_part_doubles(b, std::max(m, n), b)));
  return k;
}

// Y (k vectors of length rows) = A X (X: k vectors of length cols), FP64 arithmetic
hipError_t prod(hipStream_t st, const void* A, msp_dtype t, int64_t rows, int64_t cols, int64_t lda, const double* X,
                double* Y, int64_t k) {
  int nb = 0;
  if (k >= kGemmMinK)
    return launch_gemm(st, A, t, true, rows, cols, lda, X, cols, Y, rows, k, 0.0, false, nullptr, nullptr, &nb);
  if (t == MSP_F32)
    return launch_gemv_f32_as_f64(st, (const float*)A, rows, cols, lda, X, cols, Y, rows, k, 0.0, false, nullptr,
                                  nullptr, &nb);
  return launch_gemv(st, A, t, rows, cols, lda, X, cols, Y, rows, k, 0.0, false, nullptr, nullptr, &nb);
}

// Y (k vectors of length cols) = A^T X (X: k vectors of length rows), FP64 arithmetic
hipError_t prod_t(hipStream_t st, const void* A, msp_dtype t, int64_t rows, int64_t cols, int64_t lda,
                  const double* X, double* Y, int64_t k, double* part) {
  if (t == MSP_F32)
    return (k >= kGemmMinK ? launch_gemm_t_f32_as_f64 : launch_gemv_t_f32_as_f64)(st, (const float*)A, rows, cols, lda,
                                                                                 X, rows, Y, cols, k, nullptr, part);
  return (k >= kGemmMinK ? launch_gemm_t : launch_gemv_t)(st, A, t, rows, cols, lda, X, rows, Y, cols, k, nullptr,
                                                          part);
}

// Q = orth(Z) for b vectors of length n (Z^T Z through a product with Z as a b x n matrix)
hipError_t orth(hipStream_t st, const KyWs& k, const double* Z, double* Q, int64_t n, int b) {
  hipError_t e = prod(st, Z, MSP_F64, b, n, n, Z, k.G, b);
  if (e != hipSuccess) return e;
  e = launch_jacobi(st, k.G, b, k.lam, k.V);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_orth_apply, dim3((unsigned)((n + OR - 1) / OR)), dim3(OT), 0, st, Z, n, b, k.V, k.lam, Q);
  return hipGetLastError();
}

}  // namespace

extern "C" msp_status msp_kyfan_workspace(int64_t m, int64_t n, int64_t b, size_t* bytes) {
  KREQUIRE(bytes, "bytes is null");
  KREQUIRE(m >= 1 && n >= 1 && b >= 1 && b <= kMaxB, "need m, n >= 1 and 1 <= b <= %d", kMaxB);
  WsCarver w(nullptr, 0);
  kyfan_layout(w, m, n, b);
  *bytes = w.off;
  return MSP_OK;
}

extern "C" msp_status msp_kyfan(void* stream, const void* A, msp_dtype a_t, int64_t m, int64_t n, int64_t lda,
                                int64_t k, int64_t b, int32_t q, uint64_t seed, void* ws, size_t ws_bytes,
                                double* estimate, double* sigma) {
  KREQUIRE(A && estimate, "null argument");
  KREQUIRE(a_t == MSP_F64 || a_t == MSP_F32, "A must be F64 or F32");
  KREQUIRE(m >= 1 && n >= 1 && lda >= n, "need m, n >= 1 and lda >= n");
  KREQUIRE(b >= 1 && b <= kMaxB && b <= n && b <= m, "need 1 <= b <= min(%d, m, n)", kMaxB);
  KREQUIRE(k >= 1 && k <= b, "need 1 <= k <= b");
  KREQUIRE(q >= 0 && q <= 100000, "need 0 <= q <= 100000");
  size_t need = 0;
  msp_status s = msp_kyfan_workspace(m, n, b, &need);
  if (s != MSP_OK) return s;
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255))
    return msp_fail(MSP_ERR_WORKSPACE, "Ky Fan workspace needs %zu bytes, 256-B aligned", need);
  hipStream_t st = (hipStream_t)stream;
  WsCarver w(ws, ws_bytes);
  const KyWs K = kyfan_layout(w, m, n, b);
  const int bi = (int)b;
  MSP_CHECK_HIP(launch_probes(st, seed, n, b, K.Z, n));
  MSP_CHECK_HIP(orth(st, K, K.Z, K.Q, n, bi));
  for (int32_t it = 0; it < q; ++it) {
    MSP_CHECK_HIP(prod(st, A, a_t, m, n, lda, K.Q, K.T, b));
    MSP_CHECK_HIP(prod_t(st, A, a_t, m, n, lda, K.T, K.Z, b, K.part));
    MSP_CHECK_HIP(orth(st, K, K.Z, K.Q, n, bi));
  }
  // Rayleigh-Ritz: the eigenvalues of (A Q)^T (A Q)
  MSP_CHECK_HIP(prod(st, A, a_t, m, n, lda, K.Q, K.T, b));
  MSP_CHECK_HIP(prod(st, K.T, MSP_F64, b, m, m, K.T, K.G, b));
  MSP_CHECK_HIP(launch_jacobi(st, K.G, bi, K.lam, K.V));
  std::vector<double> lam(b);
  MSP_CHECK_HIP(hipMemcpyAsync(lam.data(), K.lam, sizeof(double) * b, hipMemcpyDeviceToHost, st));
  MSP_CHECK_HIP(hipStreamSynchronize(st));
  std::vector<double> sg(b);
  for (int64_t i = 0; i < b; ++i) {
    if (!std::isfinite(lam[i])) return msp_fail(MSP_ERR_NONFINITE, "a Ritz value is not finite");
    sg[i] = std::sqrt(std::max(lam[i], 0.0));
  }
  std::sort(sg.begin(), sg.end(), std::greater<double>());
  double est = 0.0;
  for (int64_t i = 0; i < k; ++i) est += sg[i];
  *estimate = est;
  if (sigma)
    for (int64_t i = 0; i < b; ++i) sigma[i] = sg[i];
  return MSP_OK;
}
