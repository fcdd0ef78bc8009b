// The A-sweeps: q = (A + lam I) p for the level-1 iteration (the dominant cost of
// Algorithms 1 and 3) and v = A^T u for the normal-equation operator of Algorithm 3.
// A is row-major and streamed once per sweep with 16-byte loads; the k vectors are
// re-read from L2/MALL. Storage FP64/FP32/BF16; arithmetic FP64 for FP64 storage and
// FP32 (converted vectors, FP32 accumulation) for the low-precision storages.
#include "msp_internal.h"

#include <hip/hip_bf16.h>

namespace {

constexpr int WAVE = 64;
constexpr int NT = 256;

template <class T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef uint32_t nu4 __attribute__((ext_vector_type(4)));

// VEC elements of A per 16-byte load, converted to TC
template <class TA, class TC, int VEC>
struct Vec16;
template <>
struct Vec16<double, double, 2> {
  static __device__ __forceinline__ void load(const double* p, double* o) {
    const nd2 v = __builtin_nontemporal_load(reinterpret_cast<const nd2*>(p));
    o[0] = v.x;
    o[1] = v.y;
  }
};
template <>
struct Vec16<float, float, 4> {
  static __device__ __forceinline__ void load(const float* p, float* o) {
    const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(p));
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <>
struct Vec16<float, double, 4> {
  static __device__ __forceinline__ void load(const float* p, double* o) {
    const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(p));
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <>
struct Vec16<__hip_bfloat16, float, 8> {
  static __device__ __forceinline__ void load(const __hip_bfloat16* p, float* o) {
    const nu4 v = __builtin_nontemporal_load(reinterpret_cast<const nu4*>(p));
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = __uint_as_float(w[i] << 16);
      o[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
    }
  }
};

template <class TA, class TC>
__device__ __forceinline__ TC scalar_as(const TA* p);
template <>
__device__ __forceinline__ double scalar_as<double, double>(const double* p) { return *p; }
template <>
__device__ __forceinline__ float scalar_as<float, float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ double scalar_as<float, double>(const float* p) { return (double)*p; }
template <>
__device__ __forceinline__ float scalar_as<__hip_bfloat16, float>(const __hip_bfloat16* p) {
  return __bfloat162float(*p);
}

template <class TA, class TC, int VEC, bool ALN>
__device__ __forceinline__ void load_vec(const TA* p, TC* o) {
  if constexpr (ALN) {
    Vec16<TA, TC, VEC>::load(p, o);
  } else {
#pragma unroll
    for (int v = 0; v < VEC; ++v) o[v] = scalar_as<TA, TC>(p + v);
  }
}

// Block of NT threads computes R rows of Y = A X (+ lam X) for K vectors; each thread
// keeps UNR 16-byte loads per row in flight.
template <class TA, class TC, int VEC, int R, int K, bool ALN, int UNR>
__global__ void __launch_bounds__(NT) k_gemv(const TA* __restrict__ A, int64_t lda, int64_t rows, int64_t cols,
                                            const double* __restrict__ X, int64_t ldx, double* __restrict__ Y,
                                            int64_t ldy, int k, int j0, double lam, int diag,
                                            const int32_t* __restrict__ skip, double* __restrict__ dot_part,
                                            int k_total) {
  __shared__ TC red[NT / WAVE][R * K];
  const int64_t r0 = (int64_t)blockIdx.x * R;
  TC acc[R][K];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < K; ++j) acc[r][j] = (TC)0;
  bool live[K];
#pragma unroll
  for (int j = 0; j < K; ++j) live[j] = (j0 + j < k) && !(skip && skip[j0 + j]);
  const int64_t cv = (cols / VEC) * VEC;
  const TA* arow[R];
#pragma unroll
  for (int r = 0; r < R; ++r) arow[r] = A + min(r0 + r, rows - 1) * lda;
  int64_t c = (int64_t)threadIdx.x * VEC;
  constexpr int64_t STEP = (int64_t)NT * VEC;
  for (; c + (UNR - 1) * STEP < cv; c += STEP * UNR) {
    TC a[UNR][R][VEC];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r) load_vec<TA, TC, VEC, ALN>(arow[r] + c + u * STEP, a[u][r]);
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      TC xv[K][VEC];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const double* xp = X + (int64_t)(j0 + (live[j] ? j : 0)) * ldx + c + u * STEP;
#pragma unroll
        for (int v = 0; v < VEC; ++v) xv[j][v] = (TC)xp[v];
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[r][j] = fma(a[u][r][v], xv[j][v], acc[r][j]);
    }
  }
  for (; c < cv; c += STEP) {
    TC xv[K][VEC];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const double* xp = X + (int64_t)(j0 + (live[j] ? j : 0)) * ldx + c;
#pragma unroll
      for (int v = 0; v < VEC; ++v) xv[j][v] = (TC)xp[v];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      TC a[VEC];
      load_vec<TA, TC, VEC, ALN>(arow[r] + c, a);
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[r][j] = fma(a[v], xv[j][v], acc[r][j]);
    }
  }
  // tail columns
  for (int64_t c = cv + threadIdx.x; c < cols; c += NT) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const TC a = scalar_as<TA, TC>(arow[r] + c);
#pragma unroll
      for (int j = 0; j < K; ++j) acc[r][j] = fma(a, (TC)X[(int64_t)(j0 + (live[j] ? j : 0)) * ldx + c], acc[r][j]);
    }
  }
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const TC v = wsum(acc[r][j]);
      if (lane == 0) red[w][r * K + j] = v;
    }
  __syncthreads();
  __shared__ double dp[R * K];
  if (threadIdx.x < R * K) {
    const int r = threadIdx.x / K, j = threadIdx.x % K;
    const int64_t row = r0 + r;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < NT / WAVE; ++q) sum += (double)red[q][threadIdx.x];
    double prod = 0.0;
    if (row < rows && live[j]) {
      const double xr = (diag || dot_part) ? X[(int64_t)(j0 + j) * ldx + row] : 0.0;
      const double y = sum + (diag ? lam * xr : 0.0);
      Y[(int64_t)(j0 + j) * ldy + row] = y;
      prod = xr * y;
    }
    dp[threadIdx.x] = prod;
  }
  __syncthreads();
  if (dot_part && threadIdx.x < K) {
    const int j = threadIdx.x;
    double t = 0.0;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) t += dp[rr * K + j];
    if (j0 + j < k) dot_part[(int64_t)blockIdx.x * k_total + j0 + j] = t;
  }
}

// Y[:, j] = A^T X[:, j]: block (column tile, row tile); partial over the row tile
template <class TA, class TC, int VEC, int K, bool ALN>
__global__ void __launch_bounds__(NT) k_gemv_t(const TA* __restrict__ A, int64_t lda, int64_t rows, int64_t cols,
                                              const double* __restrict__ X, int64_t ldx, int k, int j0,
                                              int64_t rows_per_tile, double* __restrict__ part) {
  const int64_t c = ((int64_t)blockIdx.x * NT + threadIdx.x) * VEC;
  const int64_t rb = (int64_t)blockIdx.y * rows_per_tile;
  const int64_t re = min(rows, rb + rows_per_tile);
  TC acc[K][VEC];
#pragma unroll
  for (int j = 0; j < K; ++j)
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[j][v] = (TC)0;
  const bool full = (c + VEC <= cols);
  for (int64_t r = rb; r < re; ++r) {
    TC a[VEC];
    if (full) {
      load_vec<TA, TC, VEC, ALN>(A + r * lda + c, a);
    } else {
#pragma unroll
      for (int v = 0; v < VEC; ++v) a[v] = (c + v < cols) ? scalar_as<TA, TC>(A + r * lda + c + v) : (TC)0;
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const TC x = (j0 + j < k) ? (TC)X[(int64_t)(j0 + j) * ldx + r] : (TC)0;
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[j][v] = fma(a[v], x, acc[j][v]);
    }
  }
  double* out = part + (int64_t)blockIdx.y * k * cols;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j0 + j >= k) break;
#pragma unroll
    for (int v = 0; v < VEC; ++v)
      if (c + v < cols) out[(int64_t)(j0 + j) * cols + c + v] = (double)acc[j][v];
  }
}

__global__ void k_sum_tiles(const double* __restrict__ part, int tiles, int64_t cols, int k,
                            const int32_t* __restrict__ skip, double* __restrict__ Y, int64_t ldy) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t len = cols * k;
  if (i >= len) return;
  const int j = (int)(i / cols);
  const int64_t c = i % cols;
  if (skip && skip[j]) return;
  double acc = 0.0;
  for (int t = 0; t < tiles; ++t) acc += part[(int64_t)t * len + i];
  Y[(int64_t)j * ldy + c] = acc;
}

template <class TA>
bool aligned16(const TA* A, int64_t lda) {
  return ((uintptr_t)A % 16 == 0) && ((lda * (int64_t)sizeof(TA)) % 16 == 0);
}

template <class TA, class TC, int VEC, int R, int K, int UNR = 1>
hipError_t gemv_t(hipStream_t st, const TA* A, int64_t rows, int64_t cols, int64_t lda, const double* X,
                  int64_t ldx, double* Y, int64_t ldy, int k, double lam, bool diag, const int32_t* skip,
                  double* dot_part, int* nblocks) {
  const int64_t blocks = (rows + R - 1) / R;
  const bool aln = aligned16(A, lda);
  for (int j0 = 0; j0 < k; j0 += K) {
    if (aln)
      hipLaunchKernelGGL((k_gemv<TA, TC, VEC, R, K, true, UNR>), dim3((unsigned)blocks), dim3(NT), 0, st, A, lda, rows,
                         cols, X, ldx, Y, ldy, k, j0, lam, diag ? 1 : 0, skip, dot_part, k);
    else
      hipLaunchKernelGGL((k_gemv<TA, TC, VEC, R, K, false, UNR>), dim3((unsigned)blocks), dim3(NT), 0, st, A, lda, rows,
                         cols, X, ldx, Y, ldy, k, j0, lam, diag ? 1 : 0, skip, dot_part, k);
  }
  if (nblocks) *nblocks = (int)blocks;
  return hipGetLastError();
}

template <class TA, class TC, int VEC>
hipError_t gemv_k(hipStream_t st, const TA* A, int64_t rows, int64_t cols, int64_t lda, const double* X,
                  int64_t ldx, double* Y, int64_t ldy, int k, double lam, bool diag, const int32_t* skip,
                  double* dot_part, int* nblocks) {
  if (k == 1) return gemv_t<TA, TC, VEC, 4, 1, 2>(st, A, rows, cols, lda, X, ldx, Y, ldy, k, lam, diag, skip, dot_part, nblocks);
  if (k == 2) return gemv_t<TA, TC, VEC, 8, 2>(st, A, rows, cols, lda, X, ldx, Y, ldy, k, lam, diag, skip, dot_part, nblocks);
  if (k <= 4) return gemv_t<TA, TC, VEC, 4, 4>(st, A, rows, cols, lda, X, ldx, Y, ldy, k, lam, diag, skip, dot_part, nblocks);
  return gemv_t<TA, TC, VEC, 4, 8>(st, A, rows, cols, lda, X, ldx, Y, ldy, k, lam, diag, skip, dot_part, nblocks);
}

template <class TA, class TC, int VEC>
hipError_t gemvT_k(hipStream_t st, const TA* A, int64_t rows, int64_t cols, int64_t lda, const double* X,
                   int64_t ldx, double* Y, int64_t ldy, int k, const int32_t* skip, double* part) {
  constexpr int K = 4;
  const int64_t ctiles = (cols + (int64_t)NT * VEC - 1) / ((int64_t)NT * VEC);
  int64_t rtiles = (2048 + ctiles - 1) / ctiles;
  if (rtiles > 64) rtiles = 64;
  if (rtiles > rows) rtiles = rows;
  const int64_t rpt = (rows + rtiles - 1) / rtiles;
  rtiles = (rows + rpt - 1) / rpt;
  const bool aln = aligned16(A, lda);
  for (int j0 = 0; j0 < k; j0 += K) {
    if (aln)
      hipLaunchKernelGGL((k_gemv_t<TA, TC, VEC, K, true>), dim3((unsigned)ctiles, (unsigned)rtiles), dim3(NT), 0, st,
                         A, lda, rows, cols, X, ldx, k, j0, rpt, part);
    else
      hipLaunchKernelGGL((k_gemv_t<TA, TC, VEC, K, false>), dim3((unsigned)ctiles, (unsigned)rtiles), dim3(NT), 0, st,
                         A, lda, rows, cols, X, ldx, k, j0, rpt, part);
  }
  const int64_t len = cols * k;
  hipLaunchKernelGGL(k_sum_tiles, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, part, (int)rtiles, cols, k,
                     skip, Y, ldy);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemv(hipStream_t st, const void* A, msp_dtype a_t, int64_t rows, int64_t cols, int64_t lda,
                       const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k, double lam,
                       bool diag_shift, const int32_t* skip, double* dot_part, int* nblocks) {
  const int kk = (int)k;
  switch (a_t) {
    case MSP_F64:
      return gemv_k<double, double, 2>(st, (const double*)A, rows, cols, lda, X, ldx, Y, ldy, kk, lam, diag_shift,
                                       skip, dot_part, nblocks);
    case MSP_F32:
      return gemv_k<float, float, 4>(st, (const float*)A, rows, cols, lda, X, ldx, Y, ldy, kk, lam, diag_shift,
                                     skip, dot_part, nblocks);
    case MSP_BF16:
      return gemv_k<__hip_bfloat16, float, 8>(st, (const __hip_bfloat16*)A, rows, cols, lda, X, ldx, Y, ldy, kk, lam,
                                              diag_shift, skip, dot_part, nblocks);
  }
  return hipErrorInvalidValue;
}

// FP64 arithmetic on FP32-stored A (the refinement residual on an FP32 A_hi)
hipError_t launch_gemv_f32_as_f64(hipStream_t st, const float* A, int64_t rows, int64_t cols, int64_t lda,
                                  const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k, double lam,
                                  bool diag_shift, const int32_t* skip, double* dot_part, int* nblocks) {
  return gemv_k<float, double, 4>(st, A, rows, cols, lda, X, ldx, Y, ldy, (int)k, lam, diag_shift, skip, dot_part,
                                  nblocks);
}

hipError_t launch_gemv_t_f32_as_f64(hipStream_t st, const float* A, int64_t rows, int64_t cols, int64_t lda,
                                    const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k,
                                    const int32_t* skip, double* part) {
  return gemvT_k<float, double, 4>(st, A, rows, cols, lda, X, ldx, Y, ldy, (int)k, skip, part);
}

size_t gemv_t_part_doubles(int64_t rows, int64_t cols, int64_t k) { return (size_t)64 * cols * k + 1024; }

hipError_t launch_gemv_t(hipStream_t st, const void* A, msp_dtype a_t, int64_t rows, int64_t cols, int64_t lda,
                         const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k, const int32_t* skip,
                         double* part) {
  const int kk = (int)k;
  switch (a_t) {
    case MSP_F64:
      return gemvT_k<double, double, 2>(st, (const double*)A, rows, cols, lda, X, ldx, Y, ldy, kk, skip, part);
    case MSP_F32:
      return gemvT_k<float, float, 4>(st, (const float*)A, rows, cols, lda, X, ldx, Y, ldy, kk, skip, part);
    case MSP_BF16:
      return gemvT_k<__hip_bfloat16, float, 8>(st, (const __hip_bfloat16*)A, rows, cols, lda, X, ldx, Y, ldy, kk,
                                               skip, part);
  }
  return hipErrorInvalidValue;
}
