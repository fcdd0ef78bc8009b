// Passes over the tall sketch Y (n x s, row-major): C^T v, C^T (C z), and C z, the
// products of the level-2 solve (Algorithm 2: C^T r, (C^T C + lam~ W) y, r - C y^) and
// of the level-2/3 solves of Algorithms 4-5 with A~ in place of C. One wavefront owns a
// whole row at a time (lane l holds columns l, l+64, ...), so row dots reduce inside the
// wavefront and column sums accumulate in registers; blocks emit fixed-order partials.
#include "msp_internal.h"

namespace {

constexpr int WAVE = 64;
constexpr int NT = 256;          // 4 wavefronts per block
constexpr int TALL_BLOCKS = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

template <class T>
__device__ __forceinline__ double ld(const T* p) { return (double)(*p); }

// part[b][j][c] = sum over rows of block b of Y[r, c] * V[r, j]
template <class TY, int CPL, int KG>
__global__ void __launch_bounds__(NT) k_yt_v(const TY* __restrict__ Y, int64_t n, int s, int64_t ldy,
                                            const double* __restrict__ V, int64_t ldv, int k, int j0,
                                            const int32_t* __restrict__ skip, double* __restrict__ part) {
  __shared__ double red[4][CPL * WAVE];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * per, r1 = min(n, r0 + per);
  double acc[KG][CPL];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int q = 0; q < CPL; ++q) acc[g][q] = 0.0;
  for (int64_t r = r0 + w; r < r1; r += 4) {
    double y[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane + q * WAVE;
      y[q] = (c < s) ? ld(Y + r * ldy + c) : 0.0;
    }
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      const int j = j0 + g;
      if (j >= k) break;
      const double v = V[(int64_t)j * ldv + r];
#pragma unroll
      for (int q = 0; q < CPL; ++q) acc[g][q] = fma(y[q], v, acc[g][q]);
    }
  }
  for (int g = 0; g < KG; ++g) {
    const int j = j0 + g;
    if (j >= k) break;
#pragma unroll
    for (int q = 0; q < CPL; ++q) red[w][q * WAVE + lane] = acc[g][q];
    __syncthreads();
    for (int c = threadIdx.x; c < s; c += NT) {
      const double v = red[0][c] + red[1][c] + red[2][c] + red[3][c];
      part[((int64_t)blockIdx.x * k + j) * s + c] = (skip && skip[j]) ? 0.0 : v;
    }
    __syncthreads();
  }
}

// part[b][j][c] = sum over rows of block b of Y[r, c] * (Y[r, :] . Z[:, j])
template <class TY, int CPL, int KG>
__global__ void __launch_bounds__(NT) k_yty_z(const TY* __restrict__ Y, int64_t n, int s, int64_t ldy,
                                             const double* __restrict__ Z, int k, int j0,
                                             const int32_t* __restrict__ skip, double* __restrict__ part) {
  __shared__ double red[4][CPL * WAVE];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * per, r1 = min(n, r0 + per);
  double z[KG][CPL], acc[KG][CPL];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane + q * WAVE;
      const int j = j0 + g;
      z[g][q] = (c < s && j < k) ? Z[(int64_t)j * s + c] : 0.0;
      acc[g][q] = 0.0;
    }
  for (int64_t r = r0 + w; r < r1; r += 4) {
    double y[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane + q * WAVE;
      y[q] = (c < s) ? ld(Y + r * ldy + c) : 0.0;
    }
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < CPL; ++q) t = fma(y[q], z[g][q], t);
      t = wave_sum(t);
#pragma unroll
      for (int q = 0; q < CPL; ++q) acc[g][q] = fma(y[q], t, acc[g][q]);
    }
  }
  for (int g = 0; g < KG; ++g) {
    const int j = j0 + g;
    if (j >= k) break;
#pragma unroll
    for (int q = 0; q < CPL; ++q) red[w][q * WAVE + lane] = acc[g][q];
    __syncthreads();
    for (int c = threadIdx.x; c < s; c += NT) {
      const double v = red[0][c] + red[1][c] + red[2][c] + red[3][c];
      part[((int64_t)blockIdx.x * k + j) * s + c] = (skip && skip[j]) ? 0.0 : v;
    }
    __syncthreads();
  }
}

// out[r, j] = a V[r, j] + b (Y[r, :] . Z[:, j]) ; one wavefront per row
template <class TY, int CPL, int KG>
__global__ void __launch_bounds__(NT) k_y_z(const TY* __restrict__ Y, int64_t n, int s, int64_t ldy,
                                           const double* __restrict__ Z, int k, int j0, double a,
                                           const double* __restrict__ V, int64_t ldv, double b,
                                           const int32_t* __restrict__ skip, double* __restrict__ out, int64_t ldo) {
  const int lane = threadIdx.x % WAVE;
  const int64_t wid = (blockIdx.x * (int64_t)NT + threadIdx.x) / WAVE;
  const int64_t nw = (int64_t)gridDim.x * NT / WAVE;
  double z[KG][CPL];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane + q * WAVE;
      const int j = j0 + g;
      z[g][q] = (c < s && j < k) ? Z[(int64_t)j * s + c] : 0.0;
    }
  for (int64_t r = wid; r < n; r += nw) {
    double y[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane + q * WAVE;
      y[q] = (c < s) ? ld(Y + r * ldy + c) : 0.0;
    }
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      const int j = j0 + g;
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < CPL; ++q) t = fma(y[q], z[g][q], t);
      t = wave_sum(t);
      if (lane == 0 && j < k && !(skip && skip[j])) {
        const double base = V ? a * V[(int64_t)j * ldv + r] : 0.0;
        out[(int64_t)j * ldo + r] = base + b * t;
      }
    }
  }
}

__global__ void k_reduce_parts(const double* __restrict__ part, int nparts, int64_t len, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= len) return;
  double acc = 0.0;
  for (int b = 0; b < nparts; ++b) acc += part[(int64_t)b * len + i];
  out[i] = acc;
}

// out[i, j] = sum_c M[i, c] V[c, j] ; one wavefront per row i
template <int CPL>
__global__ void __launch_bounds__(NT) k_small_mv(int s, const double* __restrict__ M, const double* __restrict__ V,
                                                int k, const int32_t* __restrict__ skip, double* __restrict__ out) {
  const int lane = threadIdx.x % WAVE;
  const int64_t i = (blockIdx.x * (int64_t)NT + threadIdx.x) / WAVE;
  if (i >= s) return;
  double m[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int c = lane + q * WAVE;
    m[q] = (c < s) ? M[i * s + c] : 0.0;
  }
  for (int j = 0; j < k; ++j) {
    if (skip && skip[j]) continue;
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane + q * WAVE;
      t = fma(m[q], (c < s) ? V[(int64_t)j * s + c] : 0.0, t);
    }
    t = wave_sum(t);
    if (lane == 0) out[(int64_t)j * s + i] = t;
  }
}

template <int CPL>
struct KGroup {
  static constexpr int value = (CPL >= 32) ? 1 : (CPL >= 16 ? 2 : 4);
};

template <class TY, int CPL>
hipError_t yt_v_t(hipStream_t st, const TY* Y, int64_t n, int s, int64_t ldy, const double* V, int64_t ldv, int k,
                  const int32_t* skip, double* part) {
  constexpr int KG = KGroup<CPL>::value;
  for (int j0 = 0; j0 < k; j0 += KG)
    hipLaunchKernelGGL((k_yt_v<TY, CPL, KG>), dim3(TALL_BLOCKS), dim3(NT), 0, st, Y, n, s, ldy, V, ldv, k, j0, skip,
                       part);
  return hipGetLastError();
}
template <class TY, int CPL>
hipError_t yty_z_t(hipStream_t st, const TY* Y, int64_t n, int s, int64_t ldy, const double* Z, int k,
                   const int32_t* skip, double* part) {
  constexpr int KG = KGroup<CPL>::value;
  for (int j0 = 0; j0 < k; j0 += KG)
    hipLaunchKernelGGL((k_yty_z<TY, CPL, KG>), dim3(TALL_BLOCKS), dim3(NT), 0, st, Y, n, s, ldy, Z, k, j0, skip,
                       part);
  return hipGetLastError();
}
template <class TY, int CPL>
hipError_t y_z_t(hipStream_t st, const TY* Y, int64_t n, int s, int64_t ldy, const double* Z, int k, double a,
                 const double* V, int64_t ldv, double b, const int32_t* skip, double* out, int64_t ldo) {
  constexpr int KG = KGroup<CPL>::value;
  if (k == 1) {
    // one column: no idle column groups, and a wavefront per row keeps every row's loads
    // in flight at once (the pass is one read of Y)
    const int64_t waves1 = n < 65536 ? n : 65536;
    const unsigned blocks1 = (unsigned)((waves1 * WAVE + NT - 1) / NT);
    hipLaunchKernelGGL((k_y_z<TY, CPL, 1>), dim3(blocks1), dim3(NT), 0, st, Y, n, s, ldy, Z, k, 0, a, V, ldv, b, skip,
                       out, ldo);
    return hipGetLastError();
  }
  const int64_t waves = n < 16384 ? n : 16384;
  const unsigned blocks = (unsigned)((waves * WAVE + NT - 1) / NT);
  for (int j0 = 0; j0 < k; j0 += KG)
    hipLaunchKernelGGL((k_y_z<TY, CPL, KG>), dim3(blocks), dim3(NT), 0, st, Y, n, s, ldy, Z, k, j0, a, V, ldv, b, skip,
                       out, ldo);
  return hipGetLastError();
}

#define MSP_CPL_DISPATCH(FN, TY, ...)                        \
  do {                                                       \
    const int cpl = (s + WAVE - 1) / WAVE;                   \
    if (cpl <= 1) return FN<TY, 1>(__VA_ARGS__);             \
    if (cpl <= 2) return FN<TY, 2>(__VA_ARGS__);             \
    if (cpl <= 4) return FN<TY, 4>(__VA_ARGS__);             \
    if (cpl <= 8) return FN<TY, 8>(__VA_ARGS__);             \
    if (cpl <= 16) return FN<TY, 16>(__VA_ARGS__);           \
    if (cpl <= 32) return FN<TY, 32>(__VA_ARGS__);           \
    return hipErrorInvalidValue;                             \
  } while (0)

}  // namespace

int tall_blocks(int64_t) { return TALL_BLOCKS; }

hipError_t launch_yt_v(hipStream_t st, const void* Y, msp_dtype y_t, int64_t n, int64_t s64, int64_t ldy,
                       const double* V, int64_t ldv, int64_t k, const int32_t* skip, double* part) {
  const int s = (int)s64;
  if (y_t == MSP_F64) MSP_CPL_DISPATCH(yt_v_t, double, st, (const double*)Y, n, s, ldy, V, ldv, (int)k, skip, part);
  MSP_CPL_DISPATCH(yt_v_t, float, st, (const float*)Y, n, s, ldy, V, ldv, (int)k, skip, part);
}

hipError_t launch_yty_z(hipStream_t st, const void* Y, msp_dtype y_t, int64_t n, int64_t s64, int64_t ldy,
                        const double* Z, int64_t k, const int32_t* skip, double* part) {
  const int s = (int)s64;
  if (y_t == MSP_F64) MSP_CPL_DISPATCH(yty_z_t, double, st, (const double*)Y, n, s, ldy, Z, (int)k, skip, part);
  MSP_CPL_DISPATCH(yty_z_t, float, st, (const float*)Y, n, s, ldy, Z, (int)k, skip, part);
}

hipError_t launch_y_z(hipStream_t st, const void* Y, msp_dtype y_t, int64_t n, int64_t s64, int64_t ldy,
                      const double* Z, int64_t k, double a, const double* V, int64_t ldv, double b,
                      const int32_t* skip, double* out, int64_t ldo) {
  const int s = (int)s64;
  if (y_t == MSP_F64)
    MSP_CPL_DISPATCH(y_z_t, double, st, (const double*)Y, n, s, ldy, Z, (int)k, a, V, ldv, b, skip, out, ldo);
  MSP_CPL_DISPATCH(y_z_t, float, st, (const float*)Y, n, s, ldy, Z, (int)k, a, V, ldv, b, skip, out, ldo);
}

hipError_t launch_reduce_parts(hipStream_t st, const double* part, int nparts, int64_t len, double* out) {
  hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, part, nparts, len, out);
  return hipGetLastError();
}

hipError_t launch_small_mv(hipStream_t st, int64_t s64, const double* M, const double* V, int64_t k,
                           const int32_t* skip, double* out) {
  const int s = (int)s64;
  const unsigned blocks = (unsigned)((s * (int64_t)WAVE + NT - 1) / NT);
  const int cpl = (s + WAVE - 1) / WAVE;
#define MV(C) hipLaunchKernelGGL(k_small_mv<C>, dim3(blocks), dim3(NT), 0, st, s, M, V, (int)k, skip, out)
  if (cpl <= 1) MV(1);
  else if (cpl <= 2) MV(2);
  else if (cpl <= 4) MV(4);
  else if (cpl <= 8) MV(8);
  else if (cpl <= 16) MV(16);
  else if (cpl <= 32) MV(32);
  else return hipErrorInvalidValue;
#undef MV
  return hipGetLastError();
}

namespace {

// 32 x 32 tiles through shared memory (padded against bank conflicts)
template <class TX>
__global__ void __launch_bounds__(256) k_transpose_f64(const TX* __restrict__ X, int64_t rows, int64_t cols,
                                                      int64_t ldx, double* __restrict__ out, int64_t ldo) {
  __shared__ double t[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8
  for (int q = ty; q < 32; q += 8) {
    const int64_t r = r0 + q, c = c0 + tx;
    t[q][tx] = (r < rows && c < cols) ? (double)X[r * ldx + c] : 0.0;
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {
    const int64_t c = c0 + q, r = r0 + tx;
    if (c < cols && r < rows) out[c * ldo + r] = t[tx][q];
  }
}

}  // namespace

hipError_t launch_transpose_f64(hipStream_t st, const void* X, msp_dtype x_t, int64_t rows, int64_t cols,
                                int64_t ldx, double* out, int64_t ldo) {
  dim3 grd((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  if (x_t == MSP_F64)
    hipLaunchKernelGGL(k_transpose_f64<double>, grd, dim3(256), 0, st, (const double*)X, rows, cols, ldx, out, ldo);
  else if (x_t == MSP_F32)
    hipLaunchKernelGGL(k_transpose_f64<float>, grd, dim3(256), 0, st, (const float*)X, rows, cols, ldx, out, ldo);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
