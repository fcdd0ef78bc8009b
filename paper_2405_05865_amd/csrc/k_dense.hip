// Small dense FP64 work on s x s matrices: the Gram products C~^T C~ and A^^T A^
// (Algorithms 1 and 3), symmetric combinations, and the explicit
// SPD inverses M2^{-1}, M3a^{-1}, M3b^{-1} the algorithms precompute.
//
// The inverse is computed by block Gauss-Jordan sweeps without pivoting. For SPD M
// every pivot block is a Schur complement of M, hence SPD, so no pivoting is needed;
// each pivot block is factored by Cholesky (a non-positive pivot flags the matrix as
// not positive definite) and the Schur complements are formed in Cholesky form.
#include "msp_internal.h"

#include <hip/hip_bf16.h>

namespace {

constexpr int TILE = 64;
constexpr int KCH = 16;

// Gram partial: G_part[z] = X[rows of split z]^T X[rows of split z], lower tiles, mirrored
template <class T>
__global__ void __launch_bounds__(256) k_gram(const T* __restrict__ X, int64_t rows, int64_t s, int64_t ldx,
                                              int64_t rows_per_split, double* __restrict__ Gp) {
  // map blockIdx.x to a lower tile (ti >= tj)
  int t = blockIdx.x, ti = 0;
  while (t > ti) { t -= ti + 1; ++ti; }
  const int tj = t;
  const int64_t i0 = (int64_t)ti * TILE, j0 = (int64_t)tj * TILE;
  const int64_t rb = (int64_t)blockIdx.y * rows_per_split;
  const int64_t re = min(rows, rb + rows_per_split);
  __shared__ double As[KCH][TILE + 1];
  __shared__ double Bs[KCH][TILE + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int64_t k0 = rb; k0 < re; k0 += KCH) {
    for (int e = threadIdx.x; e < KCH * TILE; e += 256) {
      const int kk = e / TILE, c = e % TILE;
      const int64_t r = k0 + kk;
      As[kk][c] = (r < re && i0 + c < s) ? (double)X[r * ldx + i0 + c] : 0.0;
      Bs[kk][c] = (r < re && j0 + c < s) ? (double)X[r * ldx + j0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KCH; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty * 4 + q];
        b[q] = Bs[kk][tx * 4 + q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
    }
    __syncthreads();
  }
  double* G = Gp + (int64_t)blockIdx.y * s * s;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = i0 + ty * 4 + p, j = j0 + tx * 4 + q;
      if (i < s && j < s) {
        G[i * s + j] = acc[p][q];
        G[j * s + i] = acc[p][q];
      }
    }
}

__global__ void k_sum_splits(const double* __restrict__ Gp, int splits, int64_t len, double* __restrict__ G) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= len) return;
  double acc = 0.0;
  for (int z = 0; z < splits; ++z) acc += Gp[(int64_t)z * len + i];
  G[i] = acc;
}

// out = sym(a P + b Q) + c I, one thread per unordered pair (safe in place)
__global__ void k_combine_sym(int64_t s, double a, const double* P, double b, const double* Q, double c,
                              double* out) {
  const int64_t i = blockIdx.y * (int64_t)blockDim.y + threadIdx.y;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= s || j >= s || j > i) return;
  double v = 0.5 * a * (P[i * s + j] + P[j * s + i]);
  if (Q) v += 0.5 * b * (Q[i * s + j] + Q[j * s + i]);
  if (i == j) v += c;
  out[i * s + j] = v;
  out[j * s + i] = v;
}

__global__ void k_trace(int64_t s, const double* __restrict__ M, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < s; i += 256) acc += M[i * s + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_add_diag_scaled(int64_t s, double* M, const double* tr, double rel) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < s) M[i * s + i] += rel * (*tr) / (double)s;
}

// One block Gauss-Jordan sweep over pivots K = [k0, k0 + nbk). Tile of 64 x 64 per block.
// The pivot block is factored X_KK = L L^T (Cholesky, in shared memory; a pivot <= 0
// flags the matrix as not positive definite) and every product with X_KK^{-1} is taken
// through Li = L^{-1}:
//   X_KK <- Li^T Li,  X_KJ <- Li^T (Li X_KJ),  X_IK <- -(X_IK Li^T) Li,
//   X_IJ <- X_IJ - (X_IK Li^T)(Li X_KJ).
// The trailing update is then the Cholesky form of the Schur complement, whose error
// does not grow with the conditioning of X_KK (an explicit inverse of the pivot block
// there would lose the small trailing pivots of ill-conditioned SPD matrices).
template <int NB>
__global__ void __launch_bounds__(256) k_bgj_step(const double* __restrict__ in, double* __restrict__ out, int s,
                                                  int k0, int32_t* status) {
  __shared__ double L[NB][NB + 1];     // pivot block, then its Cholesky factor
  __shared__ double Li[NB][NB + 1];    // L^{-1}
  __shared__ double Lk[TILE][NB + 1];  // X[I, K], then X[I, K] Li^T
  __shared__ double Uk[NB][TILE + 1];  // X[K, J], then Li X[K, J]
  __shared__ int bad;
  const int nbk = min(NB, s - k0);
  const int I = blockIdx.y * TILE, J = blockIdx.x * TILE;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int e = t; e < NB * NB; e += 256) {
    const int a = e / NB, b = e % NB;
    L[a][b] = (a < nbk && b < nbk) ? in[(int64_t)(k0 + a) * s + k0 + b] : (a == b ? 1.0 : 0.0);
    Li[a][b] = 0.0;
  }
  for (int e = t; e < TILE * NB; e += 256) {
    const int a = e / NB, b = e % NB;
    const int i = I + a;
    Lk[a][b] = (i < s && b < nbk) ? in[(int64_t)i * s + k0 + b] : 0.0;
  }
  for (int e = t; e < NB * TILE; e += 256) {
    const int a = e / TILE, b = e % TILE;
    const int j = J + b;
    Uk[a][b] = (j < s && a < nbk) ? in[(int64_t)(k0 + a) * s + j] : 0.0;
  }
  __syncthreads();
  // Cholesky of the pivot block (lower triangle)
  for (int p = 0; p < NB; ++p) {
    if (t == 0) {
      const double d = L[p][p];
      if (!(d > 0.0)) bad = 1;
      L[p][p] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    if (t > p && t < NB) L[t][p] /= L[p][p];
    __syncthreads();
    for (int e = t; e < NB * NB; e += 256) {
      const int i = e / NB, j = e % NB;
      if (j > p && i >= j) L[i][j] -= L[i][p] * L[j][p];
    }
    __syncthreads();
  }
  if (t == 0 && bad && blockIdx.x == 0 && blockIdx.y == 0) *status = 1;
  // Li = L^{-1} (column c by thread c, forward substitution)
  if (t < NB) {
    const int c = t;
    for (int i = c; i < NB; ++i) {
      double acc = (i == c) ? 1.0 : 0.0;
      for (int j = c; j < i; ++j) acc -= L[i][j] * Li[j][c];
      Li[i][c] = acc / L[i][i];
    }
  }
  __syncthreads();
  // Uk <- Li Uk ; Lk <- Lk Li^T   (results staged in registers)
  {
    constexpr int PER = (NB * TILE + 255) / 256;
    double tu[PER], tl[PER];
    int q = 0;
    for (int e = t; e < NB * TILE; e += 256, ++q) {
      const int a = e / TILE, b = e % TILE;  // Uk row a, column b
      double acc = 0.0;
      for (int c = 0; c <= a; ++c) acc = fma(Li[a][c], Uk[c][b], acc);
      tu[q] = acc;
      const int r = e / NB, cc = e % NB;  // Lk row r, column cc
      double acl = 0.0;
      for (int c = 0; c <= cc; ++c) acl = fma(Lk[r][c], Li[cc][c], acl);
      tl[q] = acl;
    }
    __syncthreads();
    q = 0;
    for (int e = t; e < NB * TILE; e += 256, ++q) {
      Uk[e / TILE][e % TILE] = tu[q];
      Lk[e / NB][e % NB] = tl[q];
    }
    __syncthreads();
  }
  const bool rows_hit = (I < k0 + nbk) && (I + TILE > k0);
  const bool cols_hit = (J < k0 + nbk) && (J + TILE > k0);
  for (int e = t; e < TILE * TILE; e += 256) {
    const int a = e / TILE, b = e % TILE;
    const int i = I + a, j = J + b;
    if (i >= s || j >= s) continue;
    const bool ik = rows_hit && i >= k0 && i < k0 + nbk;
    const bool jk = cols_hit && j >= k0 && j < k0 + nbk;
    double v = 0.0;
    if (ik && jk) {
      for (int c = 0; c < NB; ++c) v = fma(Li[c][i - k0], Li[c][j - k0], v);
    } else if (ik) {
      for (int c = 0; c < NB; ++c) v = fma(Li[c][i - k0], Uk[c][b], v);
    } else if (jk) {
      for (int c = 0; c < NB; ++c) v = fma(Lk[a][c], Li[c][j - k0], v);
      v = -v;
    } else {
      for (int c = 0; c < NB; ++c) v = fma(Lk[a][c], Uk[c][b], v);
      v = in[(int64_t)i * s + j] - v;
    }
    out[(int64_t)i * s + j] = v;
  }
}

__global__ void k_copy(int64_t len, const double* __restrict__ a, double* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < len) b[i] = a[i];
}

// symmetrise the final inverse (rounding leaves it nearly symmetric)
__global__ void k_sym_avg(int64_t s, double* M) {
  const int64_t i = blockIdx.y * (int64_t)blockDim.y + threadIdx.y;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= s || j >= s || j >= i) return;
  const double v = 0.5 * (M[i * s + j] + M[j * s + i]);
  M[i * s + j] = v;
  M[j * s + i] = v;
}

// out[slot] = sum_i A[i, i] in FP64 (one block, fixed order)
template <class T>
__global__ void __launch_bounds__(256) k_diag_sum(const T* __restrict__ A, int64_t n, int64_t lda, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += (double)A[i * lda + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// the estimate (2/l) max(tr A - <Winv, C^T C>_F, 0) with tr A already in scal[0]; the
// Frobenius product in one block of 1024 threads in a fixed order; scal[1] = <Winv, C^T C>_F,
// scal[2] = the estimate
__global__ void __launch_bounds__(1024) k_lambda0_est(const double* __restrict__ Winv, const double* __restrict__ CtC,
                                                      int64_t len, double l, double* scal) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += 1024) acc = fma(Winv[i], CtC[i], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scal[1] = red[0];
    const double deficit = scal[0] - red[0];
    // below 1e-6 tr A: the mu bias and rounding of an exact recovery (rank A <= s), taken as 0
    scal[2] = deficit > 1e-6 * scal[0] ? (2.0 / l) * deficit : 0.0;
  }
}

}  // namespace

hipError_t launch_diag_sum(hipStream_t st, const void* A, msp_dtype t, int64_t n, int64_t lda, double* out) {
  if (t == MSP_F64)
    hipLaunchKernelGGL(k_diag_sum<double>, dim3(1), dim3(256), 0, st, (const double*)A, n, lda, out);
  else if (t == MSP_F32)
    hipLaunchKernelGGL(k_diag_sum<float>, dim3(1), dim3(256), 0, st, (const float*)A, n, lda, out);
  else
    hipLaunchKernelGGL(k_diag_sum<__hip_bfloat16>, dim3(1), dim3(256), 0, st, (const __hip_bfloat16*)A, n, lda,
                       out);
  return hipGetLastError();
}

hipError_t launch_lambda0_est(hipStream_t st, const double* Winv, const double* CtC, int64_t s, double l,
                              double* scal) {
  hipLaunchKernelGGL(k_lambda0_est, dim3(1), dim3(1024), 0, st, Winv, CtC, s * s, l, scal);
  return hipGetLastError();
}

template <class T>
hipError_t gram_t(hipStream_t st, const T* X, int64_t rows, int64_t s, int64_t ldx, double* G, double* part,
                  int splits) {
  const int nt = (int)((s + TILE - 1) / TILE);
  const int tiles = nt * (nt + 1) / 2;
  const int64_t rps = ((rows + splits - 1) / splits + KCH - 1) / KCH * KCH;
  double* dst = (splits == 1) ? G : part;
  hipLaunchKernelGGL(k_gram<T>, dim3(tiles, splits), dim3(256), 0, st, X, rows, s, ldx, rps, dst);
  if (splits > 1) {
    const int64_t len = s * s;
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, part, splits, len, G);
  }
  return hipGetLastError();
}

hipError_t launch_gram(hipStream_t st, const double* X, int64_t rows, int64_t s, int64_t ldx, double* G,
                       double* part, int splits) {
  return gram_t<double>(st, X, rows, s, ldx, G, part, splits);
}

hipError_t launch_gram_f32(hipStream_t st, const float* X, int64_t rows, int64_t s, int64_t ldx, double* G,
                           double* part, int splits) {
  return gram_t<float>(st, X, rows, s, ldx, G, part, splits);
}

int gram_splits(int64_t rows, int64_t s) {
  const int nt = (int)((s + TILE - 1) / TILE);
  const int tiles = nt * (nt + 1) / 2;
  int splits = (512 + tiles - 1) / tiles;
  const int64_t max_by_rows = (rows + 255) / 256;
  if (splits > max_by_rows) splits = (int)max_by_rows;
  if (splits < 1) splits = 1;
  if (splits > 16) splits = 16;
  return splits;
}

hipError_t launch_combine_sym(hipStream_t st, int64_t s, double a, const double* P, double b, const double* Q,
                              double c, double* out) {
  dim3 blk(16, 16), grd((unsigned)((s + 15) / 16), (unsigned)((s + 15) / 16));
  hipLaunchKernelGGL(k_combine_sym, grd, blk, 0, st, s, a, P, b, Q, c, out);
  return hipGetLastError();
}

hipError_t launch_symmetrize(hipStream_t st, int64_t s, double* Wm) {
  return launch_combine_sym(st, s, 1.0, Wm, 0.0, nullptr, 0.0, Wm);
}

hipError_t launch_trace(hipStream_t st, int64_t s, const double* M, double* out) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, st, s, M, out);
  return hipGetLastError();
}

hipError_t spd_inverse(hipStream_t st, int64_t s, double* M, double* tmp, double shift_rel, double* scal,
                       int32_t* status) {
  constexpr int NB = 32;
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, st, s, M, scal);
  hipLaunchKernelGGL(k_add_diag_scaled, dim3((unsigned)((s + 255) / 256)), dim3(256), 0, st, s, M, scal, shift_rel);
  const int nt = (int)((s + TILE - 1) / TILE);
  double* a = M;
  double* b = tmp;
  for (int k0 = 0; k0 < s; k0 += NB) {
    hipLaunchKernelGGL(k_bgj_step<NB>, dim3(nt, nt), dim3(256), 0, st, a, b, (int)s, k0, status);
    double* t = a;
    a = b;
    b = t;
  }
  if (a != M) {
    const int64_t len = s * s;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, len, a, M);
  }
  dim3 blk(16, 16), grd((unsigned)((s + 15) / 16), (unsigned)((s + 15) / 16));
  hipLaunchKernelGGL(k_sym_avg, grd, blk, 0, st, s, M);
  return hipGetLastError();
}
