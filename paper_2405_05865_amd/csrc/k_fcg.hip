// Flexible PCG (Polak-Ribiere beta) as a device-resident state machine. Each level
// of the method (Algorithm 1/3 level 1, Algorithms 2/4 level 2, Algorithm 5 level 3)
// runs the same five kernels on its own vectors and scalars; no host round trip is
// needed per step. Column j of a block iterates independently and stops on its own
// residual; finished columns are skipped by every kernel.
#include "msp_internal.h"

#include <algorithm>

namespace {

constexpr int NT = 256;
constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// sum of v over the block (valid in thread 0)
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < NT / WAVE; ++q) t += sh[q];
  return t;
}

// sum of v over the block, valid in every thread
__device__ __forceinline__ double block_sum_all(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < NT / WAVE; ++q) t += sh[q];
  __syncthreads();
  return t;
}

// true in every thread of the last block of the grid to reach this point
__device__ __forceinline__ bool last_block(int32_t* counter) {
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int total = gridDim.x * gridDim.y;
    const int t = atomicAdd(counter, 1);
    is_last = (t == total - 1);
  }
  __syncthreads();
  if (is_last) __threadfence();
  return is_last != 0;
}

__device__ __forceinline__ void count_active(FcgState S, int32_t* mirror) {
  // called by the last block; all threads participate
  __shared__ int cnt, mx;
  if (threadIdx.x == 0) {
    cnt = 0;
    mx = 0;
  }
  __syncthreads();
  int mine = 0, it = 0;
  for (int64_t j = threadIdx.x; j < S.k; j += NT) {
    mine += (S.done[j] == 0);
    it = max(it, S.iters[j]);
  }
  atomicAdd(&cnt, mine);
  atomicMax(&mx, it);
  __syncthreads();
  if (threadIdx.x == 0) {
    *S.active = cnt;
    if (mirror) {
      // mirror[0] = columns still iterating, mirror[1] = most iterations taken; the host
      // reads them only after synchronising the stream, which orders them (no fence here)
      __hip_atomic_store(mirror, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(mirror + 1, mx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    *S.counter = 0;
  }
}

// fixed-order parallel sum of part[b * stride] over b < count; valid in every thread
__device__ __forceinline__ double strided_sum(const double* base, int count, int64_t stride, double* sh) {
  double t = 0.0;
  for (int b = threadIdx.x; b < count; b += NT) t += base[(int64_t)b * stride];
  return block_sum_all(t, sh);
}

__device__ __forceinline__ int64_t chunk_begin(int64_t len) {
  const int64_t per = (len + gridDim.x - 1) / gridDim.x;
  return blockIdx.x * per;
}
__device__ __forceinline__ int64_t chunk_end(int64_t len) {
  const int64_t per = (len + gridDim.x - 1) / gridDim.x;
  return min(len, (int64_t)(blockIdx.x + 1) * per);
}

__global__ void __launch_bounds__(NT) k_init(FcgState S, int64_t len, const double* __restrict__ b, int64_t ldb,
                                            double* __restrict__ r, double* __restrict__ x,
                                            const int32_t* __restrict__ parent_done, int32_t* mirror) {
  __shared__ double sh[NT / WAVE];
  const int j = blockIdx.y;
  const bool pd = parent_done && parent_done[j] != 0;
  double acc = 0.0;
  for (int64_t i = chunk_begin(len) + threadIdx.x; i < chunk_end(len); i += NT) {
    const double v = pd ? 0.0 : b[(int64_t)j * ldb + i];
    r[(int64_t)j * len + i] = v;
    if (x) x[(int64_t)j * len + i] = 0.0;
    acc = fma(v, v, acc);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) S.part[(int64_t)blockIdx.x * S.k + j] = t;
  if (!last_block(S.counter)) return;
  for (int64_t jj = 0; jj < S.k; ++jj) {
    const double sum = strided_sum(S.part + jj, gridDim.x, S.k, sh);
    if (threadIdx.x != 0) continue;
    const double bn = sqrt(sum);
    const bool p = parent_done && parent_done[jj] != 0;
    S.bnorm[jj] = bn;
    S.rnorm[jj] = bn;
    S.iters[jj] = 0;
    S.rz[jj] = 0.0;
    S.alpha[jj] = 0.0;
    S.beta[jj] = 0.0;
    S.done[jj] = (p || bn == 0.0) ? 1 : 0;
  }
  __syncthreads();
  count_active(S, mirror);
}

__global__ void __launch_bounds__(NT) k_first_dir(FcgState S, int64_t len, const double* __restrict__ r,
                                                 const double* __restrict__ z, double* __restrict__ p) {
  __shared__ double sh[NT / WAVE];
  const int j = blockIdx.y;
  const bool live = S.done[j] == 0;
  double acc = 0.0;
  if (live)
    for (int64_t i = chunk_begin(len) + threadIdx.x; i < chunk_end(len); i += NT) {
      const int64_t o = (int64_t)j * len + i;
      const double zv = z[o];
      p[o] = zv;
      acc = fma(r[o], zv, acc);
    }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) S.part[(int64_t)blockIdx.x * S.k + j] = t;
  if (!last_block(S.counter)) return;
  for (int64_t jj = 0; jj < S.k; ++jj) {
    if (S.done[jj] != 0) continue;
    const double sum = strided_sum(S.part + jj, gridDim.x, S.k, sh);
    if (threadIdx.x == 0) S.rz[jj] = sum;
  }
  if (threadIdx.x == 0) *S.counter = 0;
}

__global__ void k_alpha_parts(FcgState S, const double* __restrict__ pq_part, int nparts) {
  for (int64_t j = threadIdx.x; j < S.k; j += blockDim.x) {
    if (S.done[j] != 0) {
      S.alpha[j] = 0.0;
      continue;
    }
    double pq = 0.0;
    for (int b = 0; b < nparts; ++b) pq += pq_part[(int64_t)b * S.k + j];
    if (!(pq > 0.0)) {
      S.done[j] = 2;
      S.alpha[j] = 0.0;
    } else {
      S.alpha[j] = S.rz[j] / pq;
    }
  }
}

// one block per column: alpha = rz / <p, q>
__global__ void __launch_bounds__(NT) k_alpha_dot(FcgState S, int64_t len, const double* __restrict__ p,
                                                 const double* __restrict__ q) {
  __shared__ double sh[NT / WAVE];
  const int j = blockIdx.x;
  if (S.done[j] != 0) {
    if (threadIdx.x == 0) S.alpha[j] = 0.0;
    return;
  }
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += NT) acc = fma(p[(int64_t)j * len + i], q[(int64_t)j * len + i], acc);
  const double pq = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    if (!(pq > 0.0)) {
      S.done[j] = 2;
      S.alpha[j] = 0.0;
    } else {
      S.alpha[j] = S.rz[j] / pq;
    }
  }
}

__global__ void __launch_bounds__(NT) k_update(FcgState S, int64_t len, double* __restrict__ x,
                                              double* __restrict__ r, double* __restrict__ r_old,
                                              const double* __restrict__ p, const double* __restrict__ q, double tol,
                                              int32_t max_iter, int32_t* mirror, const double* __restrict__ pq_part,
                                              int nparts, int decide) {
  __shared__ double sh[NT / WAVE];
  const int j = blockIdx.y;
  const bool live = S.done[j] == 0;
  double acc = 0.0;
  if (live) {
    double a;
    if (pq_part) {
      double t = 0.0;
      for (int b = threadIdx.x; b < nparts; b += NT) t += pq_part[(int64_t)b * S.k + j];
      const double pq = block_sum_all(t, sh);
      a = (pq > 0.0) ? S.rz[j] / pq : 0.0;
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        S.alpha[j] = a;
        S.brk[j] = (pq > 0.0) ? 0 : 1;
      }
    } else {
      a = S.alpha[j];
    }
    for (int64_t i = chunk_begin(len) + threadIdx.x; i < chunk_end(len); i += NT) {
      const int64_t o = (int64_t)j * len + i;
      x[o] = fma(a, p[o], x[o]);
      const double rv = r[o];
      r_old[o] = rv;
      const double rn = fma(-a, q[o], rv);
      r[o] = rn;
      acc = fma(rn, rn, acc);
    }
  }
  if (!decide) return;
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) S.part[(int64_t)blockIdx.x * S.k + j] = t;
}

// the decision after k_update, in one block (a separate launch instead of a last-block
// hand-off: a device-scope fence in every block of the update costs more than a launch):
// |r| from the nblocks partials, breakdown, tolerance, iteration cap; mirror <- active
__global__ void __launch_bounds__(NT) k_decide(FcgState S, int nblocks, double tol, int32_t max_iter,
                                              int32_t* mirror, int check_brk) {
  __shared__ double sh[NT / WAVE];
  for (int64_t jj = 0; jj < S.k; ++jj) {
    if (S.done[jj] != 0) continue;  // uniform in the block
    const double sum = strided_sum(S.part + jj, nblocks, S.k, sh);
    if (threadIdx.x != 0) continue;
    if (check_brk && S.brk[jj]) {
      S.done[jj] = 2;
      continue;
    }
    const double rn = sqrt(sum);
    S.rnorm[jj] = rn;
    const int it = S.iters[jj] + 1;
    S.iters[jj] = it;
    if (!(rn == rn)) S.done[jj] = 2;  // NaN
    else if (rn <= tol * S.bnorm[jj]) S.done[jj] = 1;
    else if (it >= max_iter) S.done[jj] = 3;
  }
  __syncthreads();
  count_active(S, mirror);
}

__global__ void __launch_bounds__(NT) k_beta(FcgState S, int64_t len, const double* __restrict__ r,
                                            const double* __restrict__ r_old, const double* __restrict__ z) {
  __shared__ double sh[NT / WAVE];
  const int j = blockIdx.y;
  const bool live = S.done[j] == 0;
  double a1 = 0.0, a2 = 0.0;
  if (live)
    for (int64_t i = chunk_begin(len) + threadIdx.x; i < chunk_end(len); i += NT) {
      const int64_t o = (int64_t)j * len + i;
      const double zv = z[o];
      a1 = fma(zv, r[o], a1);
      a2 = fma(zv, r_old[o], a2);
    }
  const double t1 = block_sum(a1, sh);
  const double t2 = block_sum(a2, sh);
  if (threadIdx.x == 0) {
    S.part[((int64_t)blockIdx.x * S.k + j) * 2 + 0] = t1;
    S.part[((int64_t)blockIdx.x * S.k + j) * 2 + 1] = t2;
  }
}

// beta = <z, r - r_old> / rz and rz = <z, r> from the partials of k_beta, in one block (a
// separate launch instead of a fenced last-block hand-off). When the denominator
// rz = <r_old, z_old> is zero or not finite no conjugate direction exists (an inexact
// preconditioner that is not positive definite): the column stops as a breakdown and
// keeps its iterate; k_pupdate then leaves p alone and the next decision recounts the
// active columns.
__global__ void __launch_bounds__(NT) k_beta_fin(FcgState S, int nblocks) {
  __shared__ double sh[NT / WAVE];
  for (int64_t jj = 0; jj < S.k; ++jj) {
    if (S.done[jj] != 0) continue;
    const double zr = strided_sum(S.part + jj * 2 + 0, nblocks, S.k * 2, sh);
    const double zro = strided_sum(S.part + jj * 2 + 1, nblocks, S.k * 2, sh);
    if (threadIdx.x == 0) {
      const double rz = S.rz[jj];
      if (rz != 0.0 && isfinite(rz)) {
        S.beta[jj] = (zr - zro) / rz;
        S.rz[jj] = zr;
      } else {
        S.beta[jj] = 0.0;
        S.done[jj] = 2;
      }
    }
  }
}

__global__ void __launch_bounds__(NT) k_pupdate(FcgState S, int64_t len, const double* __restrict__ z,
                                               double* __restrict__ p) {
  const int j = blockIdx.y;
  if (S.done[j] != 0) return;
  const double bt = S.beta[j];
  for (int64_t i = chunk_begin(len) + threadIdx.x; i < chunk_end(len); i += NT) {
    const int64_t o = (int64_t)j * len + i;
    p[o] = fma(bt, p[o], z[o]);
  }
}

__global__ void __launch_bounds__(NT) k_confirm(FcgState S, int64_t len, const double* __restrict__ rtrue,
                                               double* __restrict__ r, double tol, double* relres, int32_t* mirror) {
  __shared__ double sh[NT / WAVE];
  const int j = blockIdx.y;
  double acc = 0.0;
  for (int64_t i = chunk_begin(len) + threadIdx.x; i < chunk_end(len); i += NT) {
    const double v = rtrue[(int64_t)j * len + i];
    acc = fma(v, v, acc);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) S.part[(int64_t)blockIdx.x * S.k + j] = t;
  __shared__ int restart;
  const bool last = last_block(S.counter);
  if (!last) return;
  __syncthreads();
  for (int64_t jj = 0; jj < S.k; ++jj) {
    const double sum = strided_sum(S.part + jj, gridDim.x, S.k, sh);
    if (threadIdx.x != 0) continue;
    const double bn = S.bnorm[jj];
    const double rel = bn > 0.0 ? sqrt(sum) / bn : 0.0;
    relres[jj] = rel;
    if (S.done[jj] == 1) S.done[jj] = (rel <= tol) ? 4 : 0;
  }
  __syncthreads();
  // restarted columns take the recomputed residual
  (void)restart;
  for (int64_t jj = 0; jj < S.k; ++jj) {
    if (S.done[jj] != 0) continue;
    for (int64_t i = threadIdx.x; i < len; i += NT) r[jj * len + i] = rtrue[jj * len + i];
  }
  __syncthreads();
  count_active(S, mirror);
}

__global__ void k_axpby(int64_t len, int k, double a, const double* __restrict__ x, int64_t ldx, double b,
                        const double* __restrict__ y, int64_t ldy, double* __restrict__ out, int64_t ldo,
                        const int32_t* __restrict__ skip) {
  const int j = blockIdx.y;
  if (skip && skip[j]) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    double v = a * x[(int64_t)j * ldx + i];
    if (y) v = fma(b, y[(int64_t)j * ldy + i], v);
    out[(int64_t)j * ldo + i] = v;
  }
}

__global__ void __launch_bounds__(NT) k_coldot(int64_t len, const double* __restrict__ x, int64_t ldx,
                                              const double* __restrict__ y, int64_t ldy, double* out) {
  __shared__ double sh[NT / WAVE];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += NT) acc = fma(x[(int64_t)j * ldx + i], y[(int64_t)j * ldy + i], acc);
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[j] = t;
}

__global__ void k_outer_neg(int64_t n, int k, const double* __restrict__ dB, int64_t lddb,
                            const double* __restrict__ X, int64_t ldx, double* __restrict__ dA, int64_t ldda) {
  for (int64_t i = blockIdx.y; i < n; i += gridDim.y)
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
      double acc = 0.0;
      for (int j = 0; j < k; ++j) acc = fma(dB[(int64_t)j * lddb + i], X[(int64_t)j * ldx + c], acc);
      dA[i * ldda + c] = -acc;
    }
}

// part[b] = max over the rows of block b (a wavefront per row, rows strided by the grid)
// of sum_j |A[i, j]| in FP64; a max is exact, so the result does not depend on the grid
template <class TA>
__global__ void __launch_bounds__(NT) k_row_abs_max(const TA* __restrict__ A, int64_t rows, int64_t cols, int64_t lda,
                                                   double* part) {
  __shared__ double sh[NT / WAVE];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  double mx = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * (NT / WAVE) + w; r < rows; r += (int64_t)gridDim.x * (NT / WAVE)) {
    const TA* row = A + r * lda;
    double t0 = 0.0, t1 = 0.0;
    int64_t c = lane;
    for (; c + WAVE < cols; c += 2 * WAVE) {
      t0 += fabs((double)row[c]);
      t1 += fabs((double)row[c + WAVE]);
    }
    if (c < cols) t0 += fabs((double)row[c]);
    mx = fmax(mx, wave_sum(t0 + t1));
  }
  if (lane == 0) sh[w] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int q = 0; q < NT / WAVE; ++q) m = fmax(m, sh[q]);
    part[blockIdx.x] = m;
  }
}

__global__ void __launch_bounds__(NT) k_max_parts(const double* __restrict__ part, int nparts, double* out) {
  __shared__ double sh[NT];
  double m = 0.0;
  for (int b = threadIdx.x; b < nparts; b += NT) m = fmax(m, part[b]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

unsigned grid_x(int64_t len) {
  int64_t b = (len + NT * 2 - 1) / (NT * 2);
  if (b < 1) b = 1;
  if (b > 256) b = 256;
  return (unsigned)b;
}

}  // namespace

size_t fcg_part_doubles(int64_t len, int64_t k) { return (size_t)grid_x(len) * k * 2 + 64; }

FcgState carve_fcg_state(WsCarver& w, int64_t len, int64_t k) {
  FcgState S;
  S.k = k;
  S.rz = w.take<double>(k);
  S.alpha = w.take<double>(k);
  S.beta = w.take<double>(k);
  S.bnorm = w.take<double>(k);
  S.rnorm = w.take<double>(k);
  S.done = w.take<int32_t>(k);
  S.iters = w.take<int32_t>(k);
  S.active = w.take<int32_t>(1);
  S.counter = w.take<int32_t>(1);
  S.part = w.take<double>(fcg_part_doubles(len, k));
  S.brk = w.take<int32_t>(k);
  S.done_next = w.take<int32_t>(k);
  S.iters_next = w.take<int32_t>(k);
  return S;
}

hipError_t fcg_init(hipStream_t st, FcgState S, int64_t len, const double* b, int64_t ldb, double* r, double* x,
                    const int32_t* parent_done, int32_t* mirror) {
  hipLaunchKernelGGL(k_init, dim3(grid_x(len), (unsigned)S.k), dim3(NT), 0, st, S, len, b, ldb, r, x, parent_done,
                     mirror);
  return hipGetLastError();
}
hipError_t fcg_first_dir(hipStream_t st, FcgState S, int64_t len, const double* r, const double* z, double* p) {
  hipLaunchKernelGGL(k_first_dir, dim3(grid_x(len), (unsigned)S.k), dim3(NT), 0, st, S, len, r, z, p);
  return hipGetLastError();
}
hipError_t fcg_alpha_parts(hipStream_t st, FcgState S, const double* pq_part, int nparts) {
  hipLaunchKernelGGL(k_alpha_parts, dim3(1), dim3(NT), 0, st, S, pq_part, nparts);
  return hipGetLastError();
}
hipError_t fcg_alpha_dot(hipStream_t st, FcgState S, int64_t len, const double* p, const double* q) {
  hipLaunchKernelGGL(k_alpha_dot, dim3((unsigned)S.k), dim3(NT), 0, st, S, len, p, q);
  return hipGetLastError();
}
hipError_t fcg_update(hipStream_t st, FcgState S, int64_t len, double* x, double* r, double* r_old, const double* p,
                      const double* q, double tol, int32_t max_iter, int32_t* mirror, const double* pq_part,
                      int nparts) {
  hipLaunchKernelGGL(k_update, dim3(grid_x(len), (unsigned)S.k), dim3(NT), 0, st, S, len, x, r, r_old, p, q, tol,
                     max_iter, mirror, pq_part, nparts, 1);
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(NT), 0, st, S, (int)grid_x(len), tol, max_iter, mirror,
                     pq_part ? 1 : 0);
  return hipGetLastError();
}

// the same update without the convergence decision (the general path decides on rho)
hipError_t fcg_update_nodecide(hipStream_t st, FcgState S, int64_t len, double* x, double* r, double* r_old,
                               const double* p, const double* q) {
  hipLaunchKernelGGL(k_update, dim3(grid_x(len), (unsigned)S.k), dim3(NT), 0, st, S, len, x, r, r_old, p, q, 0.0, 0,
                     nullptr, nullptr, 0, 0);
  return hipGetLastError();
}

// rho -= alpha t (the residual of A x = b carried next to the normal-equation residual);
// the decision (tol, cap, NaN, breakdown) is taken on |rho|
__global__ void __launch_bounds__(NT) k_rho_update(FcgState S, int64_t len, double* __restrict__ rho,
                                                  const double* __restrict__ t, double tol, int32_t max_iter,
                                                  int32_t* mirror) {
  __shared__ double sh[NT / WAVE];
  const int j = blockIdx.y;
  double acc = 0.0;
  if (S.done[j] == 0) {
    const double a = S.alpha[j];
    for (int64_t i = chunk_begin(len) + threadIdx.x; i < chunk_end(len); i += NT) {
      const int64_t o = (int64_t)j * len + i;
      const double v = fma(-a, t[o], rho[o]);
      rho[o] = v;
      acc = fma(v, v, acc);
    }
  }
  const double tt = block_sum(acc, sh);
  if (threadIdx.x == 0) S.part[(int64_t)blockIdx.x * S.k + j] = tt;
  if (!last_block(S.counter)) return;
  for (int64_t jj = 0; jj < S.k; ++jj) {
    if (S.done[jj] != 0) continue;
    const double sum = strided_sum(S.part + jj, gridDim.x, S.k, sh);
    if (threadIdx.x != 0) continue;
    const double rn = sqrt(sum);
    S.rnorm[jj] = rn;
    const int it = S.iters[jj] + 1;
    S.iters[jj] = it;
    if (S.alpha[jj] == 0.0 || !(rn == rn)) S.done[jj] = 2;
    else if (rn <= tol * S.bnorm[jj]) S.done[jj] = 1;
    else if (it >= max_iter) S.done[jj] = 3;
  }
  __syncthreads();
  count_active(S, mirror);
}

hipError_t fcg_rho_update(hipStream_t st, FcgState S, int64_t len, double* rho, const double* t, double tol,
                          int32_t max_iter, int32_t* mirror) {
  hipLaunchKernelGGL(k_rho_update, dim3(grid_x(len), (unsigned)S.k), dim3(NT), 0, st, S, len, rho, t, tol, max_iter,
                     mirror);
  return hipGetLastError();
}

// done = 0 for columns whose done flag equals `from` (restart after a failed confirmation
// is handled by k_confirm; this re-arms columns for a fresh solve)
__global__ void k_set_done(FcgState S, const int32_t* src) {
  for (int64_t j = threadIdx.x; j < S.k; j += blockDim.x) S.done[j] = src ? src[j] : 0;
}
hipError_t fcg_copy_done(hipStream_t st, FcgState S, const int32_t* src) {
  hipLaunchKernelGGL(k_set_done, dim3(1), dim3(256), 0, st, S, src);
  return hipGetLastError();
}
hipError_t fcg_direction(hipStream_t st, FcgState S, int64_t len, const double* r, const double* r_old,
                         const double* z, double* p) {
  hipLaunchKernelGGL(k_beta, dim3(grid_x(len), (unsigned)S.k), dim3(NT), 0, st, S, len, r, r_old, z);
  hipLaunchKernelGGL(k_beta_fin, dim3(1), dim3(NT), 0, st, S, (int)grid_x(len));
  hipLaunchKernelGGL(k_pupdate, dim3(grid_x(len), (unsigned)S.k), dim3(NT), 0, st, S, len, z, p);
  return hipGetLastError();
}
hipError_t fcg_confirm(hipStream_t st, FcgState S, int64_t len, const double* rtrue, double* r, double tol,
                       double* relres, int32_t* mirror) {
  hipLaunchKernelGGL(k_confirm, dim3(grid_x(len), (unsigned)S.k), dim3(NT), 0, st, S, len, rtrue, r, tol, relres,
                     mirror);
  return hipGetLastError();
}
hipError_t launch_axpby(hipStream_t st, int64_t len, int64_t k, double a, const double* x, int64_t ldx, double b,
                        const double* y, int64_t ldy, double* out, int64_t ldo, const int32_t* skip) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_x(len), (unsigned)k), dim3(NT), 0, st, len, (int)k, a, x, ldx, b, y, ldy, out,
                     ldo, skip);
  return hipGetLastError();
}
hipError_t launch_coldots(hipStream_t st, int64_t len, int64_t k, const double* x, int64_t ldx, const double* y,
                          int64_t ldy, double* dev_out) {
  hipLaunchKernelGGL(k_coldot, dim3((unsigned)k), dim3(NT), 0, st, len, x, ldx, y, ldy, dev_out);
  return hipGetLastError();
}
hipError_t launch_outer_neg(hipStream_t st, int64_t n, int64_t k, const double* dB, int64_t lddb, const double* X,
                            int64_t ldx, double* dA, int64_t ldda) {
  hipLaunchKernelGGL(k_outer_neg, dim3((unsigned)((n + 255) / 256 > 64 ? 64 : (n + 255) / 256),
                                      (unsigned)(n < 16384 ? n : 16384)),
                     dim3(256), 0, st, n, (int)k, dB, lddb, X, ldx, dA, ldda);
  return hipGetLastError();
}
hipError_t launch_row_abs_max(hipStream_t st, const void* A, msp_dtype t, int64_t rows, int64_t cols, int64_t lda,
                              double* part, int64_t part_doubles, double* out) {
  int64_t nb = std::min<int64_t>(2048, (rows + NT / WAVE - 1) / (NT / WAVE));
  nb = std::max<int64_t>(1, std::min(nb, part_doubles));
  if (t == MSP_F64)
    hipLaunchKernelGGL(k_row_abs_max<double>, dim3((unsigned)nb), dim3(NT), 0, st, (const double*)A, rows, cols, lda,
                       part);
  else if (t == MSP_F32)
    hipLaunchKernelGGL(k_row_abs_max<float>, dim3((unsigned)nb), dim3(NT), 0, st, (const float*)A, rows, cols, lda,
                       part);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_max_parts, dim3(1), dim3(NT), 0, st, part, (int)nb, out);
  return hipGetLastError();
}

hipError_t launch_copy_block(hipStream_t st, int64_t len, int64_t k, const double* x, int64_t ldx, double* y,
                             int64_t ldy) {
  return launch_axpby(st, len, k, 1.0, x, ldx, 0.0, nullptr, 0, y, ldy, nullptr);
}
