// Inner flexible-PCG steps on a formed operator in two kernels per step: the level-3 solves
// of Algorithm 5 with the s x s A~^T A~ (+ sigma I) and the s x s preconditioner M3^{-1},
// for blocks of up to kL2fMaxK columns. Step t of the recurrence
//   q_t = (H + sigma I) p_t,  alpha_t = <r_t, z_t> / <p_t, q_t>,  y += alpha_t p_t,
//   r_{t+1} = r_t - alpha_t q_t,  z_{t+1} = Minv r_{t+1},
//   beta_{t+1} = <z_{t+1}, r_{t+1} - r_t> / <r_t, z_t>,  p_{t+1} = z_{t+1} + beta_{t+1} p_t
// runs as
//   k_l2f_op    the decision on |r_t| and beta_t from the previous step's partials (every
//               block sums them in the same order), p_t = z_t + beta_t p_{t-1} for the
//               block's rows, q_t = (H + sigma I) p_t for the block's rows (each block forms
//               the whole p_t it needs on the fly, staged in LDS by chunks), <p_t, q_t> partials;
//   k_l2f_prec  alpha_t from those partials (again in every block), r_{t+1} formed on the fly
//               the same way, y and r for the block's rows, z_{t+1} = Minv r_{t+1} for the
//               block's rows, and the partials of <z, r_{t+1}>, <z, r_t> and |r_{t+1}|^2.
// The same iteration as the six-kernel step (flexible PCG, Polak-Ribiere beta, the same
// stop and breakdown rules), with the matrix products as plain FP64 row dots instead of
// matrix-core block products: only the summation order differs. p and r alternate between
// two buffers by step parity (a block reads the whole previous vector while others write
// their rows of the next one); the per-column state is double-buffered the same way.
#include "msp_internal.h"

namespace {

constexpr int WAVE = 64;
constexpr int NT = 256;
constexpr int RB = kL2fRows;   // rows of the product per block
constexpr int CH = 256;        // reduction chunk staged in LDS
constexpr int KM = kL2fMaxK;   // columns handled per launch

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// rows r0 .. r0 + RB of out = M x, x[j][c] = u[j][c] + coef_j * v[j][c] formed on the fly
// (v may be null), for the live columns. Wavefront w takes rows r0 + 2w and r0 + 2w + 1;
// lane l takes the reduction indices l + 64 i of each chunk. acc[2][KM] returned per lane
// (not yet reduced over the wavefront).
__device__ __forceinline__ void rows_product(const double* __restrict__ M, int s, int k, int r0,
                                             const double* __restrict__ u, const double* __restrict__ v,
                                             const double* coef, const int* live, double (*xs)[CH],
                                             double (&acc)[2][KM]) {
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int rA = r0 + 2 * w, rB = rA + 1;
#pragma unroll
  for (int j = 0; j < KM; ++j) acc[0][j] = acc[1][j] = 0.0;
  for (int c0 = 0; c0 < s; c0 += CH) {
    for (int idx = tid; idx < CH * k; idx += NT) {
      const int j = idx / CH, cc = idx % CH, c = c0 + cc;
      double x = 0.0;
      if (c < s && live[j]) {
        x = u[(int64_t)j * s + c];
        if (v) x = fma(coef[j], v[(int64_t)j * s + c], x);
      }
      xs[j][cc] = x;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CH / WAVE; ++i) {
      const int cc = lane + WAVE * i, c = c0 + cc;
      if (c < s) {
        const double hA = rA < s ? M[(int64_t)rA * s + c] : 0.0;
        const double hB = rB < s ? M[(int64_t)rB * s + c] : 0.0;
#pragma unroll
        for (int j = 0; j < KM; ++j) {
          if (j < k) {
            const double x = xs[j][cc];
            acc[0][j] = fma(hA, x, acc[0][j]);
            acc[1][j] = fma(hB, x, acc[1][j]);
          }
        }
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(NT) k_l2f_op(L2fArgs a, int t, int fresh) {
  __shared__ double xs[KM][CH];
  __shared__ double beta_s[KM];
  __shared__ int live_s[KM];
  __shared__ double red[4][2][KM];
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int par = t & 1, nxt = par ^ 1;
  const int s = a.s, k = a.k;
  // ---- decision on |r_t| and beta_t (the same in every block) ----
  if (tid < k) {
    const int j = tid;
    int dj = fresh ? a.S.done[j] : a.done[par][j];
    int it = fresh ? a.S.iters[j] : a.iters[par][j];
    double rz = fresh ? a.S.rz[j] : a.rz[par][j];
    double beta = 0.0;
    if (!fresh && dj == 0) {
      double zr = 0.0, zro = 0.0, rr = 0.0;
      for (int b = 0; b < a.nb; ++b) {
        const double* d = a.dpart + ((int64_t)b * k + j) * 3;
        zr += d[0];
        zro += d[1];
        rr += d[2];
      }
      ++it;
      const double rn = sqrt(rr);
      if (a.brk[j] || !(rn == rn)) dj = 2;
      else if (rn <= a.tol * a.S.bnorm[j]) dj = 1;
      else if (it >= a.max_iter) dj = 3;
      if (dj == 0) {
        // beta's denominator <r_{t-1}, z_{t-1}> zero or not finite: no conjugate direction
        // exists; the column stops as a breakdown and keeps its iterate
        if (rz != 0.0 && isfinite(rz)) {
          beta = (zr - zro) / rz;
          rz = zr;
        } else {
          dj = 2;
        }
      }
      if (blockIdx.x == 0) a.S.rnorm[j] = rn;
    }
    live_s[j] = dj == 0;
    beta_s[j] = beta;
    if (blockIdx.x == 0) {
      a.done[nxt][j] = dj;
      a.iters[nxt][j] = it;
      a.rz[nxt][j] = rz;
    }
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    if (tid == 0) {
      int cnt = 0, mx = 0;
      for (int j = 0; j < k; ++j) {
        cnt += live_s[j];
        mx = max(mx, a.iters[nxt][j]);
      }
      if (a.mirror) {
        __hip_atomic_store(a.mirror, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(a.mirror + 1, mx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
  int any = 0;
  for (int j = 0; j < k; ++j) any |= live_s[j];
  if (!any) return;  // uniform in the block
  const double* pc = a.p[par];
  double* pn = a.p[nxt];
  const int r0 = blockIdx.x * RB;
  // p_t for the block's own rows (the previous direction for the first step: p = z)
  for (int idx = tid; idx < RB * k; idx += NT) {
    const int j = idx / RB, row = r0 + idx % RB;
    if (row < s && live_s[j]) pn[(int64_t)j * s + row] = fresh ? pc[(int64_t)j * s + row]
                                                                : fma(beta_s[j], pc[(int64_t)j * s + row],
                                                                      a.z[(int64_t)j * s + row]);
  }
  double acc[2][KM];
  if (fresh)
    rows_product(a.H, s, k, r0, pc, nullptr, beta_s, live_s, xs, acc);
  else
    rows_product(a.H, s, k, r0, a.z, pc, beta_s, live_s, xs, acc);
  // q rows and their <p, q> contributions
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    if (j >= k) continue;
    const double qa = wave_sum(acc[0][j]), qb = wave_sum(acc[1][j]);
    double pa = 0.0, pb = 0.0;
    if (lane == 0 && live_s[j]) {
      const int rA = r0 + 2 * w, rB = rA + 1;
      if (rA < s) {
        const double pv = fresh ? pc[(int64_t)j * s + rA] : fma(beta_s[j], pc[(int64_t)j * s + rA], a.z[(int64_t)j * s + rA]);
        const double qv = fma(a.sigma, pv, qa);
        a.q[(int64_t)j * s + rA] = qv;
        pa = pv * qv;
      }
      if (rB < s) {
        const double pv = fresh ? pc[(int64_t)j * s + rB] : fma(beta_s[j], pc[(int64_t)j * s + rB], a.z[(int64_t)j * s + rB]);
        const double qv = fma(a.sigma, pv, qb);
        a.q[(int64_t)j * s + rB] = qv;
        pb = pv * qv;
      }
    }
    if (lane == 0) {
      red[w][0][j] = pa;
      red[w][1][j] = pb;
    }
  }
  __syncthreads();
  if (tid < k) {
    const int j = tid;
    double t2 = 0.0;
    for (int ww = 0; ww < 4; ++ww) t2 += red[ww][0][j] + red[ww][1][j];
    a.ppart[(int64_t)blockIdx.x * k + j] = t2;
  }
}

__global__ void __launch_bounds__(NT) k_l2f_prec(L2fArgs a, int t) {
  __shared__ double xs[KM][CH];
  __shared__ double alpha_s[KM];
  __shared__ int live_s[KM];
  __shared__ double red[4][2][3][KM];
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int par = t & 1, nxt = par ^ 1;
  const int s = a.s, k = a.k;
  // alpha_t = <r_t, z_t> / <p_t, q_t> (the same in every block)
  if (tid < k) {
    const int j = tid;
    const int dj = a.done[nxt][j];
    double al = 0.0;
    if (dj == 0) {
      double pq = 0.0;
      for (int b = 0; b < a.nb; ++b) pq += a.ppart[(int64_t)b * k + j];
      const bool brk = !(pq > 0.0);
      al = brk ? 0.0 : a.rz[nxt][j] / pq;
      if (blockIdx.x == 0) {
        a.brk[j] = brk ? 1 : 0;
        a.alpha[j] = al;
      }
    }
    live_s[j] = dj == 0;
    alpha_s[j] = -al;  // r_{t+1} = r_t + (-alpha) q_t
  }
  __syncthreads();
  int any = 0;
  for (int j = 0; j < k; ++j) any |= live_s[j];
  if (!any) return;
  const double* rc = a.r[par];
  double* rn = a.r[nxt];
  const double* pn = a.p[nxt];
  const int r0 = blockIdx.x * RB;
  // y and r_{t+1} for the block's own rows
  for (int idx = tid; idx < RB * k; idx += NT) {
    const int j = idx / RB, row = r0 + idx % RB;
    if (row < s && live_s[j]) {
      const int64_t o = (int64_t)j * s + row;
      a.y[o] = fma(-alpha_s[j], pn[o], a.y[o]);
      rn[o] = fma(alpha_s[j], a.q[o], rc[o]);
    }
  }
  double acc[2][KM];
  rows_product(a.Minv, s, k, r0, rc, a.q, alpha_s, live_s, xs, acc);
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    if (j >= k) continue;
    const double za = wave_sum(acc[0][j]), zb = wave_sum(acc[1][j]);
    double d[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    if (lane == 0 && live_s[j]) {
      const int rows[2] = {r0 + 2 * w, r0 + 2 * w + 1};
      const double zz[2] = {za, zb};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int row = rows[h];
        if (row >= s) continue;
        const int64_t o = (int64_t)j * s + row;
        const double rnew = fma(alpha_s[j], a.q[o], rc[o]);
        a.z[o] = zz[h];
        d[h][0] = zz[h] * rnew;
        d[h][1] = zz[h] * rc[o];
        d[h][2] = rnew * rnew;
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 3; ++e) red[w][h][e][j] = d[h][e];
    }
  }
  __syncthreads();
  if (tid < 3 * k) {
    const int j = tid / 3, e = tid % 3;
    double t2 = 0.0;
    for (int ww = 0; ww < 4; ++ww) t2 += red[ww][0][e][j] + red[ww][1][e][j];
    a.dpart[((int64_t)blockIdx.x * k + j) * 3 + e] = t2;
  }
}

}  // namespace

int l2f_blocks(int64_t s) { return (int)((s + RB - 1) / RB); }

L2fArgs l2f_carve(WsCarver& w, int64_t s, int64_t k) {
  L2fArgs a{};
  a.s = (int)s;
  a.k = (int)k;
  a.nb = l2f_blocks(s);
  a.p[1] = w.take<double>(s * k);
  a.rz[0] = w.take<double>(k);
  a.rz[1] = w.take<double>(k);
  a.alpha = w.take<double>(k);
  a.ppart = w.take<double>((size_t)a.nb * k);
  a.dpart = w.take<double>((size_t)a.nb * k * 3);
  a.done[0] = w.take<int32_t>(k);
  a.done[1] = w.take<int32_t>(k);
  a.iters[0] = w.take<int32_t>(k);
  a.iters[1] = w.take<int32_t>(k);
  a.brk = w.take<int32_t>(k);
  return a;
}

hipError_t l2f_op(hipStream_t st, const L2fArgs& a, int t, int fresh) {
  hipLaunchKernelGGL(k_l2f_op, dim3((unsigned)a.nb), dim3(NT), 0, st, a, t, fresh);
  return hipGetLastError();
}

hipError_t l2f_prec(hipStream_t st, const L2fArgs& a, int t) {
  hipLaunchKernelGGL(k_l2f_prec, dim3((unsigned)a.nb), dim3(NT), 0, st, a, t);
  return hipGetLastError();
}
