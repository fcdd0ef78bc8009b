// Inner flexible-PCG steps on a formed operator in two kernels per step: the level-3 solves
// of Algorithm 5 with the s x s A~^T A~ (+ sigma I) and the s x s preconditioner M3^{-1},
// for blocks of up to kL2fMaxK columns and s <= kL2fMaxS. Step t of the recurrence
//   q_t = (H + sigma I) p_t,  alpha_t = <r_t, z_t> / <p_t, q_t>,  y += alpha_t p_t,
//   r_{t+1} = r_t - alpha_t q_t,  z_{t+1} = Minv r_{t+1},
//   beta_{t+1} = <z_{t+1}, r_{t+1} - r_t> / <r_t, z_t>,  p_{t+1} = z_{t+1} + beta_{t+1} p_t
// runs as
//   k_l2f_op    the decision on |r_t| and beta_t from the previous step's partials (every
//               block sums them in the same order), p_t = z_t + beta_t p_{t-1}, q_t for the
//               block's rows and the <p_t, q_t> partials;
//   k_l2f_prec  alpha_t from those partials (again in every block), y and r_{t+1} for the
//               block's rows, z_{t+1} = Minv r_{t+1} for them and the partials of
//               <z, r_{t+1}>, <z, r_t> and |r_{t+1}|^2.
// The same iteration as the generic step (flexible PCG, Polak-Ribiere beta, the same stop and
// breakdown rules) with the matrix products as plain FP64 row dots: only the summation order
// differs. Both kernels are bound by latency, not bandwidth (the s x s operands stay in the
// caches between steps), so each makes as few dependent round trips as it can: a block of
// eight wavefronts owns eight rows, one each (four rows per wavefront, a quarter of the blocks
// and of the bytes staged, measured slower at s = 2048: 79 against 66 us per step); the vector
// it multiplies (p_t, resp. r_{t+1},
// formed on the fly from the two vectors that define it) is staged whole into LDS for eight
// columns at a time, every thread issuing its loads in batches before storing any; the
// partial sums of the previous kernel are reduced by whole wavefronts. p and r alternate
// between two buffers by step parity (a block reads the whole previous vector while others
// write their rows of the next one); the per-column state is double-buffered the same way.
#include "msp_internal.h"

#include <mutex>

namespace {

constexpr int WAVE = 64;
constexpr int NWV = kL2fRows;     // wavefronts per block
constexpr int NT = NWV * WAVE;
constexpr int KG = 8;             // columns per staging pass
constexpr int KM = kL2fMaxK;      // columns per launch
constexpr int BATCH = 16;         // staged elements per thread per batch of loads

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// sum over b < nb of part[b * stride + e], by one wavefront in a fixed order (valid in
// every lane)
__device__ __forceinline__ double wave_parts(const double* part, int nb, int64_t stride, int e) {
  const int lane = threadIdx.x % WAVE;
  double t = 0.0;
  for (int b = lane; b < nb; b += WAVE) t += part[(int64_t)b * stride + e];
  return wave_sum(t);
}

// xs[jj * s + c] = u[j][c] + coef[j] v[j][c] (v null: u[j][c]) for the kg columns
// j = j0 + jj, zero for finished columns; every thread issues BATCH loads of each vector
// before storing any
__device__ __forceinline__ void stage(const double* __restrict__ u, const double* __restrict__ v,
                                      const double* coef, const int* live, int s, int j0, int kg, double* xs) {
  const int total = kg * s;
  for (int base = 0; base < total; base += NT * BATCH) {
    double uv[BATCH], vv[BATCH];
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int idx = base + q * NT + (int)threadIdx.x;
      uv[q] = 0.0;
      vv[q] = 0.0;
      if (idx < total) {
        const int jj = idx / s, c = idx - jj * s;
        if (live[j0 + jj]) {
          uv[q] = u[(int64_t)(j0 + jj) * s + c];
          if (v) vv[q] = v[(int64_t)(j0 + jj) * s + c];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int idx = base + q * NT + (int)threadIdx.x;
      if (idx < total) {
        const int jj = idx / s;
        xs[idx] = v ? fma(coef[j0 + jj], vv[q], uv[q]) : uv[q];
      }
    }
  }
}

// acc[i][jj] = sum_c M[row_i][c] xs[jj * s + c] over this lane's columns c = lane + 64 m,
// rows row_i = row0 + NWV i
template <int RPW>
__device__ __forceinline__ void row_dots(const double* __restrict__ M, int s, int row0, int kg, const double* xs,
                                         double (&acc)[RPW][KG]) {
  const int lane = threadIdx.x % WAVE;
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int jj = 0; jj < KG; ++jj) acc[i][jj] = 0.0;
#pragma unroll 16
  for (int c = lane; c < s; c += WAVE) {
    double h[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int row = row0 + NWV * i;
      h[i] = row < s ? M[(int64_t)row * s + c] : 0.0;
    }
#pragma unroll
    for (int jj = 0; jj < KG; ++jj) {
      if (jj < kg) {
        const double x = xs[jj * s + c];
#pragma unroll
        for (int i = 0; i < RPW; ++i) acc[i][jj] = fma(h[i], x, acc[i][jj]);
      }
    }
  }
}

template <int RPW>
__global__ void __launch_bounds__(NT) k_l2f_op(L2fArgs a, int t, int fresh) {
  extern __shared__ double xs[];  // KG * s doubles
  __shared__ double beta_s[KM];
  __shared__ int live_s[KM];
  __shared__ double red[NWV][KM];
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int par = t & 1, nxt = par ^ 1;
  const int s = a.s, k = a.k;
  // ---- decision on |r_t| and beta_t (the same in every block): wavefront w takes the
  // columns w, w + NWV ----
  for (int j = w; j < k; j += NWV) {
    int dj = fresh ? a.S.done[j] : a.done[par][j];
    int it = fresh ? a.S.iters[j] : a.iters[par][j];
    double rz = fresh ? a.S.rz[j] : a.rz[par][j];
    double beta = 0.0;
    if (!fresh && dj == 0) {  // uniform in the wavefront
      const double zr = wave_parts(a.dpart, a.nb, (int64_t)k * 3, j * 3 + 0);
      const double zro = wave_parts(a.dpart, a.nb, (int64_t)k * 3, j * 3 + 1);
      const double rr = wave_parts(a.dpart, a.nb, (int64_t)k * 3, j * 3 + 2);
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
      if (blockIdx.x == 0 && lane == 0) a.S.rnorm[j] = rn;
    }
    if (lane == 0) {
      live_s[j] = dj == 0;
      beta_s[j] = beta;
      if (blockIdx.x == 0) {
        a.done[nxt][j] = dj;
        a.iters[nxt][j] = it;
        a.rz[nxt][j] = rz;
      }
    }
  }
  __syncthreads();
  if (blockIdx.x == 0 && tid == 0 && a.mirror) {
    int cnt = 0, mx = 0;
    for (int j = 0; j < k; ++j) {
      cnt += live_s[j];
      mx = max(mx, a.iters[nxt][j]);
    }
    __hip_atomic_store(a.mirror, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(a.mirror + 1, mx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  const double* pc = a.p[par];
  double* pn = a.p[nxt];
  const int row0 = blockIdx.x * NWV * RPW + w;
  for (int j0 = 0; j0 < k; j0 += KG) {
    const int kg = min(KG, k - j0);
    int any = 0;
    for (int jj = 0; jj < kg; ++jj) any |= live_s[j0 + jj];
    if (!any) {  // uniform in the block
      if (tid < kg)
        for (int ww = 0; ww < NWV; ++ww) red[ww][j0 + tid] = 0.0;
      continue;
    }
    // p_t = z_t + beta_t p_{t-1} (p_0 = z_0, held in p[0]) for every row, staged
    if (fresh)
      stage(pc, nullptr, beta_s, live_s, s, j0, kg, xs);
    else
      stage(a.z, pc, beta_s, live_s, s, j0, kg, xs);
    __syncthreads();
    double acc[RPW][KG];
    row_dots<RPW>(a.H, s, row0, kg, xs, acc);
    // lane jj finishes column j0 + jj of the wavefront's rows: p_t, q_t and <p_t, q_t>
    double pq = 0.0;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int row = row0 + NWV * i;
      double mine = 0.0;
#pragma unroll
      for (int jj = 0; jj < KG; ++jj) {
        const double qs = wave_sum(acc[i][jj]);
        if (lane == jj) mine = qs;
      }
      if (lane < kg) {
        const int j = j0 + lane;
        if (row < s && live_s[j]) {
          const double pv = xs[lane * s + row];
          const double qv = fma(a.sigma, pv, mine);
          pn[(int64_t)j * s + row] = pv;
          a.q[(int64_t)j * s + row] = qv;
          pq = fma(pv, qv, pq);
        }
      }
    }
    if (lane < kg) red[w][j0 + lane] = pq;
    __syncthreads();  // xs is restaged by the next pass; red is complete
  }
  if (tid < k) {
    double t2 = 0.0;
    for (int ww = 0; ww < NWV; ++ww) t2 += red[ww][tid];
    a.ppart[(int64_t)blockIdx.x * k + tid] = t2;
  }
}

template <int RPW>
__global__ void __launch_bounds__(NT) k_l2f_prec(L2fArgs a, int t) {
  extern __shared__ double xs[];  // KG * s doubles
  __shared__ double alpha_s[KM];
  __shared__ int live_s[KM];
  __shared__ double red[NWV][KM][3];
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int par = t & 1, nxt = par ^ 1;
  const int s = a.s, k = a.k;
  // alpha_t = <r_t, z_t> / <p_t, q_t> (the same in every block)
  for (int j = w; j < k; j += NWV) {
    const int dj = a.done[nxt][j];
    double al = 0.0;
    if (dj == 0) {  // uniform in the wavefront
      const double pq = wave_parts(a.ppart, a.nb, k, j);
      const bool brk = !(pq > 0.0);
      al = brk ? 0.0 : a.rz[nxt][j] / pq;
      if (blockIdx.x == 0 && lane == 0) {
        a.brk[j] = brk ? 1 : 0;
        a.alpha[j] = al;
      }
    }
    if (lane == 0) {
      live_s[j] = dj == 0;
      alpha_s[j] = -al;  // r_{t+1} = r_t + (-alpha) q_t
    }
  }
  __syncthreads();
  const double* rc = a.r[par];
  double* rn = a.r[nxt];
  const double* pn = a.p[nxt];
  const int row0 = blockIdx.x * NWV * RPW + w;
  for (int j0 = 0; j0 < k; j0 += KG) {
    const int kg = min(KG, k - j0);
    int any = 0;
    for (int jj = 0; jj < kg; ++jj) any |= live_s[j0 + jj];
    if (!any) {
      if (tid < kg)
        for (int ww = 0; ww < NWV; ++ww)
          for (int e = 0; e < 3; ++e) red[ww][j0 + tid][e] = 0.0;
      continue;
    }
    stage(rc, a.q, alpha_s, live_s, s, j0, kg, xs);  // r_{t+1}
    __syncthreads();
    double acc[RPW][KG];
    row_dots<RPW>(a.Minv, s, row0, kg, xs, acc);
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int row = row0 + NWV * i;
      double mine = 0.0;
#pragma unroll
      for (int jj = 0; jj < KG; ++jj) {
        const double zs = wave_sum(acc[i][jj]);
        if (lane == jj) mine = zs;
      }
      if (lane < kg) {
        const int j = j0 + lane;
        if (row < s && live_s[j]) {
          const int64_t o = (int64_t)j * s + row;
          const double rnew = xs[lane * s + row];
          const double rold = rc[o];
          a.y[o] = fma(-alpha_s[j], pn[o], a.y[o]);
          rn[o] = rnew;
          a.z[o] = mine;
          d0 = fma(mine, rnew, d0);
          d1 = fma(mine, rold, d1);
          d2 = fma(rnew, rnew, d2);
        }
      }
    }
    if (lane < kg) {
      const int j = j0 + lane;
      red[w][j][0] = d0;
      red[w][j][1] = d1;
      red[w][j][2] = d2;
    }
    __syncthreads();
  }
  if (tid < 3 * k) {
    const int j = tid / 3, e = tid % 3;
    double t2 = 0.0;
    for (int ww = 0; ww < NWV; ++ww) t2 += red[ww][j][e];
    a.dpart[((int64_t)blockIdx.x * k + j) * 3 + e] = t2;
  }
}

size_t lds_bytes(int s) { return (size_t)KG * (size_t)s * sizeof(double); }

// rows per wavefront: the kernels are written for RPW rows, one measured fastest
constexpr int kRowsPerWave = 1;

std::once_flag g_lds_once;
hipError_t g_lds_err = hipSuccess;

// the staging array exceeds the default 64 KiB of dynamic LDS for s > 1024
hipError_t allow_lds() {
  std::call_once(g_lds_once, [] {
    const int bytes = (int)lds_bytes(kL2fMaxS);
    const void* fns[] = {(const void*)k_l2f_op<kRowsPerWave>, (const void*)k_l2f_prec<kRowsPerWave>};
    for (const void* f : fns)
      if (g_lds_err == hipSuccess) g_lds_err = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  });
  return g_lds_err;
}

}  // namespace

int l2f_blocks(int64_t s) {
  const int rb = NWV * kRowsPerWave;
  return (int)((s + rb - 1) / rb);
}

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
  if (a.s < 1 || a.s > kL2fMaxS || a.k < 1 || a.k > kL2fMaxK || a.nb != l2f_blocks(a.s)) return hipErrorInvalidValue;
  hipError_t e = allow_lds();
  if (e != hipSuccess) return e;
  const size_t lds = lds_bytes(a.s);
  hipLaunchKernelGGL(k_l2f_op<kRowsPerWave>, dim3((unsigned)a.nb), dim3(NT), lds, st, a, t, fresh);
  return hipGetLastError();
}

hipError_t l2f_prec(hipStream_t st, const L2fArgs& a, int t) {
  if (a.s < 1 || a.s > kL2fMaxS || a.k < 1 || a.k > kL2fMaxK || a.nb != l2f_blocks(a.s)) return hipErrorInvalidValue;
  hipError_t e = allow_lds();
  if (e != hipSuccess) return e;
  const size_t lds = lds_bytes(a.s);
  hipLaunchKernelGGL(k_l2f_prec<kRowsPerWave>, dim3((unsigned)a.nb), dim3(NT), lds, st, a, t);
  return hipGetLastError();
}
