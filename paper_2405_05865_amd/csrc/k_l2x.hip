// Inner flexible-PCG iterations with an explicit s x s operator, one kernel per step.
//
// Under level2_form 1 the level-2 solve of Algorithm 2 applies the formed operator
// H = C^T C + lam~ W with the preconditioner M2^{-1}. Both H and Minv are fixed, so with
// G = H Minv (formed once per solve) the operator image of the direction follows from the
// residual:
//   z_t = Minv r_t,   p_t = z_t + beta_t p_{t-1},   u_t = H p_t = G r_t + beta_t u_{t-1}.
// A step then needs one pass over the rows of [Minv; G] with r_{t+1}; everything else is
// s-length vector work. Every block evaluates the s-length dots of the step redundantly,
// with the same code on the same data (identical bits in every block), and computes the
// matrix rows it owns. Columns (right-hand sides) are the grid's second dimension; with
// one column the first block publishes the host mirror itself, with several a one-block
// kernel does it after a chunk of steps. Vectors that every block reads in full (r, z, g,
// p, u) alternate between two buffers by step parity, so no block overwrites what another
// block of the same launch still reads; y is updated in place by the owner of each element.
//
// beta is the flexible (Polak-Ribiere) choice <z_t, r_t - r_{t-1}> / <z_{t-1}, r_{t-1}>,
// with r_t - r_{t-1} = -alpha_{t-1} u_{t-1}. The stop rule is the one of the other inner
// kernels: |r| <= tol |b| on the recurrence residual, breakdown, or the iteration cap.
// The recurrence for u is exact only in exact arithmetic: with H and Minv as ill-conditioned
// as the general level-3 matrices (A~^T A~, whose spread is kappa(A)^2) u drifts from H p
// and the iterate stalls far above the tolerance, so those solves keep direct products.
#include "msp_internal.h"

namespace {

constexpr int WAVE = 64;
constexpr int NT = 256;  // four wavefronts
constexpr int NW = NT / WAVE;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// block-wide sums of two values, fixed order, valid in every thread
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh /*2*NW*/) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) {
    sh[w] = a;
    sh[NW + w] = b;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    ta += sh[q];
    tb += sh[NW + q];
  }
  a = ta;
  b = tb;
}

__device__ __forceinline__ double block_sum1(double a, double* sh) {
  double b = 0.0;
  block_sum2(a, b, sh);
  return a;
}

// rows [row0, row0 + NW*RPW) of z = Minv r and g = G r from r staged in LDS (rs, zero
// beyond s); wavefront w takes rows row0 + w + NW*q
template <int CPL, int RPW>
__device__ __forceinline__ void rows_pass(const L2xArgs& a, int row0, const double* rs, double* zo, double* go) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int s = a.s;
#pragma unroll
  for (int q = 0; q < RPW; ++q) {
    const int i = row0 + w + NW * q;
    if (i >= s) break;
    const double* mr = a.Minv + (int64_t)i * s;
    const double* gr = a.G + (int64_t)i * s;
    double tz = 0.0, tg = 0.0;
#pragma unroll
    for (int c4 = 0; c4 < CPL; ++c4) {
      const int c = lane + c4 * WAVE;
      if (c < s) {
        const double rv = rs[c];
        tz = fma(mr[c], rv, tz);
        tg = fma(gr[c], rv, tg);
      }
    }
    tz = wave_sum(tz);
    tg = wave_sum(tg);
    if (lane == 0) {
      zo[i] = tz;
      go[i] = tg;
    }
  }
}

// With one row per wavefront (s <= 512) the wavefront's rows of Minv and G are loaded into
// registers at the start of a kernel, so their latency overlaps the vector loads and block
// sums instead of following them; the pass then reads only r from LDS.
template <int CPL>
struct RowRegs {
  double m[CPL], g[CPL];
};

template <int CPL>
__device__ __forceinline__ void load_rows(const L2xArgs& a, int row0, RowRegs<CPL>& R) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int s = a.s, i = row0 + w;
#pragma unroll
  for (int c4 = 0; c4 < CPL; ++c4) {
    const int c = lane + c4 * WAVE;
    const bool in = i < s && c < s;
    R.m[c4] = in ? a.Minv[(int64_t)i * s + c] : 0.0;
    R.g[c4] = in ? a.G[(int64_t)i * s + c] : 0.0;
  }
}

template <int CPL>
__device__ __forceinline__ void rows_pass_regs(const L2xArgs& a, int row0, const double* rs, const RowRegs<CPL>& R,
                                               double* zo, double* go) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int i = row0 + w;
  if (i >= a.s) return;
  double tz = 0.0, tg = 0.0;
#pragma unroll
  for (int c4 = 0; c4 < CPL; ++c4) {
    const double rv = rs[lane + c4 * WAVE];  // zero beyond s
    tz = fma(R.m[c4], rv, tz);
    tg = fma(R.g[c4], rv, tg);
  }
  tz = wave_sum(tz);
  tg = wave_sum(tg);
  if (lane == 0) {
    zo[i] = tz;
    go[i] = tg;
  }
}

// first step's inputs: |b| from r_0 (written by the right-hand-side kernel), the
// decision (parent done or b = 0), z_0 and g_0
template <int CPL, int RPW>
__global__ void __launch_bounds__(NT) k_l2x_start(L2xArgs a) {
  constexpr int EPT = (CPL * WAVE + NT - 1) / NT;
  __shared__ double rs[CPL * WAVE];
  __shared__ double sh[2 * NW];
  const int tid = threadIdx.x, s = a.s;
  const int row0 = blockIdx.x * NW * RPW;
  RowRegs<CPL> R;
  if constexpr (RPW == 1) load_rows<CPL>(a, row0, R);
  int cnt = 0;
  {
    const int j = blockIdx.y;
    const int64_t o = (int64_t)j * s;
    double rv[EPT];
    double sq = 0.0;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * NT;
      rv[q] = (e < s) ? a.r[0][o + e] : 0.0;
      sq = fma(rv[q], rv[q], sq);
    }
    const double bn = sqrt(block_sum1(sq, sh));
    const bool pd = a.parent_done && a.parent_done[j];
    const int dj = (pd || bn == 0.0) ? 1 : 0;
    if (blockIdx.x == 0 && tid == 0) {
      a.bn[j] = bn;
      a.rz[0][j] = 0.0;
      a.al[0][j] = 0.0;
      a.done[0][j] = dj;
      a.it[0][j] = 0;
    }
    if (dj == 0) {  // uniform in the block
      ++cnt;
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * NT;
        if (e < CPL * WAVE) rs[e] = rv[q];
      }
      __syncthreads();
      if constexpr (RPW == 1)
        rows_pass_regs<CPL>(a, row0, rs, R, a.z[0] + o, a.g[0] + o);
      else
        rows_pass<CPL, RPW>(a, row0, rs, a.z[0] + o, a.g[0] + o);
    }
  }
  if (gridDim.y == 1 && blockIdx.x == 0 && tid == 0 && a.mirror) {
    __hip_atomic_store(a.mirror, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(a.mirror + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// step t: reads parity par (r_t, z_t, g_t, p_{t-1}, u_{t-1}, state), writes parity par^1
// (r_{t+1}, z_{t+1}, g_{t+1}, p_t, u_t, state) and y += alpha_t p_t on the owned rows
template <int CPL, int RPW>
__global__ void __launch_bounds__(NT) k_l2x_step(L2xArgs a, int par, int first) {
  constexpr int EPT = (CPL * WAVE + NT - 1) / NT;
  __shared__ double rs[CPL * WAVE];
  __shared__ double sh[2 * NW];
  const int tid = threadIdx.x, s = a.s;
  const int cur = par, nxt = par ^ 1;
  const int row0 = blockIdx.x * NW * RPW;
  const int row1 = min(s, row0 + NW * RPW);
  const bool lead = blockIdx.x == 0 && tid == 0;
  const bool publish = gridDim.y == 1 && lead && a.mirror;
  const int j = blockIdx.y;
  const int64_t o = (int64_t)j * s;
  RowRegs<CPL> R;
  if constexpr (RPW == 1) load_rows<CPL>(a, row0, R);
  const int dcur = a.done[cur][j];
  if (dcur != 0) {  // carry the finished column's state to the next parity
    const int itc = a.it[cur][j];
    if (lead) {
      a.done[nxt][j] = dcur;
      a.it[nxt][j] = itc;
      a.rz[nxt][j] = a.rz[cur][j];
      a.al[nxt][j] = a.al[cur][j];
    }
    if (publish) {
      __hip_atomic_store(a.mirror, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(a.mirror + 1, itc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    return;  // uniform in the block
  }
  {
    double zv[EPT], rv[EPT], pv[EPT], uv[EPT], gv[EPT];
    double zr = 0.0, zu = 0.0;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * NT;
      const bool in = e < s;
      zv[q] = in ? a.z[cur][o + e] : 0.0;
      rv[q] = in ? a.r[cur][o + e] : 0.0;
      pv[q] = (in && !first) ? a.p[cur][o + e] : 0.0;
      uv[q] = (in && !first) ? a.u[cur][o + e] : 0.0;
      gv[q] = in ? a.g[cur][o + e] : 0.0;
      zr = fma(zv[q], rv[q], zr);
      zu = fma(zv[q], uv[q], zu);
    }
    block_sum2(zr, zu, sh);
    // beta's denominator <r_{t-1}, z_{t-1}> zero or not finite: no conjugate direction
    // exists; the column stops as a breakdown below (alpha = 0 keeps its iterate)
    const double rzo = a.rz[cur][j];
    const bool rzbad = !first && !(rzo != 0.0 && isfinite(rzo));
    const double beta = (first || rzbad) ? 0.0 : -a.al[cur][j] * zu / rzo;
    double pq = 0.0;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      pv[q] = fma(beta, pv[q], zv[q]);
      uv[q] = fma(beta, uv[q], gv[q]);
      pq = fma(pv[q], uv[q], pq);
    }
    pq = block_sum1(pq, sh);
    const bool brk = rzbad || !(pq > 0.0);
    const double alpha = brk ? 0.0 : zr / pq;
    double rr = 0.0;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      rv[q] = fma(-alpha, uv[q], rv[q]);
      rr = fma(rv[q], rv[q], rr);
    }
    rr = block_sum1(rr, sh);
    const double rn = sqrt(rr);
    const int it = a.it[cur][j] + 1;
    int dj = 0;
    if (brk || !(rn == rn)) dj = 2;
    else if (rn <= a.tol * a.bn[j]) dj = 1;
    else if (it >= a.max_iter) dj = 3;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * NT;
      if (e >= row0 && e < row1) {
        a.p[nxt][o + e] = pv[q];
        a.u[nxt][o + e] = uv[q];
        a.r[nxt][o + e] = rv[q];
        a.y[o + e] = fma(alpha, pv[q], a.y[o + e]);
      }
    }
    if (lead) {
      a.done[nxt][j] = dj;
      a.it[nxt][j] = it;
      a.rz[nxt][j] = zr;
      a.al[nxt][j] = alpha;
    }
    if (publish) {
      __hip_atomic_store(a.mirror, dj == 0 ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(a.mirror + 1, it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (dj == 0) {  // uniform in the block
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * NT;
        if (e < CPL * WAVE) rs[e] = rv[q];
      }
      __syncthreads();
      if constexpr (RPW == 1)
        rows_pass_regs<CPL>(a, row0, rs, R, a.z[nxt] + o, a.g[nxt] + o);
      else
        rows_pass<CPL, RPW>(a, row0, rs, a.z[nxt] + o, a.g[nxt] + o);
    }
  }
}

// the host mirror for several columns: active count and largest iteration count of the
// state at parity par
__global__ void __launch_bounds__(NT) k_l2x_publish(L2xArgs a, int par) {
  __shared__ int cnt, mx;
  if (threadIdx.x == 0) {
    cnt = 0;
    mx = 0;
  }
  __syncthreads();
  int c = 0, m = 0;
  for (int j = threadIdx.x; j < a.k; j += NT) {
    c += a.done[par][j] == 0 ? 1 : 0;
    m = max(m, a.it[par][j]);
  }
  atomicAdd(&cnt, c);
  atomicMax(&mx, m);
  __syncthreads();
  if (threadIdx.x == 0 && a.mirror) {
    __hip_atomic_store(a.mirror, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(a.mirror + 1, mx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// rows per wavefront: about 128 blocks whatever s
inline int rpw_for(int s) { return s <= 512 ? 1 : (s <= 1024 ? 2 : 4); }

template <int CPL, int RPW>
hipError_t launch_t(hipStream_t st, const L2xArgs& a, int mode, int par, int first) {
  const unsigned blocks = (unsigned)((a.s + NW * RPW - 1) / (NW * RPW));
  if (mode == 0)
    hipLaunchKernelGGL((k_l2x_start<CPL, RPW>), dim3(blocks, (unsigned)a.k), dim3(NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_l2x_step<CPL, RPW>), dim3(blocks, (unsigned)a.k), dim3(NT), 0, st, a, par, first);
  return hipGetLastError();
}

hipError_t dispatch(hipStream_t st, const L2xArgs& a, int mode, int par, int first) {
  const int cpl = (a.s + WAVE - 1) / WAVE;
  const int rpw = rpw_for(a.s);
  if (cpl <= 1) return launch_t<1, 1>(st, a, mode, par, first);
  if (cpl <= 2) return launch_t<2, 1>(st, a, mode, par, first);
  if (cpl <= 4) return launch_t<4, 1>(st, a, mode, par, first);
  if (cpl <= 8) return launch_t<8, 1>(st, a, mode, par, first);
  if (cpl <= 16 && rpw == 2) return launch_t<16, 2>(st, a, mode, par, first);
  if (cpl <= 32 && rpw == 4) return launch_t<32, 4>(st, a, mode, par, first);
  return hipErrorInvalidValue;
}

}  // namespace

size_t l2x_doubles(int64_t s, int64_t k) { return (size_t)(10 * s * k + 9 * k) + 64 * 12; }

L2xArgs l2x_carve(WsCarver& w, int64_t s, int64_t k) {
  L2xArgs a{};
  a.s = (int)s;
  a.k = (int)k;
  for (int q = 0; q < 2; ++q) {
    a.r[q] = w.take<double>(s * k);
    a.z[q] = w.take<double>(s * k);
    a.g[q] = w.take<double>(s * k);
    a.p[q] = w.take<double>(s * k);
    a.u[q] = w.take<double>(s * k);
    a.rz[q] = w.take<double>(k);
    a.al[q] = w.take<double>(k);
    a.done[q] = w.take<int32_t>(k);
    a.it[q] = w.take<int32_t>(k);
  }
  a.bn = w.take<double>(k);
  return a;
}

hipError_t l2x_start(hipStream_t st, const L2xArgs& a) {
  if (a.s < 1 || a.s > kL2xMaxS || a.k < 1 || a.k > kL2xMaxK) return hipErrorInvalidValue;
  return dispatch(st, a, 0, 0, 0);
}

hipError_t l2x_step(hipStream_t st, const L2xArgs& a, int par, int first) {
  if (a.s < 1 || a.s > kL2xMaxS || a.k < 1 || a.k > kL2xMaxK) return hipErrorInvalidValue;
  return dispatch(st, a, 1, par & 1, first ? 1 : 0);
}

hipError_t l2x_publish(hipStream_t st, const L2xArgs& a, int par) {
  if (a.k <= 1) return hipSuccess;  // published by the step and start kernels
  hipLaunchKernelGGL(k_l2x_publish, dim3(1), dim3(NT), 0, st, a, par & 1);
  return hipGetLastError();
}
