// One step of the inner iterations on the sketch Y (n x s): the level-2 solve of
// Algorithm 2 ((C^T C + lam~ W) y = C^T r with M2^{-1}) and the level-3 solves of
// Algorithm 5 ((A~^T A~ + sigma I) u = r with M3a^{-1} or M3b^{-1}). The operator is
//   q = Y^T (Y p) + wscale * W p + sigma * p        (W optional)
// and a flexible-PCG step takes three kernels:
//   k_l2_op      one pass over Y (row dots inside a wavefront, column sums in registers)
//                plus the rows of W p; per-block partials of Y^T Y p and <p, q>
//   k_l2_update  fixed-order reduction of the partials, alpha, y/r update, |r|
//   k_l2_prec    z = Minv r, <z, r>, <z, r_old>, beta, p = z + beta p
// and k_l2_init forms the right-hand side Y^T v. All reductions run in a fixed order,
// so every block that needs a scalar computes the same bits.
#include "msp_internal.h"

#include <hip/hip_bf16.h>

namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < NT / WAVE; ++q) t += sh[q];
  __syncthreads();
  return t;  // valid in every thread
}

// the last block of the grid to arrive (device-scope fence in every block)
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

// columns up to which the last block of k_l2_dir publishes (its fences are cheap for a
// few blocks); beyond, a one-block kernel does it after k_l2_dir
constexpr int kDirFenceMaxK = 16;
// columns from which the explicit-operator update runs one block per column
constexpr int kUpdateColMinK = 32;

template <class T>
__device__ __forceinline__ double ldy(const T* p) { return (double)(*p); }

// ---- pass over Y: part[b][j][c] = sum_rows Y[r,c] * t_r,j with t = Y p (mode 0) or
// t = v (mode 1: Y^T v for the right-hand side); pqpart[b][j] = sum_rows t^2 (mode 0).
// Blocks >= nbC compute rows of W p (mode 0, W != null): wp[j][i], pqw[j][i] = p_i (W p)_i.
constexpr int GROUP = 16;  // Y-pass blocks pre-reduced by the last block of each group

template <class TY, int CPL, int KG, int MODE>
__global__ void __launch_bounds__(256) k_l2_op(const TY* __restrict__ Y, int64_t n, int s, int64_t ldy_,
                                              const double* __restrict__ v, int64_t ldv, int k, int j0,
                                              const int32_t* __restrict__ done, double* __restrict__ part,
                                              double* __restrict__ pqpart, const double* __restrict__ W,
                                              double* __restrict__ wp, double* __restrict__ pqw, int nbC) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  if ((int)blockIdx.x >= nbC) {
    // rows of W p
    const int i = ((int)blockIdx.x - nbC) * 4 + w;
    if (i >= s) return;
    double m[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane + q * WAVE;
      m[q] = (c < s) ? W[(int64_t)i * s + c] : 0.0;
    }
    for (int g = 0; g < KG; ++g) {
      const int j = j0 + g;
      if (j >= k || (done && done[j])) continue;
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const int c = lane + q * WAVE;
        t = fma(m[q], (c < s) ? v[(int64_t)j * s + c] : 0.0, t);
      }
      t = wave_sum(t);
      if (lane == 0) {
        wp[(int64_t)j * s + i] = t;
        pqw[(int64_t)j * s + i] = v[(int64_t)j * s + i] * t;
      }
    }
    return;
  }
  __shared__ double red[4][CPL * WAVE];
  __shared__ double pqs[4][KG];
  const int64_t per = (n + nbC - 1) / nbC;
  const int64_t r0 = blockIdx.x * per, r1 = min(n, r0 + per);
  bool live[KG];
  double z[KG][CPL], acc[KG][CPL], pq[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) {
    const int j = j0 + g;
    live[g] = (j < k) && !(done && done[j]);
    pq[g] = 0.0;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane + q * WAVE;
      z[g][q] = (MODE == 0 && live[g] && c < s) ? v[(int64_t)j * s + c] : 0.0;
      acc[g][q] = 0.0;
    }
  }
  // two rows per step for memory-level parallelism
  int64_t r = r0 + w;
  for (; r + 4 < r1; r += 8) {
    double ya[CPL], yb[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane + q * WAVE;
      ya[q] = (c < s) ? ldy(Y + r * ldy_ + c) : 0.0;
      yb[q] = (c < s) ? ldy(Y + (r + 4) * ldy_ + c) : 0.0;
    }
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      double ta, tb;
      if (MODE == 0) {
        ta = 0.0;
        tb = 0.0;
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
          ta = fma(ya[q], z[g][q], ta);
          tb = fma(yb[q], z[g][q], tb);
        }
        ta = wave_sum(ta);
        tb = wave_sum(tb);
        pq[g] = fma(ta, ta, fma(tb, tb, pq[g]));
      } else {
        const int j = j0 + g;
        ta = live[g] ? v[(int64_t)j * ldv + r] : 0.0;
        tb = live[g] ? v[(int64_t)j * ldv + r + 4] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < CPL; ++q) acc[g][q] = fma(ya[q], ta, fma(yb[q], tb, acc[g][q]));
    }
  }
  for (; r < r1; r += 4) {
    double ya[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane + q * WAVE;
      ya[q] = (c < s) ? ldy(Y + r * ldy_ + c) : 0.0;
    }
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      double ta;
      if (MODE == 0) {
        ta = 0.0;
#pragma unroll
        for (int q = 0; q < CPL; ++q) ta = fma(ya[q], z[g][q], ta);
        ta = wave_sum(ta);
        pq[g] = fma(ta, ta, pq[g]);
      } else {
        const int j = j0 + g;
        ta = live[g] ? v[(int64_t)j * ldv + r] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < CPL; ++q) acc[g][q] = fma(ya[q], ta, acc[g][q]);
    }
  }
  for (int g = 0; g < KG; ++g) {
    const int j = j0 + g;
    if (j >= k) break;
#pragma unroll
    for (int q = 0; q < CPL; ++q) red[w][q * WAVE + lane] = acc[g][q];
    if (lane == 0) pqs[w][g] = pq[g];
    __syncthreads();
    for (int c = threadIdx.x; c < s; c += 256)
      part[((int64_t)blockIdx.x * k + j) * s + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
    if (MODE == 0 && threadIdx.x == 0)
      pqpart[(int64_t)blockIdx.x * k + j] = pqs[0][g] + pqs[1][g] + pqs[2][g] + pqs[3][g];
    __syncthreads();
  }
}

// group sums of the Y-pass partials: gpart[g][j][c] = sum_{b in group g} part[b][j][c]
__global__ void __launch_bounds__(256) k_l2_gsum(const double* __restrict__ part, const double* __restrict__ pqpart,
                                                int nbC, int k, int s, double* __restrict__ gpart,
                                                double* __restrict__ gpq) {
  const int g = blockIdx.x, j = blockIdx.y;
  const int b0 = g * GROUP, b1 = min(nbC, b0 + GROUP);
  for (int c = threadIdx.x; c < s; c += 256) {
    double t[GROUP];
#pragma unroll
    for (int q = 0; q < GROUP; ++q) t[q] = (b0 + q < b1) ? part[((int64_t)(b0 + q) * k + j) * s + c] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < GROUP; ++q) acc += t[q];
    gpart[((int64_t)g * k + j) * s + c] = acc;
  }
  if (pqpart && threadIdx.x == 0) {
    double acc = 0.0;
    for (int b = b0; b < b1; ++b) acc += pqpart[(int64_t)b * k + j];
    gpq[(int64_t)g * k + j] = acc;
  }
}

struct L2Args {
  int s, k, nbC;
  const double* gpart;   // [ngroups][k][s]  group sums of the Y-pass partials
  const double* gpq;     // [ngroups][k]
  const double* wp;      // [k][s] or null
  const double* pqw;     // [k][s] or null
  double wscale, sigma;
  double *y, *r, *ro, *z, *p, *q;  // [k][s]
  const double* Minv;
  FcgState S;
  double* upart;         // [ceil(s/64)][k]      |r|^2 partials of k_l2_update / k_l2_init
  double* dpart;         // [ceil(s/4)][k][2]    <z, r>, <z, r_old> partials of k_l2_prec
  double tol;
  int max_iter;
  int32_t* mirror;
  const int32_t* parent_done;
  const double* rhs;     // k_l2_init: given right-hand side (s x k) or null
  int ndp;               // blocks of dot partials in dpart (read by k_l2_dir)
};

constexpr int NTU = 1024;  // 16 wavefronts

__host__ __device__ inline int ngroups(int nbC) { return (nbC + GROUP - 1) / GROUP; }
__host__ __device__ inline int ublocks(int s) { return (s + WAVE - 1) / WAVE; }
__host__ __device__ inline int pblocks(int s) { return (s + 3) / 4; }
__host__ __device__ inline int dblocks(int s) { return (s + 255) / 256; }

// z = Minv r on the matrix cores (then k_l2_dots) instead of k_l2_prec
inline bool mfma_prec(const L2Step& a) { return a.gscratch && a.k >= kGemmMinK && a.Minv; }

// fixed-order parallel sum over count strided values, valid in every thread
template <int NT>
__device__ __forceinline__ double strided_sum(const double* base, int count, int64_t stride, double* sh) {
  double t = 0.0;
  for (int b = threadIdx.x; b < count; b += NT) t += base[(int64_t)b * stride];
  return block_sum<NT>(t, sh);
}

// sum over the groups of gpart[g][j][c] for the 64 outputs c0 + lane (wave w takes
// g = w mod 16); valid in wave 0
__device__ __forceinline__ double reduce_groups_col(const double* gpart, int ng, int k, int s, int j, int c,
                                                    double* sh /*16*64*/) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  double a0 = 0.0;
  if (c < s)
    for (int g = w; g < ng; g += NTU / WAVE) a0 += gpart[((int64_t)g * k + j) * s + c];
  sh[w * WAVE + lane] = a0;
  __syncthreads();
  double t = 0.0;
  if (w == 0)
#pragma unroll
    for (int q = 0; q < NTU / WAVE; ++q) t += sh[q * WAVE + lane];
  __syncthreads();
  return t;
}

// ---- right-hand side: rhs = sum of the group partials of Y^T v; y = 0, r = rhs ------
__global__ void __launch_bounds__(NTU) k_l2_init(L2Args a) {
  __shared__ double sh[NTU];
  __shared__ double shs[NTU / WAVE];
  const int j = blockIdx.y, lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int c = blockIdx.x * WAVE + lane;
  const bool pd = a.parent_done && a.parent_done[j];
  const double rhs = a.rhs ? ((c < a.s) ? a.rhs[(int64_t)j * a.s + c] : 0.0)
                           : reduce_groups_col(a.gpart, ngroups(a.nbC), a.k, a.s, j, c, sh);
  double sq = 0.0;
  if (w == 0 && c < a.s) {
    const double v = pd ? 0.0 : rhs;
    a.r[(int64_t)j * a.s + c] = v;
    a.y[(int64_t)j * a.s + c] = 0.0;
    sq = v * v;
  }
  const double t = block_sum<NTU>(sq, shs);
  if (threadIdx.x == 0) a.upart[(int64_t)blockIdx.x * a.k + j] = t;
}

// ---- the same step for an explicit operator (no Y-pass partials, nbC = 0): one block of
// 256 threads per column; wavefront w of round m owns the 64 elements of chunk 4m + w, so
// the |r|^2 partial of every 64-element chunk is one wavefront sum, as in k_l2_update
__global__ void __launch_bounds__(256) k_l2_update_m(L2Args a) {
  __shared__ double shs[4];
  const int j = blockIdx.x, lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  if (a.S.done[j] != 0) return;
  double t = 0.0;
  for (int i = threadIdx.x; i < a.s; i += 256) {
    const double pi = a.p[(int64_t)j * a.s + i];
    if (a.pqw) t = fma(a.wscale, a.pqw[(int64_t)j * a.s + i], t);
    else if (a.wp) t = fma(a.wscale * pi, a.wp[(int64_t)j * a.s + i], t);
    t = fma(a.sigma * pi, pi, t);
  }
  const double pq = block_sum<256>(t, shs);
  const bool brk = !(pq > 0.0);
  const double alpha = brk ? 0.0 : a.S.rz[j] / pq;
  for (int base = 0; base < a.s; base += 256) {
    const int c = base + threadIdx.x;
    double sq = 0.0;
    if (c < a.s) {
      const int64_t o = (int64_t)j * a.s + c;
      const double pv = a.p[o];
      double qv = a.sigma * pv;
      if (a.wp) qv = fma(a.wscale, a.wp[o], qv);
      a.q[o] = qv;
      a.y[o] = fma(alpha, pv, a.y[o]);
      const double rv = a.r[o];
      a.ro[o] = rv;
      const double rn = fma(-alpha, qv, rv);
      a.r[o] = rn;
      sq = rn * rn;
    }
    const double cs = wave_sum(sq);
    if (lane == 0 && base + w * WAVE < a.s) a.upart[(int64_t)(base / WAVE + w) * a.k + j] = cs;
  }
  if (threadIdx.x == 0) {
    a.S.alpha[j] = alpha;
    a.S.brk[j] = brk ? 1 : 0;
  }
}

// ---- q, alpha, y += alpha p, r_old = r, r -= alpha q, |r|^2 partials ---------------
__global__ void __launch_bounds__(NTU) k_l2_update(L2Args a) {
  __shared__ double sh[NTU];
  __shared__ double shs[NTU / WAVE];
  const int j = blockIdx.y, lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int c = blockIdx.x * WAVE + lane;
  if (a.S.done[j] != 0) return;
  // <p, q> = sum_g gpq + wscale * sum_i pqw + sigma * |p|^2, identical in every block
  double t = 0.0;
  for (int g = threadIdx.x; g < ngroups(a.nbC); g += NTU) t += a.gpq[(int64_t)g * a.k + j];
  for (int i = threadIdx.x; i < a.s; i += NTU) {
    const double pi = a.p[(int64_t)j * a.s + i];
    if (a.pqw) t = fma(a.wscale, a.pqw[(int64_t)j * a.s + i], t);
    else if (a.wp) t = fma(a.wscale * pi, a.wp[(int64_t)j * a.s + i], t);
    t = fma(a.sigma * pi, pi, t);
  }
  const double pq = block_sum<NTU>(t, shs);
  const double qa = reduce_groups_col(a.gpart, ngroups(a.nbC), a.k, a.s, j, c, sh);
  const bool brk = !(pq > 0.0);
  const double alpha = brk ? 0.0 : a.S.rz[j] / pq;
  double sq = 0.0;
  if (w == 0 && c < a.s) {
    const int64_t o = (int64_t)j * a.s + c;
    const double pv = a.p[o];
    double qv = qa + a.sigma * pv;
    if (a.wp) qv = fma(a.wscale, a.wp[o], qv);
    a.q[o] = qv;
    a.y[o] = fma(alpha, pv, a.y[o]);
    const double rv = a.r[o];
    a.ro[o] = rv;
    const double rn = fma(-alpha, qv, rv);
    a.r[o] = rn;
    sq = rn * rn;
  }
  const double tt = block_sum<NTU>(sq, shs);
  if (threadIdx.x == 0) {
    a.upart[(int64_t)blockIdx.x * a.k + j] = tt;
    if (blockIdx.x == 0) {
      a.S.alpha[j] = alpha;
      a.S.brk[j] = brk ? 1 : 0;
    }
  }
}

// ---- convergence decision, z = Minv r, partials of <z, r> and <z, r_old> ------------
// decide = 1 after k_l2_update (|r| test, iteration count), 2 after k_l2_init (|b| = |r|).
// Every block takes the same decision from values no block writes in this kernel;
// block 0 records it in done_next / iters_next, which k_l2_dir commits.
template <int CPL>
__global__ void __launch_bounds__(256) k_l2_prec(L2Args a, int decide) {
  __shared__ double d1[4], d2[4];
  __shared__ int live_sh;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int i = blockIdx.x * 4 + w;
  const int nu = ublocks(a.s);
  double m[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int c = lane + q * WAVE;
    m[q] = (i < a.s && c < a.s) ? a.Minv[(int64_t)i * a.s + c] : 0.0;
  }
  for (int j = 0; j < a.k; ++j) {
    if (threadIdx.x == 0) {
      int dj = a.S.done[j];
      int it = a.S.iters[j];
      double sum = 0.0;
      for (int b = 0; b < nu; ++b) sum += a.upart[(int64_t)b * a.k + j];
      const double rn = sqrt(sum);
      if (decide == 2) {
        const bool pd = a.parent_done && a.parent_done[j];
        dj = (pd || rn == 0.0) ? 1 : 0;
        it = 0;
        if (blockIdx.x == 0) {
          a.S.bnorm[j] = rn;
          a.S.rnorm[j] = rn;
          a.S.rz[j] = 0.0;
          a.S.beta[j] = 0.0;
        }
      } else if (dj == 0) {
        ++it;
        if (a.S.brk[j] || !(rn == rn)) dj = 2;
        else if (rn <= a.tol * a.S.bnorm[j]) dj = 1;
        else if (it >= a.max_iter) dj = 3;
        if (blockIdx.x == 0) a.S.rnorm[j] = rn;
      }
      if (blockIdx.x == 0) {
        a.S.done_next[j] = dj;
        a.S.iters_next[j] = it;
      }
      live_sh = (dj == 0);
    }
    __syncthreads();
    const bool live = live_sh != 0;
    double zr = 0.0, zro = 0.0;
    if (live && i < a.s) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const int c = lane + q * WAVE;
        t = fma(m[q], (c < a.s) ? a.r[(int64_t)j * a.s + c] : 0.0, t);
      }
      t = wave_sum(t);
      const int64_t o = (int64_t)j * a.s + i;
      if (lane == 0) a.z[o] = t;
      zr = t * a.r[o];
      zro = (decide == 2) ? 0.0 : t * a.ro[o];
    }
    if (lane == 0) {
      d1[w] = zr;
      d2[w] = zro;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      a.dpart[((int64_t)blockIdx.x * a.k + j) * 2 + 0] = (d1[0] + d1[1]) + (d1[2] + d1[3]);
      a.dpart[((int64_t)blockIdx.x * a.k + j) * 2 + 1] = (d2[0] + d2[1]) + (d2[2] + d2[3]);
    }
    __syncthreads();
  }
}

// ---- after z = Minv r on the matrix cores: z from the product's segment partials (when
// it was split), the decision of k_l2_prec for column blockIdx.y and the partials of
// <z, r> and <z, r_old> over 256 rows per block
__global__ void __launch_bounds__(256) k_l2_dots(L2Args a, int decide, const double* __restrict__ zpart, int nseg) {
  __shared__ double sh[4];
  __shared__ int live_sh;
  const int j = blockIdx.y;
  const int nu = ublocks(a.s);
  if (threadIdx.x == 0) {
    int dj = a.S.done[j];
    int it = a.S.iters[j];
    double sum = 0.0;
    for (int b = 0; b < nu; ++b) sum += a.upart[(int64_t)b * a.k + j];
    const double rn = sqrt(sum);
    if (decide == 2) {
      const bool pd = a.parent_done && a.parent_done[j];
      dj = (pd || rn == 0.0) ? 1 : 0;
      it = 0;
      if (blockIdx.x == 0) {
        a.S.bnorm[j] = rn;
        a.S.rnorm[j] = rn;
        a.S.rz[j] = 0.0;
        a.S.beta[j] = 0.0;
      }
    } else if (dj == 0) {
      ++it;
      if (a.S.brk[j] || !(rn == rn)) dj = 2;
      else if (rn <= a.tol * a.S.bnorm[j]) dj = 1;
      else if (it >= a.max_iter) dj = 3;
      if (blockIdx.x == 0) a.S.rnorm[j] = rn;
    }
    if (blockIdx.x == 0) {
      a.S.done_next[j] = dj;
      a.S.iters_next[j] = it;
    }
    live_sh = (dj == 0);
  }
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  double zr = 0.0, zro = 0.0;
  if (live_sh && i < a.s) {
    const int64_t o = (int64_t)j * a.s + i;
    double t;
    if (nseg > 1) {  // the product's segment partials, added in segment order (k_gemm_sum's order)
      t = 0.0;
      for (int sg = 0; sg < nseg; ++sg) t += zpart[((int64_t)sg * a.k + j) * a.s + i];
      a.z[o] = t;
    } else {
      t = a.z[o];
    }
    zr = t * a.r[o];
    zro = (decide == 2) ? 0.0 : t * a.ro[o];
  }
  const double s1 = block_sum<256>(zr, sh);
  const double s2 = block_sum<256>(zro, sh);
  if (threadIdx.x == 0) {
    a.dpart[((int64_t)blockIdx.x * a.k + j) * 2 + 0] = s1;
    a.dpart[((int64_t)blockIdx.x * a.k + j) * 2 + 1] = s2;
  }
}

// active count and largest iteration count of done_next / iters_next (one block)
__device__ __forceinline__ void publish_next(const L2Args& a) {
  __shared__ int cnt, mx;
  if (threadIdx.x == 0) {
    cnt = 0;
    mx = 0;
  }
  __syncthreads();
  for (int jj = threadIdx.x; jj < a.k; jj += 256) {
    atomicAdd(&cnt, a.S.done_next[jj] == 0 ? 1 : 0);
    atomicMax(&mx, a.S.iters_next[jj]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *a.S.active = cnt;
    if (a.mirror) {
      __hip_atomic_store(a.mirror, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(a.mirror + 1, mx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// ---- commit the decision; beta = <z, r - r_old> / rz ; rz = <r, z> ; p = z + beta p.
// One block per column; the last block to finish publishes the active count and the
// largest iteration count.
__global__ void __launch_bounds__(256) k_l2_dir(L2Args a, int first) {
  __shared__ double shs[4];
  const int j = blockIdx.x;
  const int np = a.ndp;
  int dj = a.S.done_next[j];
  // beta's denominator <r_old, z_old> zero or not finite: no conjugate direction exists
  // (an inexact preconditioner that is not positive definite); the column stops as a
  // breakdown and keeps its iterate
  const double rzo = a.S.rz[j];
  if (dj == 0 && !first && !(rzo != 0.0 && isfinite(rzo))) {
    dj = 2;
    __syncthreads();  // every thread has read done_next[j] before thread 0 rewrites it
    if (threadIdx.x == 0) a.S.done_next[j] = 2;
  }
  if (dj == 0) {
    const double zr = strided_sum<256>(a.dpart + (int64_t)j * 2 + 0, np, (int64_t)a.k * 2, shs);
    const double zro = strided_sum<256>(a.dpart + (int64_t)j * 2 + 1, np, (int64_t)a.k * 2, shs);
    const double beta = first ? 0.0 : (zr - zro) / rzo;
    for (int c = threadIdx.x; c < a.s; c += 256) {
      const int64_t o = (int64_t)j * a.s + c;
      a.p[o] = first ? a.z[o] : fma(beta, a.p[o], a.z[o]);
    }
    if (threadIdx.x == 0) {
      a.S.beta[j] = beta;
      a.S.rz[j] = zr;
    }
  }
  if (threadIdx.x == 0) {
    a.S.done[j] = dj;
    a.S.iters[j] = a.S.iters_next[j];
  }
  // one column: publish here; a few: the last block publishes; more: k_l2_publish after
  // this kernel (a device-scope fence in every one of many blocks costs more than a launch)
  if (gridDim.x == 1) {
    publish_next(a);
  } else if (a.k <= kDirFenceMaxK && last_block(a.S.counter)) {
    publish_next(a);
    if (threadIdx.x == 0) *a.S.counter = 0;
  }
}

// ---- active count and largest iteration count of the committed decisions, for the host
__global__ void __launch_bounds__(256) k_l2_publish(L2Args a) { publish_next(a); }

// ---- the inner operator through an explicit s x s matrix W, every column in one pass:
// wp = W v and pqw = v .* (W v) (a wavefront per row of W)
template <int CPL>
__global__ void __launch_bounds__(256) k_w_rows(const double* __restrict__ W, int s, const double* __restrict__ v,
                                               int k, const int32_t* __restrict__ done, double* __restrict__ wp,
                                               double* __restrict__ pqw) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int i = blockIdx.x * 4 + w;
  if (i >= s) return;  // whole wavefronts; no block barrier below
  double m[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int c = lane + q * WAVE;
    m[q] = (c < s) ? W[(int64_t)i * s + c] : 0.0;
  }
  for (int j = 0; j < k; ++j) {
    if (done && done[j]) continue;
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane + q * WAVE;
      t = fma(m[q], (c < s) ? v[(int64_t)j * s + c] : 0.0, t);
    }
    t = wave_sum(t);
    if (lane == 0) {
      wp[(int64_t)j * s + i] = t;
      pqw[(int64_t)j * s + i] = v[(int64_t)j * s + i] * t;
    }
  }
}

template <class TY, int CPL, int KG, int MODE>
hipError_t op_tk(hipStream_t st, const TY* Y, int64_t n, int s, int64_t ldy, const double* v, int64_t ldv, int k,
                 const int32_t* done, double* part, double* pqpart, const double* W, double* wp, double* pqw,
                 int nbC) {
  const int nbW = (MODE == 0 && W) ? (s + 3) / 4 : 0;
  for (int j0 = 0; j0 < k; j0 += KG)
    hipLaunchKernelGGL((k_l2_op<TY, CPL, KG, MODE>), dim3(nbC + nbW), dim3(256), 0, st, Y, n, s, ldy, v, ldv, k, j0,
                       done, part, pqpart, W, wp, pqw, nbC);
  // buffer layout (see l2_op_part_doubles): block partials, then group sums
  double* gpart = part + (size_t)nbC * k * s;
  double* gpq = pqpart ? pqpart + (size_t)nbC * k : nullptr;
  if (nbC > 0)
    hipLaunchKernelGGL(k_l2_gsum, dim3(ngroups(nbC), k), dim3(256), 0, st, part, MODE == 0 ? pqpart : nullptr, nbC,
                       k, s, gpart, gpq);
  return hipGetLastError();
}

// columns per pass: as many as registers allow (4 at <= 8 columns per lane), never
// more than there are right-hand sides
template <class TY, int CPL, int MODE>
hipError_t op_t(hipStream_t st, const TY* Y, int64_t n, int s, int64_t ldy, const double* v, int64_t ldv, int k,
                const int32_t* done, double* part, double* pqpart, const double* W, double* wp, double* pqw,
                int nbC) {
  constexpr int KGMAX = (CPL >= 32) ? 1 : (CPL >= 16 ? 2 : 4);
  if (k == 1 || KGMAX == 1)
    return op_tk<TY, CPL, 1, MODE>(st, Y, n, s, ldy, v, ldv, k, done, part, pqpart, W, wp, pqw, nbC);
  if (k == 2 || KGMAX == 2)
    return op_tk<TY, CPL, (KGMAX >= 2 ? 2 : 1), MODE>(st, Y, n, s, ldy, v, ldv, k, done, part, pqpart, W, wp, pqw, nbC);
  return op_tk<TY, CPL, KGMAX, MODE>(st, Y, n, s, ldy, v, ldv, k, done, part, pqpart, W, wp, pqw, nbC);
}

template <class TY, int MODE>
hipError_t op_dispatch(hipStream_t st, const TY* Y, int64_t n, int s, int64_t ldy, const double* v, int64_t ldv,
                       int k, const int32_t* done, double* part, double* pqpart, const double* W, double* wp,
                       double* pqw, int nbC) {
  const int cpl = (s + WAVE - 1) / WAVE;
#define OPC(C) return op_t<TY, C, MODE>(st, Y, n, s, ldy, v, ldv, k, done, part, pqpart, W, wp, pqw, nbC)
  if (cpl <= 1) OPC(1);
  if (cpl <= 2) OPC(2);
  if (cpl <= 4) OPC(4);
  if (cpl <= 8) OPC(8);
  if (cpl <= 16) OPC(16);
  if (cpl <= 32) OPC(32);
#undef OPC
  return hipErrorInvalidValue;
}

L2Args make_args(const L2Step& a) {
  L2Args x;
  x.s = (int)a.s;
  x.k = (int)a.k;
  x.nbC = a.nbC;
  x.gpart = a.part + (size_t)a.nbC * a.k * a.s;
  x.gpq = a.pqpart ? a.pqpart + (size_t)a.nbC * a.k : nullptr;
  x.wp = a.wp;
  x.pqw = a.pqw;
  x.wscale = a.wscale;
  x.sigma = a.sigma;
  x.y = a.y;
  x.r = a.r;
  x.ro = a.ro;
  x.z = a.z;
  x.p = a.p;
  x.q = a.q;
  x.Minv = a.Minv;
  x.S = a.S;
  x.upart = a.bpart;
  x.dpart = a.bpart + (size_t)ublocks((int)a.s) * a.k + 8;
  x.tol = a.tol;
  x.max_iter = a.max_iter;
  x.mirror = a.mirror;
  x.parent_done = a.parent_done;
  x.rhs = a.rhs;
  x.ndp = mfma_prec(a) ? dblocks((int)a.s) : pblocks((int)a.s);
  return x;
}

__global__ void __launch_bounds__(NTU) k_l2_reduce_to(L2Args a, double* out, const int32_t* skip) {
  __shared__ double sh[NTU];
  const int j = blockIdx.y, lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int c = blockIdx.x * WAVE + lane;
  if (skip && skip[j]) return;
  const double v = reduce_groups_col(a.gpart, ngroups(a.nbC), a.k, a.s, j, c, sh);
  if (w == 0 && c < a.s) out[(int64_t)j * a.s + c] = v;
}

hipError_t prec_launch(hipStream_t st, const L2Step& a, int decide) {
  const int cpl = (int)((a.s + WAVE - 1) / WAVE);
  const unsigned blocks = (unsigned)pblocks((int)a.s);
  L2Args x = make_args(a);
  if (mfma_prec(a)) {
    // columns already done keep their z; at the first application every column is new
    // the segment sum of z is left to k_l2_dots (one launch less per step)
    int nseg = 1;
    hipError_t e = launch_gemm_seg(st, a.Minv, a.s, a.s, a.r, a.s, a.z, a.s, a.k, decide == 2 ? nullptr : a.S.done,
                                   a.gscratch, a.gscratch_n, kSegSmall, &nseg, true);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_l2_dots, dim3((unsigned)dblocks((int)a.s), (unsigned)a.k), dim3(256), 0, st, x, decide,
                       a.gscratch, nseg);
    return hipGetLastError();
  }
  if (cpl <= 1) hipLaunchKernelGGL(k_l2_prec<1>, dim3(blocks), dim3(256), 0, st, x, decide);
  else if (cpl <= 2) hipLaunchKernelGGL(k_l2_prec<2>, dim3(blocks), dim3(256), 0, st, x, decide);
  else if (cpl <= 4) hipLaunchKernelGGL(k_l2_prec<4>, dim3(blocks), dim3(256), 0, st, x, decide);
  else if (cpl <= 8) hipLaunchKernelGGL(k_l2_prec<8>, dim3(blocks), dim3(256), 0, st, x, decide);
  else if (cpl <= 16) hipLaunchKernelGGL(k_l2_prec<16>, dim3(blocks), dim3(256), 0, st, x, decide);
  else if (cpl <= 32) hipLaunchKernelGGL(k_l2_prec<32>, dim3(blocks), dim3(256), 0, st, x, decide);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

int l2_blocks(int64_t n) {
  int64_t b = (n + 31) / 32;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

size_t l2_op_part_doubles(int64_t n, int64_t s, int64_t k) {
  const int nbC = l2_blocks(n);
  return (size_t)(nbC + ngroups(nbC)) * k * s + 64;
}
size_t l2_op_pq_doubles(int64_t n, int64_t k) {
  const int nbC = l2_blocks(n);
  return (size_t)(nbC + ngroups(nbC)) * k + 8;
}
size_t l2_bpart_doubles(int64_t s, int64_t k) {
  return (size_t)ublocks((int)s) * k + 8 + (size_t)pblocks((int)s) * k * 2 + 64;
}

hipError_t l2_op(hipStream_t st, const void* Y, msp_dtype y_t, int64_t n, int64_t s, int64_t ldy, const double* v,
                 int64_t ldv, int64_t k, const int32_t* done, double* part, double* pqpart, const double* W,
                 double* wp, double* pqw, bool rhs_mode) {
  const int nbC = l2_blocks(n);
  const int si = (int)s, ki = (int)k;
  if (y_t == MSP_F64) {
    if (rhs_mode) return op_dispatch<double, 1>(st, (const double*)Y, n, si, ldy, v, ldv, ki, done, part, pqpart, W, wp, pqw, nbC);
    return op_dispatch<double, 0>(st, (const double*)Y, n, si, ldy, v, ldv, ki, done, part, pqpart, W, wp, pqw, nbC);
  }
  if (rhs_mode) return op_dispatch<float, 1>(st, (const float*)Y, n, si, ldy, v, ldv, ki, done, part, pqpart, W, wp, pqw, nbC);
  return op_dispatch<float, 0>(st, (const float*)Y, n, si, ldy, v, ldv, ki, done, part, pqpart, W, wp, pqw, nbC);
}

// the inner operator through an explicit s x s matrix M: wp = M v and pqw = v .* (M v)
// (the W-row part of the Y pass alone; steps built on it use nbC = 0)
hipError_t l2_op_matrix(hipStream_t st, const double* M, int64_t s, const double* v, int64_t k, const int32_t* done,
                        double* wp, double* pqw, double* scratch, size_t scratch_n) {
  if (scratch && k >= kGemmMinK)
    return launch_gemm_seg(st, M, s, s, v, s, wp, s, k, done, scratch, scratch_n, kSegSmall);
  const int cpl = (int)((s + WAVE - 1) / WAVE);
  const unsigned blocks = (unsigned)((s + 3) / 4);
  const int si = (int)s, ki = (int)k;
#define WR(C) hipLaunchKernelGGL(k_w_rows<C>, dim3(blocks), dim3(256), 0, st, M, si, v, ki, done, wp, pqw)
  if (cpl <= 1) WR(1);
  else if (cpl <= 2) WR(2);
  else if (cpl <= 4) WR(4);
  else if (cpl <= 8) WR(8);
  else if (cpl <= 16) WR(16);
  else if (cpl <= 32) WR(32);
  else return hipErrorInvalidValue;
#undef WR
  return hipGetLastError();
}

// rhs reduction, then the first preconditioner application (p = z = Minv r)
hipError_t l2_init(hipStream_t st, const L2Step& a) {
  hipLaunchKernelGGL(k_l2_init, dim3((unsigned)ublocks((int)a.s), (unsigned)a.k), dim3(NTU), 0, st, make_args(a));
  hipError_t e = prec_launch(st, a, 2);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_l2_dir, dim3((unsigned)a.k), dim3(256), 0, st, make_args(a), 1);
  if (a.k > kDirFenceMaxK) hipLaunchKernelGGL(k_l2_publish, dim3(1), dim3(256), 0, st, make_args(a));
  return hipGetLastError();
}

// the right-hand-side kernel alone: r = rhs (zero for finished parent columns), y = 0
hipError_t l2_rhs(hipStream_t st, const L2Step& a) {
  hipLaunchKernelGGL(k_l2_init, dim3((unsigned)ublocks((int)a.s), (unsigned)a.k), dim3(NTU), 0, st, make_args(a));
  return hipGetLastError();
}

hipError_t l2_reduce_to(hipStream_t st, const L2Step& a, double* out, const int32_t* skip) {
  hipLaunchKernelGGL(k_l2_reduce_to, dim3((unsigned)ublocks((int)a.s), (unsigned)a.k), dim3(NTU), 0, st, make_args(a),
                     out, skip);
  return hipGetLastError();
}

// one step after l2_op(p): update, decision + preconditioner, new direction
hipError_t l2_step(hipStream_t st, const L2Step& a, bool publish) {
  if (a.nbC == 0 && a.k >= kUpdateColMinK)
    hipLaunchKernelGGL(k_l2_update_m, dim3((unsigned)a.k), dim3(256), 0, st, make_args(a));
  else
    hipLaunchKernelGGL(k_l2_update, dim3((unsigned)ublocks((int)a.s), (unsigned)a.k), dim3(NTU), 0, st,
                       make_args(a));
  hipError_t e = prec_launch(st, a, 1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_l2_dir, dim3((unsigned)a.k), dim3(256), 0, st, make_args(a), 0);
  if (a.k > kDirFenceMaxK && publish)
    hipLaunchKernelGGL(k_l2_publish, dim3(1), dim3(256), 0, st, make_args(a));
  return hipGetLastError();
}
