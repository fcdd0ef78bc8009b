// Inner flexible-PCG steps on a formed operator in two kernels per step: the level-3 solves
// of Algorithm 5 with the s x s A~^T A~ (+ sigma I) and the s x s preconditioner M3^{-1},
// for blocks of up to kL2fMaxK columns and s <= kL2fMaxS. Step t of the recurrence
//   q_t = (H + sigma I) p_t,  alpha_t = <r_t, z_t> / <p_t, q_t>,  y += alpha_t p_t,
//   r_{t+1} = r_t - alpha_t q_t,  z_{t+1} = Minv r_{t+1},
//   beta_{t+1} = <z_{t+1}, r_{t+1} - r_t> / <r_t, z_t>,  p_{t+1} = z_{t+1} + beta_{t+1} p_t
// runs as
//   k_l2f_op    the decision on |r_t| and beta_t from the previous step's partials (every
//               block sums them in the same order), p_t = z_t + beta_t p_{t-1}, the block's
//               part of q_t and of <p_t, q_t>;
//   k_l2f_prec  alpha_t from those partials (again in every block), y and r_{t+1}, the
//               block's part of z_{t+1} = Minv r_{t+1} and of <z, r_{t+1}>, <z, r_t>,
//               |r_{t+1}|^2.
// The same iteration as the generic step (flexible PCG, Polak-Ribiere beta, the same stop and
// breakdown rules) with the matrix products as plain FP64 row dots: only the summation order
// differs. Both kernels are bound by latency, not bandwidth (the s x s operands stay in the
// caches between steps), so the work is cut for short dependent chains in many blocks: a block
// of eight wavefronts takes rpw rows per wavefront and one segment of kL2fSegW operator
// columns (kL2fSegWSmall when s <= kL2fSegW, for more blocks on the small operators). It
// stages only its segment of the vector it multiplies (formed on the fly from the vectors
// that define it), so the LDS per block and the LDS reads per row do not grow with s. The products are left as one partial per column segment: q_t and
// z_{t+1} exist only as the fixed-order sums of their nseg partials, which the consumers form
// where they read them (every reader of an element forms it with the same expression, so
// every copy has the same bits). The dots are linear in q and z and are taken on the partials.
// Within a kernel every global load that does not wait on the per-column scalars is issued
// first; the wavefront's rpw x 8 row dots are finished by one halving butterfly (32
// exchanges for 32 values instead of 192). At s = 2048 and 8 columns, four rows
// per wavefront (256 blocks, one per CU) measured fastest: more blocks with fewer rows each
// stage the vector more often and run in several rounds.
// p and r alternate between two buffers by step parity (a block reads the previous vector
// while others write the next one); the per-column state is double-buffered the same way.
#include "msp_internal.h"

namespace {

constexpr int WAVE = 64;
constexpr int NWV = kL2fRows;     // wavefronts per block
constexpr int NT = NWV * WAVE;
constexpr int KG = 8;             // columns per staging pass
constexpr int KM = kL2fMaxK;      // columns per launch
// operator columns per block: kL2fSegW, or kL2fSegWSmall for s <= kL2fSegW (more blocks
// for the small operators); at most MAXSEG segments either way
constexpr int MAXSEG = (kL2fMaxS + kL2fSegW - 1) / kL2fSegW;
static_assert((kL2fSegW + kL2fSegWSmall - 1) / kL2fSegWSmall <= MAXSEG, "segment counts");

template <int SW>
struct Seg {
  static constexpr int SPT = KG * SW / NT;  // staged elements per thread
  static_assert(KG * SW % NT == 0, "the staging pass is whole per thread");
  static_assert(SW % WAVE == 0, "segment columns are whole per lane");
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// sums over b < nb of part[b * stride + e + i] for i < NQ, by one wavefront in a fixed order
// (valid in every lane): lane l adds the partials b = l, l + 64, ... in order, four rows of
// partials per round with all their loads issued before the first add
template <int NQ>
__device__ __forceinline__ void wave_parts(const double* __restrict__ part, int nb, int64_t stride, int e,
                                           double (&out)[NQ]) {
  constexpr int U = 4;
  const int lane = threadIdx.x % WAVE;
  double t[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) t[i] = 0.0;
  for (int b0 = 0; b0 < nb; b0 += U * WAVE) {
    double v[U][NQ];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u * WAVE + lane;
#pragma unroll
      for (int i = 0; i < NQ; ++i) v[u][i] = b < nb ? part[(int64_t)b * stride + e + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < NQ; ++i)
        if (b0 + u * WAVE + lane < nb) t[i] += v[u][i];
  }
#pragma unroll
  for (int i = 0; i < NQ; ++i) out[i] = wave_sum(t[i]);
}

// element o of the vector held as NS column-segment partials (stride sk), summed in segment
// order; the one expression every reader uses
template <int NS>
__device__ __forceinline__ double seg_sum(const double* __restrict__ part, int64_t sk, int64_t o) {
  double v = part[o];
#pragma unroll
  for (int g = 1; g < NS; ++g) v += part[(int64_t)g * sk + o];
  return v;
}

// the loads of one staging pass, issued before anything that waits on them: u at the
// segment's elements (j0 + jj, c0 + cc) of this thread and, with want_part, the sum of the
// NS partials there; zero outside the kg columns and the segment
template <int NS, int SW>
__device__ __forceinline__ void load_seg(const double* __restrict__ u, const double* __restrict__ part, bool want_part,
                                         int64_t sk, int j0, int kg, int c0, int cw, int s,
                                         double (&uv)[Seg<SW>::SPT], double (&gv)[Seg<SW>::SPT]) {
#pragma unroll
  for (int q = 0; q < Seg<SW>::SPT; ++q) {
    const int idx = (int)threadIdx.x + q * NT;
    const int jj = idx / SW, cc = idx % SW;
    uv[q] = 0.0;
    gv[q] = 0.0;
    if (jj < kg && cc < cw) {
      const int64_t o = (int64_t)(j0 + jj) * s + c0 + cc;
      uv[q] = u[o];
      if (want_part) gv[q] = seg_sum<NS>(part, sk, o);
    }
  }
}

// h[m][i] = M[row_i][c0 + lane + 64 m] (zero outside the matrix), rows row_i = row0 + NWV i
template <int RPW, int SW>
__device__ __forceinline__ void load_rows(const double* __restrict__ M, int s, int row0, int c0, int cw,
                                          double (&h)[SW / WAVE][RPW]) {
  const int lane = threadIdx.x % WAVE;
#pragma unroll
  for (int m = 0; m < SW / WAVE; ++m) {
    const int cc = lane + WAVE * m;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int row = row0 + NWV * i;
      h[m][i] = (cc < cw && row < s) ? M[(int64_t)row * s + c0 + cc] : 0.0;
    }
  }
}

// acc[i][jj] = sum over the segment's columns of h[.][i] xs[jj][.] (xs is zero outside the
// live columns and the segment)
template <int RPW, int SW>
__device__ __forceinline__ void row_dots(const double (&h)[SW / WAVE][RPW], const double* xs,
                                         double (&acc)[RPW][KG]) {
  const int lane = threadIdx.x % WAVE;
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int jj = 0; jj < KG; ++jj) acc[i][jj] = 0.0;
#pragma unroll
  for (int m = 0; m < SW / WAVE; ++m) {
#pragma unroll
    for (int jj = 0; jj < KG; ++jj) {
      const double x = xs[jj * SW + lane + WAVE * m];
#pragma unroll
      for (int i = 0; i < RPW; ++i) acc[i][jj] = fma(h[m][i], x, acc[i][jj]);
    }
  }
}

constexpr int log2i(int x) { return x <= 1 ? 0 : 1 + log2i(x / 2); }

// wavefront sums of NV values per lane (NV a power of two, at most 64) by a halving
// butterfly: at each of the first log2(NV) exchanges a lane keeps half of its values and adds
// the partner's copy of that half, then log2(64 / NV) exchanges finish the sums. Lane l
// returns the total of value l >> log2(64 / NV) (every value is held by 64 / NV lanes). The
// order of the additions is fixed.
// exchange ST of the halving butterfly and the ones after it (every trip count a constant)
template <int NV, int ST>
__device__ __forceinline__ void halve(double (&v)[NV], int lane) {
  if constexpr (ST <= log2i(NV)) {
    constexpr int h = NV >> ST, msk = WAVE >> ST;
    const bool up = (lane & msk) != 0;
#pragma unroll
    for (int q = 0; q < h; ++q) {
      const double send = up ? v[q] : v[q + h];
      const double keep = up ? v[q + h] : v[q];
      v[q] = keep + __shfl_xor(send, msk, WAVE);
    }
    halve<NV, ST + 1>(v, lane);
  }
}

template <int NV>
__device__ __forceinline__ double scatter_sums(double (&v)[NV]) {
  static_assert(NV >= 1 && NV <= WAVE && (NV & (NV - 1)) == 0, "a power of two up to the wavefront");
  const int lane = threadIdx.x % WAVE;
  halve<NV, 1>(v, lane);
  double r = v[0];
#pragma unroll
  for (int st = 1; st <= log2i(WAVE / NV); ++st) r += __shfl_xor(r, (WAVE / NV) >> st, WAVE);
  return r;
}

// Each pass over up to KG columns issues its loads first (the staged segment, the block's
// own rows of the same vectors, the block's rows of the matrix over the segment), then waits
// for the per-column scalars, forms the staged vector and the own-row values, and takes the
// row products from registers and LDS. Thread tid < KG * RB keeps the own-row element
// (column j0 + tid / RB, row rbase + tid % RB).
template <int RPW, int NS, int SW>
__global__ void __launch_bounds__(NT) k_l2f_op(L2fArgs a, int t, int fresh) {
  constexpr int RB = NWV * RPW;
  static_assert(KG * RB <= NT, "one own-row element per thread");
  __shared__ double xs[KG * SW];
  __shared__ double own[KG][RB];  // p_t at the block's rows
  __shared__ double beta_s[KM];
  __shared__ int live_s[KM];
  __shared__ double red[NWV][RPW][KM];
  constexpr int SH = log2i(WAVE / (RPW * KG));  // lanes per value: 1 << SH
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int par = t & 1, nxt = par ^ 1;
  const int s = a.s, k = a.k;
  const double* pc = a.p[par];
  double* pn = a.p[nxt];
  const int sg = blockIdx.x % NS, rb = blockIdx.x / NS;
  const int c0 = sg * SW, cw = min(SW, s - c0);
  const int rbase = rb * RB, row0 = rbase + w;
  const int ojj = tid / RB, orow = rbase + tid % RB;
  const int64_t sk = (int64_t)s * k;
  double* qp = a.qpart + (int64_t)sg * sk;
  for (int j0 = 0; j0 < k; j0 += KG) {
    const int kg = min(KG, k - j0);
    // p_{t-1} and z_t (p_0 alone when fresh) over the segment and at the own rows; H's rows
    double uv[Seg<SW>::SPT], gv[Seg<SW>::SPT];
    load_seg<NS, SW>(pc, a.zpart, !fresh, sk, j0, kg, c0, cw, s, uv, gv);
    const bool oval = tid < KG * RB && ojj < kg && orow < s;
    const int64_t oo = (int64_t)(j0 + ojj) * s + orow;
    double ou = 0.0, og = 0.0;
    if (oval) {
      ou = pc[oo];
      if (!fresh) og = seg_sum<NS>(a.zpart, sk, oo);
    }
    double h[SW / WAVE][RPW];
    load_rows<RPW, SW>(a.H, s, row0, c0, cw, h);
    if (j0 == 0) {
      // ---- decision on |r_t| and beta_t (the same in every block): wavefront w takes
      // the columns w, w + NWV ----
      for (int j = w; j < k; j += NWV) {
        int dj = fresh ? a.S.done[j] : a.done[par][j];
        int it = fresh ? a.S.iters[j] : a.iters[par][j];
        double rz = fresh ? a.S.rz[j] : a.rz[par][j];
        double beta = 0.0;
        if (!fresh && dj == 0) {  // uniform in the wavefront
          double d[3];
          wave_parts<3>(a.dpart, a.nb, (int64_t)k * 3, j * 3, d);
          const double zr = d[0], zro = d[1], rr = d[2];
          ++it;
          const double rn = sqrt(rr);
          if (a.brk[j] || !(rn == rn)) dj = 2;
          else if (rn <= a.tol * a.S.bnorm[j]) dj = 1;
          else if (it >= a.max_iter) dj = 3;
          if (dj == 0) {
            // beta's denominator <r_{t-1}, z_{t-1}> zero or not finite: no conjugate
            // direction exists; the column stops as a breakdown and keeps its iterate
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
    }
    int any = 0;
    for (int jj = 0; jj < kg; ++jj) any |= live_s[j0 + jj];
    if (!any) {  // uniform in the block
      if (tid < kg)
        for (int ww = 0; ww < NWV; ++ww)
          for (int i = 0; i < RPW; ++i) red[ww][i][j0 + tid] = 0.0;
      continue;
    }
    // p_t = z_t + beta_t p_{t-1} (p_0 when fresh): staged, and at the own rows (segment 0
    // stores it)
#pragma unroll
    for (int q = 0; q < Seg<SW>::SPT; ++q) {
      const int idx = tid + q * NT;
      const int jj = idx / SW, cc = idx % SW;
      const bool on = jj < kg && cc < cw && live_s[j0 + jj];
      xs[idx] = on ? (fresh ? uv[q] : fma(beta_s[j0 + jj], uv[q], gv[q])) : 0.0;
    }
    if (tid < KG * RB) {
      double pv = 0.0;
      if (oval && live_s[j0 + ojj]) {
        pv = fresh ? ou : fma(beta_s[j0 + ojj], ou, og);
        if (sg == 0) pn[oo] = pv;
      }
      own[ojj][tid % RB] = pv;
    }
    __syncthreads();
    double v[RPW * KG];
    {
      double acc[RPW][KG];
      row_dots<RPW, SW>(h, xs, acc);
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int jj = 0; jj < KG; ++jj) v[i * KG + jj] = acc[i][jj];
    }
    // the lead lane of value (i, jj) finishes row row0 + NWV i of column j0 + jj: the
    // segment's part of q_t (with sigma p_t in segment 0) and of <p_t, q_t>
    const double mine = scatter_sums<RPW * KG>(v);
    const int q = lane >> SH, i = q / KG, jj = q % KG;
    if ((lane & ((1 << SH) - 1)) == 0 && jj < kg) {
      const int j = j0 + jj, row = row0 + NWV * i;
      double pq = 0.0;
      if (row < s && live_s[j]) {
        const double pv = own[jj][row - rbase];
        const double qv = sg == 0 ? fma(a.sigma, pv, mine) : mine;
        qp[(int64_t)j * s + row] = qv;
        pq = pv * qv;
      }
      red[w][i][j] = pq;
    }
    __syncthreads();  // xs and own are restaged by the next pass; red is complete
  }
  if (tid < k) {
    double t2 = 0.0;
    for (int ww = 0; ww < NWV; ++ww)
      for (int i = 0; i < RPW; ++i) t2 += red[ww][i][tid];
    a.ppart[(int64_t)blockIdx.x * k + tid] = t2;
  }
}

template <int RPW, int NS, int SW>
__global__ void __launch_bounds__(NT) k_l2f_prec(L2fArgs a, int t) {
  constexpr int RB = NWV * RPW;
  static_assert(KG * RB <= NT, "one own-row element per thread");
  __shared__ double xs[KG * SW];
  __shared__ double own[2][KG][RB];  // r_{t+1} and r_t at the block's rows
  __shared__ double alpha_s[KM];
  __shared__ int live_s[KM];
  __shared__ double red[NWV][RPW][KM][3];
  constexpr int SH = log2i(WAVE / (RPW * KG));
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int par = t & 1, nxt = par ^ 1;
  const int s = a.s, k = a.k;
  const double* rc = a.r[par];
  double* rn = a.r[nxt];
  const double* pn = a.p[nxt];
  const int sg = blockIdx.x % NS, rb = blockIdx.x / NS;
  const int c0 = sg * SW, cw = min(SW, s - c0);
  const int rbase = rb * RB, row0 = rbase + w;
  const int ojj = tid / RB, orow = rbase + tid % RB;
  const int64_t sk = (int64_t)s * k;
  double* zp = a.zpart + (int64_t)sg * sk;
  for (int j0 = 0; j0 < k; j0 += KG) {
    const int kg = min(KG, k - j0);
    // r_t and q_t over the segment and at the own rows (with p_t and y there in segment 0);
    // Minv's rows
    double uv[Seg<SW>::SPT], gv[Seg<SW>::SPT];
    load_seg<NS, SW>(rc, a.qpart, true, sk, j0, kg, c0, cw, s, uv, gv);
    const bool oval = tid < KG * RB && ojj < kg && orow < s;
    const int64_t oo = (int64_t)(j0 + ojj) * s + orow;
    double ou = 0.0, og = 0.0, op = 0.0, oy = 0.0;
    if (oval) {
      ou = rc[oo];
      og = seg_sum<NS>(a.qpart, sk, oo);
      if (sg == 0) {
        op = pn[oo];
        oy = a.y[oo];
      }
    }
    double h[SW / WAVE][RPW];
    load_rows<RPW, SW>(a.Minv, s, row0, c0, cw, h);
    if (j0 == 0) {
      // alpha_t = <r_t, z_t> / <p_t, q_t> (the same in every block)
      for (int j = w; j < k; j += NWV) {
        const int dj = a.done[nxt][j];
        double al = 0.0;
        if (dj == 0) {  // uniform in the wavefront
          double pqs[1];
          wave_parts<1>(a.ppart, a.nb, k, j, pqs);
          const double pq = pqs[0];
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
    }
    int any = 0;
    for (int jj = 0; jj < kg; ++jj) any |= live_s[j0 + jj];
    if (!any) {
      if (tid < kg)
        for (int ww = 0; ww < NWV; ++ww)
          for (int i = 0; i < RPW; ++i)
            for (int e = 0; e < 3; ++e) red[ww][i][j0 + tid][e] = 0.0;
      continue;
    }
    // r_{t+1} = r_t - alpha_t q_t: staged, and at the own rows (segment 0 stores it and
    // y += alpha_t p_t)
#pragma unroll
    for (int q = 0; q < Seg<SW>::SPT; ++q) {
      const int idx = tid + q * NT;
      const int jj = idx / SW, cc = idx % SW;
      const bool on = jj < kg && cc < cw && live_s[j0 + jj];
      xs[idx] = on ? fma(alpha_s[j0 + jj], gv[q], uv[q]) : 0.0;
    }
    if (tid < KG * RB) {
      double rnew = 0.0, rold = 0.0;
      if (oval && live_s[j0 + ojj]) {
        rold = ou;
        rnew = fma(alpha_s[j0 + ojj], og, ou);
        if (sg == 0) {
          a.y[oo] = fma(-alpha_s[j0 + ojj], op, oy);
          rn[oo] = rnew;
        }
      }
      own[0][ojj][tid % RB] = rnew;
      own[1][ojj][tid % RB] = rold;
    }
    __syncthreads();
    double v[RPW * KG];
    {
      double acc[RPW][KG];
      row_dots<RPW, SW>(h, xs, acc);
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int jj = 0; jj < KG; ++jj) v[i * KG + jj] = acc[i][jj];
    }
    // the lead lane of value (i, jj) finishes row row0 + NWV i of column j0 + jj: the
    // segment's part of z_{t+1} and of its two dots; |r_{t+1}|^2 in segment 0
    const double mine = scatter_sums<RPW * KG>(v);
    const int q = lane >> SH, i = q / KG, jj = q % KG;
    if ((lane & ((1 << SH) - 1)) == 0 && jj < kg) {
      const int j = j0 + jj, row = row0 + NWV * i;
      double d0 = 0.0, d1 = 0.0, d2 = 0.0;
      if (row < s && live_s[j]) {
        const double rnew = own[0][jj][row - rbase];
        const double rold = own[1][jj][row - rbase];
        zp[(int64_t)j * s + row] = mine;
        if (sg == 0) d2 = rnew * rnew;
        d0 = mine * rnew;
        d1 = mine * rold;
      }
      red[w][i][j][0] = d0;
      red[w][i][j][1] = d1;
      red[w][i][j][2] = d2;
    }
    __syncthreads();
  }
  if (tid < 3 * k) {
    const int j = tid / 3, e = tid % 3;
    double t2 = 0.0;
    for (int ww = 0; ww < NWV; ++ww)
      for (int i = 0; i < RPW; ++i) t2 += red[ww][i][j][e];
    a.dpart[((int64_t)blockIdx.x * k + j) * 3 + e] = t2;
  }
}

// rows per wavefront: the most (of 4, 2, 1) that still leaves 256 blocks
int pick_rpw(int64_t s, int nseg) {
  for (int r = 4; r > 1; r /= 2)
    if ((s + NWV * r - 1) / (NWV * r) * nseg >= 256) return r;
  return 1;
}

template <int RPW, int NS, int SW>
hipError_t launch_pair(hipStream_t st, const L2fArgs& a, int t, int fresh, bool op) {
  if (op)
    hipLaunchKernelGGL((k_l2f_op<RPW, NS, SW>), dim3((unsigned)a.nb), dim3(NT), 0, st, a, t, fresh);
  else
    hipLaunchKernelGGL((k_l2f_prec<RPW, NS, SW>), dim3((unsigned)a.nb), dim3(NT), 0, st, a, t);
  return hipGetLastError();
}

template <int RPW, int SW>
hipError_t launch_ns(hipStream_t st, const L2fArgs& a, int t, int fresh, bool op) {
  static_assert(MAXSEG == 4, "one instantiation per segment count");
  switch (a.nseg) {
    case 1: return launch_pair<RPW, 1, SW>(st, a, t, fresh, op);
    case 2: return launch_pair<RPW, 2, SW>(st, a, t, fresh, op);
    case 3: return launch_pair<RPW, 3, SW>(st, a, t, fresh, op);
    case 4: return launch_pair<RPW, 4, SW>(st, a, t, fresh, op);
  }
  return hipErrorInvalidValue;
}

hipError_t launch(hipStream_t st, const L2fArgs& a, int t, int fresh, bool op) {
  int nseg = 0, rpw = 0, nb = 0, segw = 0;
  if (a.s < 1 || a.s > kL2fMaxS || a.k < 1 || a.k > kL2fMaxK) return hipErrorInvalidValue;
  l2f_shape(a.s, &nseg, &rpw, &nb, &segw);
  if (a.nseg != nseg || a.rpw != rpw || a.nb != nb || a.segw != segw) return hipErrorInvalidValue;
  if (a.segw == kL2fSegWSmall) {  // s <= kL2fSegW: one row per wavefront (pick_rpw)
    if (a.rpw != 1) return hipErrorInvalidValue;
    return launch_ns<1, kL2fSegWSmall>(st, a, t, fresh, op);
  }
  switch (a.rpw) {
    case 1: return launch_ns<1, kL2fSegW>(st, a, t, fresh, op);
    case 2: return launch_ns<2, kL2fSegW>(st, a, t, fresh, op);
    case 4: return launch_ns<4, kL2fSegW>(st, a, t, fresh, op);
  }
  return hipErrorInvalidValue;
}

}  // namespace

void l2f_shape(int64_t s, int* nseg, int* rpw, int* nb, int* segw) {
  *segw = s <= kL2fSegW ? kL2fSegWSmall : kL2fSegW;
  *nseg = (int)((s + *segw - 1) / *segw);
  *rpw = pick_rpw(s, *nseg);
  *nb = (int)((s + NWV * *rpw - 1) / (NWV * *rpw)) * *nseg;
}

L2fArgs l2f_carve(WsCarver& w, int64_t s, int64_t k) {
  L2fArgs a{};
  a.s = (int)s;
  a.k = (int)k;
  l2f_shape(s, &a.nseg, &a.rpw, &a.nb, &a.segw);
  a.p[1] = w.take<double>(s * k);
  a.rz[0] = w.take<double>(k);
  a.rz[1] = w.take<double>(k);
  a.alpha = w.take<double>(k);
  a.ppart = w.take<double>((size_t)a.nb * k);
  a.dpart = w.take<double>((size_t)a.nb * k * 3);
  a.qpart = w.take<double>((size_t)a.nseg * s * k);
  a.zpart = w.take<double>((size_t)a.nseg * s * k);
  a.done[0] = w.take<int32_t>(k);
  a.done[1] = w.take<int32_t>(k);
  a.iters[0] = w.take<int32_t>(k);
  a.iters[1] = w.take<int32_t>(k);
  a.brk = w.take<int32_t>(k);
  return a;
}

hipError_t l2f_op(hipStream_t st, const L2fArgs& a, int t, int fresh) { return launch(st, a, t, fresh, true); }

hipError_t l2f_prec(hipStream_t st, const L2fArgs& a, int t) { return launch(st, a, t, 0, false); }
