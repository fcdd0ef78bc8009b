// Batched two-level MSP (Algorithms 1-2) for many independent PSD systems of uneven
// size in a single launch. Each workgroup owns one system and runs its whole solve:
// the level-1 flexible PCG on (A_lo + lam I) x = b, SolveM1 (level-2 flexible PCG
// preconditioned by M2^{-1}, then w = (r - C y) / lam~) for every level-1 step, the
// confirmation on the residual recomputed from A_hi, and optionally an outer FP64
// Krylov refinement on A_hi that uses the low-precision MSP solve as its flexible
// preconditioner. Nothing crosses workgroups, so there are no grid-wide waits and no
// host round trips; the hardware dispatcher hands systems to compute units as they
// free up (the host orders systems by decreasing work).
//
// Inside a workgroup (16 wavefronts, up to 16 right-hand sides):
//  * vector work: wavefront j owns column j (axpys, dots, the FCG scalars);
//  * matrix products: all wavefronts share row tiles and use 16x16x4 matrix-core
//    instructions with the 16 columns as the N dimension:
//      A-sweeps (F32 MFMA for F32/BF16 storage, F64 MFMA for F64 storage and for the
//      FP64 residuals), Y^T r, Y y, and the s x s products with M2^{-1} and with
//      H = C^T C + lam~ W.
//  The level-2 operator (C^T C + lam~ W) y is applied through H, formed once per
//  system by the host; this is the same operator as C^T (C y) + lam~ W y, evaluated
//  with s^2 instead of n s work per inner step.
//
// Teams. One compute unit streams only about 1/256 of the chip's bandwidth, so a batch
// is bound by its largest systems. A workgroup whose system is finished joins a larger
// unfinished one as a helper: the system's workgroup (the leader) publishes every A-sweep
// as an epoch in the system's team record, and the row range is cut into 512-row chunks
// handed out as slices (the Y^T r and Y y passes of SolveM1 are team jobs too). Every chunk writes its own <x, A x> partials and the leader adds
// them in chunk order, so the result is the same bits whoever computed which chunk. All
// waits are bounded by wall-clock time: a slice that no helper claims in time is taken
// by the leader, and an idle helper leaves.
#include "msp_batched.h"

#include <hip/hip_bf16.h>

namespace {

constexpr int WAVE = 64;
constexpr int NW = 16;           // wavefronts per workgroup
constexpr int NTB = NW * WAVE;   // 1024 threads
constexpr int KB = MSP_BATCH_KMAX;
constexpr int MAX_RESTARTS = 8;
constexpr int CRT = 2;              // 16-row MFMA tiles per wavefront and chunk
constexpr int CHR = MSP_BATCH_CHR;  // rows per chunk: NW wavefronts x one 32-row tile
constexpr int MAXH = MSP_BATCH_MAXH;
static_assert(CHR == NW * 16 * CRT, "a chunk is one tile row set per wavefront");
// wall-clock (100 MHz) bounds of the team waits
constexpr uint64_t CLAIM_TICKS = 10000;       // 100 us: a live helper claims its slice sooner
constexpr uint64_t SLICE_TICKS = 500000000;   // 5 s: a claimed slice must be done by then
constexpr uint64_t IDLE_TICKS = 200000000;    // 2 s without a new epoch: the helper leaves

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef uint32_t nu4 __attribute__((ext_vector_type(4)));

template <class TC>
struct V4;
template <>
struct V4<float> {
  typedef v4f t;
};
template <>
struct V4<double> {
  typedef v4d t;
};

__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Output placement of the 16x16 tiles: element e of lane l holds row out_row(l / 16, e)
// and column l % 16 (F32: rows 4 (l / 16) + e; F64: rows 4 e + l / 16).
template <class TC>
__device__ __forceinline__ int out_row(int g, int e) {
  return sizeof(TC) == 4 ? 4 * g + e : 4 * e + g;
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// Global-memory view of a pointer (the pointers reach the kernel through a descriptor
// table, so the compiler cannot infer the address space and would emit flat accesses)
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gv(const void* p) {
  return (const __attribute__((address_space(1))) T*)(p);
}

// Loads of VEC consecutive matrix elements (one 16-byte access when aligned), converted
// to the arithmetic type TC.
template <class TA, class TC>
struct Ld;
template <>
struct Ld<double, double> {
  static constexpr int VEC = 2;
  template <bool NTL>
  __device__ static void vec(const double* p, double* o) {
    nd2 v;
    if constexpr (NTL) v = __builtin_nontemporal_load(gv<nd2>(p));
    else v = *gv<nd2>(p);
    o[0] = v.x;
    o[1] = v.y;
  }
  __device__ static double one(const double* p) { return *p; }
};
template <>
struct Ld<float, float> {
  static constexpr int VEC = 4;
  template <bool NTL>
  __device__ static void vec(const float* p, float* o) {
    nf4 v;
    if constexpr (NTL) v = __builtin_nontemporal_load(gv<nf4>(p));
    else v = *gv<nf4>(p);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
  __device__ static float one(const float* p) { return *p; }
};
template <>
struct Ld<float, double> {
  static constexpr int VEC = 4;
  template <bool NTL>
  __device__ static void vec(const float* p, double* o) {
    nf4 v;
    if constexpr (NTL) v = __builtin_nontemporal_load(gv<nf4>(p));
    else v = *gv<nf4>(p);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
  __device__ static double one(const float* p) { return (double)*p; }
};
template <>
struct Ld<__hip_bfloat16, float> {
  static constexpr int VEC = 8;
  template <bool NTL>
  __device__ static void vec(const __hip_bfloat16* p, float* o) {
    nu4 v;
    if constexpr (NTL) v = __builtin_nontemporal_load(gv<nu4>(p));
    else v = *gv<nu4>(p);
    o[0] = bf_lo(v.x);
    o[1] = bf_hi(v.x);
    o[2] = bf_lo(v.y);
    o[3] = bf_hi(v.y);
    o[4] = bf_lo(v.z);
    o[5] = bf_hi(v.z);
    o[6] = bf_lo(v.w);
    o[7] = bf_hi(v.w);
  }
  __device__ static float one(const __hip_bfloat16* p) { return __bfloat162float(*p); }
};

// VEC consecutive entries of an operand vector (16-byte aligned by construction)
template <class TC, int VEC>
__device__ __forceinline__ void ld_b(const TC* p, TC* o) {
  if constexpr (sizeof(TC) == 4) {
#pragma unroll
    for (int q = 0; q < VEC / 4; ++q) {
      const nf4 v = *gv<nf4>(p + 4 * q);
      o[4 * q] = v.x;
      o[4 * q + 1] = v.y;
      o[4 * q + 2] = v.z;
      o[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < VEC / 2; ++q) {
      const nd2 v = *gv<nd2>(p + 2 * q);
      o[2 * q] = v.x;
      o[2 * q + 1] = v.y;
    }
  }
}

// One wavefront: acc[t] = A[r0 + 16 t + (0..15), 0:ncols] * Bv[0:ncols, 0..15] for t < RT.
// Bv holds column j at Bv + j * ldb (columns >= k read column k - 1; their outputs are
// not used). Lane l supplies row r0 + 16 t + l % 16 and the reduction slice
// [c0 + VEC (l / 16), +VEC) of each step; both operands use the same slice, so the
// product is exact in any order of the reduction index. Output element e of acc[t]
// in lane l is row r0 + 16 t + out_row(l / 16, e), column l % 16. Rows past nrows read
// row nrows - 1 and are not written by the callers.
template <class TA, class TC, int RT, bool ALN, bool NTL>
__device__ __forceinline__ void mm_rows(const TA* __restrict__ A, int64_t lda, int nrows, int ncols, int r0,
                                        const TC* __restrict__ Bv, int64_t ldb, int k,
                                        typename V4<TC>::t (&acc)[RT]) {
  using L = Ld<TA, TC>;
  constexpr int VEC = L::VEC;
  constexpr int STEP = 4 * VEC;
  const int lane = threadIdx.x & (WAVE - 1), i = lane & 15, g = lane >> 4;
  const int jb = i < k ? i : k - 1;
  const TC* bp = Bv + (int64_t)jb * ldb + VEC * g;
  const TA* ap[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int r = min(r0 + 16 * t + i, nrows - 1);
    ap[t] = A + (int64_t)r * lda + VEC * g;
    acc[t] = typename V4<TC>::t{0, 0, 0, 0};
  }
  int c0 = 0;
  if constexpr (ALN) {
    // trips of UN steps, double-buffered: the loads of trip t + 1 are in flight while
    // the MFMAs of trip t run
    constexpr int REGS = RT * VEC * (int)sizeof(TC) / 4;
    constexpr int UN = REGS >= 32 ? 1 : (REGS >= 16 ? 2 : (REGS >= 8 ? 4 : 8));
    constexpr int TRIP = UN * STEP;
    struct Buf {
      TC a[UN][RT][VEC];
      TC b[UN][VEC];
    };
    auto load = [&](Buf& x, int cb) {
#pragma unroll
      for (int u = 0; u < UN; ++u) {
#pragma unroll
        for (int t = 0; t < RT; ++t) L::template vec<NTL>(ap[t] + cb + u * STEP, x.a[u][t]);
        ld_b<TC, VEC>(bp + cb + u * STEP, x.b[u]);
      }
    };
    auto run = [&](const Buf& x) {
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int m = 0; m < VEC; ++m)
#pragma unroll
          for (int t = 0; t < RT; ++t) acc[t] = mfma(x.a[u][t][m], x.b[u][m], acc[t]);
    };
    const int T = ncols / TRIP;
    if (T > 0) {
      Buf x0, x1;
      load(x0, 0);
      int t = 0;
      for (; t + 2 <= T; t += 2) {
        load(x1, (t + 1) * TRIP);
        run(x0);
        if (t + 2 < T) load(x0, (t + 2) * TRIP);
        run(x1);
      }
      if (t < T) run(x0);
      c0 = T * TRIP;
    }
    for (; c0 + STEP <= ncols; c0 += STEP) {
      TC a[RT][VEC], b[VEC];
#pragma unroll
      for (int t = 0; t < RT; ++t) L::template vec<NTL>(ap[t] + c0, a[t]);
      ld_b<TC, VEC>(bp + c0, b);
#pragma unroll
      for (int m = 0; m < VEC; ++m)
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[t] = mfma(a[t][m], b[m], acc[t]);
    }
  }
  for (; c0 < ncols; c0 += STEP) {
    TC a[RT][VEC], b[VEC];
#pragma unroll
    for (int m = 0; m < VEC; ++m) {
      const bool ok = c0 + VEC * g + m < ncols;
      b[m] = ok ? bp[c0 + m] : (TC)0;
#pragma unroll
      for (int t = 0; t < RT; ++t) a[t][m] = ok ? L::one(ap[t] + c0 + m) : (TC)0;
    }
#pragma unroll
    for (int m = 0; m < VEC; ++m)
#pragma unroll
      for (int t = 0; t < RT; ++t) acc[t] = mfma(a[t][m], b[m], acc[t]);
  }
}

// Row-tile pass of the workgroup: wavefront w takes row tiles w, w + NW, ... and calls
// epi(j, row, value) for every output row < nrows and column j < k.
template <class TA, class TC, int RT, bool NTL, class Epi>
__device__ __forceinline__ void rows_pass(const TA* A, int64_t lda, int nrows, int ncols, bool aln, const TC* Bv,
                                          int64_t ldb, int k, Epi epi) {
  const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1), i = lane & 15, g = lane >> 4;
  for (int r0 = w * 16 * RT; r0 < nrows; r0 += NW * 16 * RT) {
    typename V4<TC>::t acc[RT];
    if (aln) mm_rows<TA, TC, RT, true, NTL>(A, lda, nrows, ncols, r0, Bv, ldb, k, acc);
    else mm_rows<TA, TC, RT, false, NTL>(A, lda, nrows, ncols, r0, Bv, ldb, k, acc);
    if (i < k) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = r0 + 16 * t + out_row<TC>(g, e);
          if (row < nrows) epi(i, row, (double)acc[t][e]);
        }
    }
  }
}

// Per-column FCG scalars of one level (shared memory)
struct Cols {
  double rz[KB], bn[KB], rn[KB], pq[KB], rel[KB];
  int done[KB], it[KB];
};
// done: 0 active, 1 converged by the recurrence, 2 breakdown, 3 iteration cap,
//       4 finished (confirmed, zero right-hand side, or not asked for)

struct Ctx {
  BatchSys S;
  BatchPrm P;
  int k, n, s, ldn, lds;
  double *xh, *rh, *roh, *ph, *qh, *zh;
  double *r1, *ro1, *z1, *p1, *q1;
  double *r2, *ro2, *z2, *p2, *q2, *y2, *b2;
  float* pf;
  Cols *CH, *C1, *C2;
  double lam_lo;  // shift of the low-precision sweeps: lam, plus delta under refinement
  double* red;   // [NW][256]
  double* part;  // [NW][KB]
  int* shi;      // [8] LDS ints for broadcasts
  int epoch;     // thread 0: last published sweep epoch
  int team_err;  // thread 0: a claimed slice timed out
  int helped, selfdone;  // thread 0: slices done by helpers / taken back by the leader
  int outer, inner, refine, restarts;
  uint64_t ticks[BT_NPHASE];  // thread 0, when P.profile
};

// wall-clock phase timer (thread 0 of the workgroup; phases end on a barrier)
struct PhaseTimer {
  Ctx& c;
  int ph;
  uint64_t t0;
  __device__ PhaseTimer(Ctx& cc, int p) : c(cc), ph(p), t0(0) {
    if (c.P.profile && threadIdx.x == 0) t0 = wall_clock64();
  }
  __device__ ~PhaseTimer() {
    if (c.P.profile && threadIdx.x == 0) c.ticks[ph] += wall_clock64() - t0;
  }
};

__device__ __forceinline__ int wave_id() { return threadIdx.x / WAVE; }
__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// true in every thread if some column j < k of C is active (call after a barrier)
__device__ __forceinline__ bool any_active(const Cols* C, int k) {
  bool a = false;
  for (int j = 0; j < k; ++j) a = a || (C->done[j] == 0);
  return a;
}

// ---- one A-sweep as chunked work ---------------------------------------------------
// mode 0/1: out = (A + lam I) x with per-chunk partials <x, out>; mode 2: out = rhs -
// (A + lam I) x. Bv is x in the arithmetic type (the F32 copy for low-precision A).
struct Job {
  const void* A;
  int64_t lda;
  const void* Bv;  // x in the arithmetic type, ld ldb
  int64_t ldb;
  const double* x;
  const double* rhs;
  int64_t ldr;
  double* out;
  double* cpart;
  double lam;
  int n, ncols, ldn, k, mode, aln;
};

template <class TA, class TC>
__device__ void sweep_chunks(const Job& J, int ch0, int ch1, double* part /*LDS NW*KB*/) {
  const int w = wave_id(), lane = lane_id(), i = lane & 15, g = lane >> 4;
  for (int ch = ch0; ch < ch1; ++ch) {
    const int r0 = ch * CHR + w * 16 * CRT;
    double pq = 0.0;
    if (r0 < J.n) {
      typename V4<TC>::t acc[CRT];
      if (J.aln)
        mm_rows<TA, TC, CRT, true, true>((const TA*)J.A, J.lda, J.n, J.ncols, r0, (const TC*)J.Bv, J.ldb, J.k, acc);
      else
        mm_rows<TA, TC, CRT, false, true>((const TA*)J.A, J.lda, J.n, J.ncols, r0, (const TC*)J.Bv, J.ldb, J.k, acc);
      if (i < J.k) {
#pragma unroll
        for (int t = 0; t < CRT; ++t)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int row = r0 + 16 * t + out_row<TC>(g, e);
            if (row < J.n) {
              const int64_t o = (int64_t)i * J.ldn + row;
              const double xv = J.x[o];
              const double q = (double)acc[t][e] + J.lam * xv;
              if (J.mode == 2) {
                J.out[o] = J.rhs[(int64_t)i * J.ldr + row] - q;
              } else {
                J.out[o] = q;
                pq = fma(xv, q, pq);
              }
            }
          }
      }
    }
    // the chunk's partial per column: lanes l, l+16, l+32, l+48 hold column l
    pq += __shfl_xor(pq, 16, WAVE);
    pq += __shfl_xor(pq, 32, WAVE);
    if (lane < KB) part[w * KB + lane] = pq;
    __syncthreads();
    if (threadIdx.x < (unsigned)J.k) {
      double t = 0.0;
      for (int q = 0; q < NW; ++q) t += part[q * KB + threadIdx.x];
      J.cpart[(int64_t)ch * KB + threadIdx.x] = t;
    }
    __syncthreads();
  }
}


// mode 3: out = (rhs - Y x) * lam on the rows of the chunks (x: s-vectors, ld ldb)
template <class TY>
__device__ void yz_chunks(const Job& J, int ch0, int ch1) {
  const int w = wave_id(), lane = lane_id(), i = lane & 15, g = lane >> 4;
  for (int ch = ch0; ch < ch1; ++ch) {
    const int r0 = ch * CHR + w * 16 * CRT;
    if (r0 >= J.n) continue;
    v4d acc[CRT];
    if (J.aln)
      mm_rows<TY, double, CRT, true, false>((const TY*)J.A, J.lda, J.n, J.ncols, r0, (const double*)J.Bv, J.ldb, J.k,
                                            acc);
    else
      mm_rows<TY, double, CRT, false, false>((const TY*)J.A, J.lda, J.n, J.ncols, r0, (const double*)J.Bv, J.ldb, J.k,
                                             acc);
    if (i < J.k) {
#pragma unroll
      for (int t = 0; t < CRT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = r0 + 16 * t + out_row<double>(g, e);
          if (row < J.n) {
            const int64_t o = (int64_t)i * J.ldn + row;
            J.out[o] = (J.rhs[(int64_t)i * J.ldr + row] - acc[t][e]) * J.lam;
          }
        }
    }
  }
}

// mode 4: out[ch][j][c] = sum over the rows of chunk ch of Y[row, c] rhs_j[row]; the
// 16-column tiles of Y are the MFMA rows and the chunk's rows the reduction
template <class TY>
__device__ void ytr_chunks(const Job& J, int ch0, int ch1) {
  const int w = wave_id(), lane = lane_id(), i = lane & 15, g = lane >> 4;
  const int s = J.ncols;
  const int T = (s + 15) / 16;
  const int jb = i < J.k ? i : J.k - 1;
  const TY* Y = (const TY*)J.A;
  const double* V = J.rhs + (int64_t)jb * J.ldr;
  for (int ch = ch0; ch < ch1; ++ch) {
    const int rb = ch * CHR, re = min(J.n, rb + CHR);
    for (int tile = w; tile < T; tile += NW) {
      const int c0 = tile * 16;
      const int col = min(c0 + i, s - 1);
      v4d acc = {0, 0, 0, 0};
      int r = rb;
      for (; r + 64 <= re; r += 64) {
        double a[16], b[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int row = r + 4 * u + g;
          a[u] = (double)Y[(int64_t)row * J.lda + col];
          b[u] = V[row];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) acc = mfma(a[u], b[u], acc);
      }
      for (; r < re; r += 16) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int row = r + 4 * u + g;
          const bool ok = row < re;
          a[u] = ok ? (double)Y[(int64_t)row * J.lda + col] : 0.0;
          b[u] = ok ? V[row] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = mfma(a[u], b[u], acc);
      }
      if (i < J.k)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int cc = c0 + out_row<double>(g, e);
          if (cc < s) J.out[((int64_t)ch * KB + i) * s + cc] = acc[e];
        }
    }
  }
}

template <class TLO, class THI, class TY>
__device__ void do_chunks(const Job& J, int ch0, int ch1, double* part) {
  if (J.mode == 0) {
    if constexpr (sizeof(TLO) == 8) sweep_chunks<TLO, double>(J, ch0, ch1, part);
    else sweep_chunks<TLO, float>(J, ch0, ch1, part);
  } else if (J.mode <= 2) {
    sweep_chunks<THI, double>(J, ch0, ch1, part);
  } else if (J.mode == 3) {
    yz_chunks<TY>(J, ch0, ch1);
    __syncthreads();
  } else {
    ytr_chunks<TY>(J, ch0, ch1);
    __syncthreads();
  }
}

__device__ __forceinline__ int ld_acq(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
// polling without cache maintenance; acquire once the awaited value is seen
__device__ __forceinline__ int ld_rlx(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_acq() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void st_rel(int32_t* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas_claim(int32_t* p, int e) {
  int cur = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (cur == e) return false;
  return __hip_atomic_compare_exchange_strong(p, &cur, e, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int slice_begin(int s, int nslice, int nch) { return (int)((int64_t)s * nch / nslice); }

// the leader's sweep: slices for the helpers that joined (published as a new epoch),
// slice 0 itself, then every other slice done by a helper or, unclaimed, by itself
template <class TLO, class THI, class TY>
__device__ void run_job(Ctx& c, const Job& J) {
  const int nch = (J.n + CHR - 1) / CHR;
  BatchTeam* T = c.S.team;
  if (threadIdx.x == 0) {
    int H = 0;
    if (c.P.teams && T && nch > 1) {
      H = min(__hip_atomic_load(&T->joined, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), MAXH);
      H = min(H, nch - 1);
    }
    if (H > 0) {
      T->bv = J.Bv;
      T->ldb = J.ldb;
      T->ncols = J.ncols;
      T->x = J.x;
      T->rhs = J.rhs;
      T->out = J.out;
      T->ldr = J.ldr;
      T->lam = J.lam;
      T->mode = J.mode;
      T->nslice = H + 1;
      c.epoch += 1;
      st_rel(&T->epoch, c.epoch);  // after the barrier that ended the writes of x
    }
    c.shi[0] = H;
  }
  __syncthreads();
  const int H = c.shi[0];
  do_chunks<TLO, THI, TY>(J, 0, slice_begin(1, H + 1, nch), c.part);
  for (int s = 1; s <= H; ++s) {
    if (threadIdx.x == 0) {
      int self = 0;
      const uint64_t t0 = wall_clock64();
      while (true) {
        if (ld_rlx(&T->done[s]) == c.epoch) {
          fence_acq();
          c.helped += 1;
          break;
        }
        const uint64_t dt = wall_clock64() - t0;
        if (dt > CLAIM_TICKS && cas_claim(&T->claim[s], c.epoch)) {
          self = 1;
          c.selfdone += 1;
          break;
        }
        if (dt > SLICE_TICKS) {
          c.team_err = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      c.shi[1] = self;
    }
    __syncthreads();
    if (c.shi[1]) do_chunks<TLO, THI, TY>(J, slice_begin(s, H + 1, nch), slice_begin(s + 1, H + 1, nch), c.part);
  }
  __syncthreads();
}

// sum of the chunk partials in chunk order -> C->pq (columns < k)
__device__ __forceinline__ void chunk_sum(const Ctx& c, const double* cpart, Cols* C) {
  const int nch = (c.n + CHR - 1) / CHR;
  if (threadIdx.x < (unsigned)c.k) {
    double t = 0.0;
    for (int ch = 0; ch < nch; ++ch) t += cpart[(int64_t)ch * KB + threadIdx.x];
    C->pq[threadIdx.x] = t;
  }
  __syncthreads();
}

template <class TLO, class THI, class TY>
struct Batch {
  // ---- matrix products -----------------------------------------------------------
  // q1 = (A_lo + lam_lo I) p1 and C1->pq = <p1, q1>
  static __device__ void op_lo(Ctx& c) {
    PhaseTimer tm(c, BT_SWEEP_LO);
    const int w = wave_id(), lane = lane_id();
    Job J{c.S.A_lo, c.S.lda, c.p1, c.ldn, c.p1, nullptr, 0, c.q1, c.S.cpart, c.lam_lo, c.n, c.n, c.ldn, c.k, 0,
          c.S.aln_lo};
    if constexpr (sizeof(TLO) != 8) {
      if (w < c.k)
        _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) c.pf[(int64_t)w * c.ldn + i] = (float)c.p1[(int64_t)w * c.ldn + i];
      J.Bv = c.pf;
    }
    __syncthreads();
    run_job<TLO, THI, TY>(c, J);
    chunk_sum(c, c.S.cpart, c.C1);
  }

  // FP64 products with A_hi: mode 0: qh = (A_hi + lam I) ph, CH->pq = <ph, qh>;
  // mode 1: out = rhs - (A_hi + lam I) x
  static __device__ void op_hi(Ctx& c, int mode, const double* x, const double* rhs, int64_t ldr, double* out) {
    PhaseTimer tm(c, BT_SWEEP_HI);
    const Job J{c.S.A_hi, c.S.lda, x, c.ldn, x, rhs, ldr, out, c.S.cpart, c.S.lam, c.n, c.n, c.ldn, c.k,
                mode == 0 ? 1 : 2, c.S.aln_hi};
    __syncthreads();
    run_job<TLO, THI, TY>(c, J);
    if (mode == 0) chunk_sum(c, c.S.cpart, c.CH);
  }

  // out = M v for an s x s FP64 matrix (row-major, ld s); v, out: s-vectors
  static __device__ void smv(Ctx& c, const double* M, const double* v, double* out) {
    auto epi = [&](int j, int row, double val) { out[(int64_t)j * c.lds + row] = val; };
    rows_pass<double, double, 1, false>(M, c.s, c.s, c.s, c.S.aln_m, v, c.lds, c.k, epi);
    __syncthreads();
  }

  // z1 = (r1 - Y y2) / lam~ (written for every column; only active ones are read)
  static __device__ void y_z(Ctx& c) {
    PhaseTimer tm(c, BT_YZ);
    const Job J{c.S.Y, c.S.ldy, c.y2, c.lds, nullptr, c.r1, c.ldn, c.z1, nullptr, 1.0 / c.S.lt, c.n, c.s, c.ldn, c.k, 3,
                c.S.aln_y};
    __syncthreads();
    run_job<TLO, THI, TY>(c, J);
  }

  // b2 = Y^T r1 from chunk partials (each 512 rows: 16-column tiles of Y as MFMA rows, the
  // chunk's rows as the reduction), added in chunk order
  static __device__ void yt_r(Ctx& c) {
    PhaseTimer tm(c, BT_YT);
    const Job J{c.S.Y, c.S.ldy, nullptr, 0, nullptr, c.r1, c.ldn, c.S.ypart, nullptr, 0.0, c.n, c.s, c.ldn, c.k, 4,
                c.S.aln_y};
    __syncthreads();
    run_job<TLO, THI, TY>(c, J);
    const int nch = (c.n + CHR - 1) / CHR;
    for (int t = threadIdx.x; t < c.k * c.s; t += NTB) {
      const int j = t / c.s, cc = t % c.s;
      double v = 0.0;
      for (int ch = 0; ch < nch; ++ch) v += c.S.ypart[((int64_t)ch * KB + j) * c.s + cc];
      c.b2[(int64_t)j * c.lds + cc] = v;
    }
    __syncthreads();
  }

  // max_i sum_j |A_hi[i, j]| (FP64), identical in every thread
  static __device__ double norm_inf_hi(Ctx& c) {
    const int w = wave_id(), lane = lane_id();
    const THI* A = (const THI*)c.S.A_hi;
    double mx = 0.0;
    for (int r = w; r < c.n; r += NW) {
      double t = 0.0;
      for (int j = lane; j < c.n; j += WAVE) t += fabs((double)A[(int64_t)r * c.S.lda + j]);
      mx = fmax(mx, wsum(t));
    }
    if (lane == 0) c.part[w] = mx;
    __syncthreads();
    double m = 0.0;
    for (int q = 0; q < NW; ++q) m = fmax(m, c.part[q]);
    __syncthreads();
    return m;
  }

  // ---- Algorithm 2: z1 = SolveM1(r1) for the columns active at level 1 -------------
  static __device__ void solve_m1(Ctx& c) {
    const int w = wave_id(), lane = lane_id();
    Cols* D = c.C2;
    yt_r(c);
    if (w < c.k) {
      const bool act = c.C1->done[w] == 0;
      double acc = 0.0;
      _Pragma("unroll 4") for (int i = lane; i < c.s; i += WAVE) {
        const int64_t o = (int64_t)w * c.lds + i;
        const double v = act ? c.b2[o] : 0.0;
        c.r2[o] = v;
        c.y2[o] = 0.0;
        acc = fma(v, v, acc);
      }
      const double bn = sqrt(wsum(acc));
      if (lane == 0) {
        D->bn[w] = bn;
        D->rn[w] = bn;
        D->it[w] = 0;
        D->done[w] = (!act || bn == 0.0) ? 4 : 0;
      }
    }
    __syncthreads();
    const uint64_t l2t0 = (c.P.profile && threadIdx.x == 0) ? wall_clock64() : 0;
    smv(c, c.S.Minv, c.r2, c.z2);
    if (w < c.k && D->done[w] == 0) {
      double acc = 0.0;
      _Pragma("unroll 4") for (int i = lane; i < c.s; i += WAVE) {
        const int64_t o = (int64_t)w * c.lds + i;
        const double z = c.z2[o];
        c.p2[o] = z;
        acc = fma(c.r2[o], z, acc);
      }
      acc = wsum(acc);
      if (lane == 0) D->rz[w] = acc;
    }
    int it = 0;
    while (it < c.P.max_inner) {
      __syncthreads();
      if (!any_active(D, c.k)) break;
      smv(c, c.S.H, c.p2, c.q2);
      if (w < c.k && D->done[w] == 0) {
        double pq = 0.0;
        _Pragma("unroll 4") for (int i = lane; i < c.s; i += WAVE) {
          const int64_t o = (int64_t)w * c.lds + i;
          pq = fma(c.p2[o], c.q2[o], pq);
        }
        pq = wsum(pq);
        const bool brk = !(pq > 0.0);
        const double al = brk ? 0.0 : D->rz[w] / pq;
        double acc = 0.0;
        _Pragma("unroll 4") for (int i = lane; i < c.s; i += WAVE) {
          const int64_t o = (int64_t)w * c.lds + i;
          c.y2[o] = fma(al, c.p2[o], c.y2[o]);
          const double rv = c.r2[o];
          c.ro2[o] = rv;
          const double rn = fma(-al, c.q2[o], rv);
          c.r2[o] = rn;
          acc = fma(rn, rn, acc);
        }
        const double rn = sqrt(wsum(acc));
        if (lane == 0) {
          const int itj = D->it[w] + 1;
          D->it[w] = itj;
          D->rn[w] = rn;
          if (brk || !(rn == rn)) D->done[w] = 2;
          else if (rn <= c.P.inner_tol * D->bn[w]) D->done[w] = 1;
          else if (itj >= c.P.max_inner) D->done[w] = 3;
        }
      }
      ++it;
      __syncthreads();
      if (!any_active(D, c.k)) break;
      smv(c, c.S.Minv, c.r2, c.z2);
      if (w < c.k && D->done[w] == 0) {
        double zr = 0.0, zro = 0.0;
        _Pragma("unroll 4") for (int i = lane; i < c.s; i += WAVE) {
          const int64_t o = (int64_t)w * c.lds + i;
          const double z = c.z2[o];
          zr = fma(z, c.r2[o], zr);
          zro = fma(z, c.ro2[o], zro);
        }
        zr = wsum(zr);
        zro = wsum(zro);
        const double rzo = D->rz[w];
        if (rzo != 0.0 && isfinite(rzo)) {
          const double beta = (zr - zro) / rzo;
          _Pragma("unroll 4") for (int i = lane; i < c.s; i += WAVE) {
            const int64_t o = (int64_t)w * c.lds + i;
            c.p2[o] = fma(beta, c.p2[o], c.z2[o]);
          }
          if (lane == 0) D->rz[w] = zr;
        } else if (lane == 0) {
          D->done[w] = 2;  // beta's denominator vanished: breakdown, the iterate is kept
        }
      }
    }
    if (threadIdx.x == 0) {
      c.inner += it;
      if (c.P.profile) c.ticks[BT_LEVEL2] += wall_clock64() - l2t0;
    }
    __syncthreads();
    y_z(c);
  }

  // ---- level 1 (the level-1 iteration of Algorithm 1): (A_lo + lam I) x = rhs, x -> zh ---------------
  // skip (shared, may be null): columns not to solve. With confirm, convergence is
  // checked on rhs - (A_hi + lam I) x recomputed in FP64; restarts from it otherwise.
  static __device__ void level1(Ctx& c, const double* rhs, int64_t ldr, double tol, const int* skip, bool confirm) {
    const int w = wave_id(), lane = lane_id();
    Cols* C = c.C1;
    if (w < c.k) {
      const bool sk = skip && skip[w] != 0;
      double acc = 0.0;
      _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
        const int64_t o = (int64_t)w * c.ldn + i;
        const double v = sk ? 0.0 : rhs[(int64_t)w * ldr + i];
        c.r1[o] = v;
        c.zh[o] = 0.0;
        acc = fma(v, v, acc);
      }
      const double bn = sqrt(wsum(acc));
      if (lane == 0) {
        C->bn[w] = bn;
        C->rn[w] = bn;
        C->it[w] = 0;
        C->rel[w] = 0.0;
        C->done[w] = (sk || bn == 0.0) ? 4 : 0;
      }
    }
    __syncthreads();
    int it = 0, restarts = 0;
    bool fresh = true;  // the direction must be (re)started from z1
    while (true) {
      if (fresh) {
        solve_m1(c);
        if (w < c.k && C->done[w] == 0) {
          double acc = 0.0;
          _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
            const int64_t o = (int64_t)w * c.ldn + i;
            const double z = c.z1[o];
            c.p1[o] = z;
            acc = fma(c.r1[o], z, acc);
          }
          acc = wsum(acc);
          if (lane == 0) C->rz[w] = acc;
        }
        fresh = false;
      }
      __syncthreads();
      if (!any_active(C, c.k)) {
        if (!confirm) break;
        // confirmation on the FP64 residual of A_hi
        op_hi(c, 1, c.zh, rhs, ldr, c.q1);
        if (w < c.k && C->done[w] == 1) {
          double acc = 0.0;
          _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
            const double v = c.q1[(int64_t)w * c.ldn + i];
            acc = fma(v, v, acc);
          }
          const double bn = C->bn[w];
          const double rel = bn > 0.0 ? sqrt(wsum(acc)) / bn : 0.0;
          const bool ok = rel <= tol;
          if (!ok)
            _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) c.r1[(int64_t)w * c.ldn + i] = c.q1[(int64_t)w * c.ldn + i];
          if (lane == 0) {
            C->rel[w] = rel;
            C->done[w] = ok ? 4 : 0;
          }
        }
        __syncthreads();
        if (!any_active(C, c.k)) break;
        if (restarts >= MAX_RESTARTS || it >= c.P.max_outer) {
          if (w < c.k && lane == 0 && C->done[w] == 0) C->done[w] = 3;
          __syncthreads();
          break;
        }
        ++restarts;
        fresh = true;
        continue;
      }
      if (it >= c.P.max_outer) {
        if (w < c.k && lane == 0 && C->done[w] == 0) C->done[w] = 3;
        __syncthreads();
        break;
      }
      op_lo(c);
      if (w < c.k && C->done[w] == 0) {
        const double pq = C->pq[w];
        const bool brk = !(pq > 0.0);
        const double al = brk ? 0.0 : C->rz[w] / pq;
        double acc = 0.0;
        _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
          const int64_t o = (int64_t)w * c.ldn + i;
          c.zh[o] = fma(al, c.p1[o], c.zh[o]);
          const double rv = c.r1[o];
          c.ro1[o] = rv;
          const double rn = fma(-al, c.q1[o], rv);
          c.r1[o] = rn;
          acc = fma(rn, rn, acc);
        }
        const double rn = sqrt(wsum(acc));
        if (lane == 0) {
          const int itj = C->it[w] + 1;
          C->it[w] = itj;
          C->rn[w] = rn;
          if (brk || !(rn == rn)) C->done[w] = 2;
          else if (rn <= tol * C->bn[w]) C->done[w] = 1;
          else if (itj >= c.P.max_outer) C->done[w] = 3;
        }
      }
      ++it;
      __syncthreads();
      solve_m1(c);
      if (w < c.k && C->done[w] == 0) {
        double zr = 0.0, zro = 0.0;
        _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
          const int64_t o = (int64_t)w * c.ldn + i;
          const double z = c.z1[o];
          zr = fma(z, c.r1[o], zr);
          zro = fma(z, c.ro1[o], zro);
        }
        zr = wsum(zr);
        zro = wsum(zro);
        const double rzo = C->rz[w];
        if (rzo != 0.0 && isfinite(rzo)) {
          const double beta = (zr - zro) / rzo;
          _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
            const int64_t o = (int64_t)w * c.ldn + i;
            c.p1[o] = fma(beta, c.p1[o], c.z1[o]);
          }
          if (lane == 0) C->rz[w] = zr;
        } else if (lane == 0) {
          C->done[w] = 2;  // beta's denominator vanished: breakdown, the iterate is kept
        }
      }
    }
    if (threadIdx.x == 0) {
      c.outer += it;
      c.restarts += restarts;
    }
    __syncthreads();
  }

  // ---- FP64 Krylov refinement on A_hi with the low-precision MSP as preconditioner --
  static __device__ void refine(Ctx& c) {
    const int w = wave_id(), lane = lane_id();
    Cols* R = c.CH;
    const double* B = c.S.B;
    const int64_t ldb = c.S.ldb;
    if (w < c.k) {
      double acc = 0.0;
      _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
        const int64_t o = (int64_t)w * c.ldn + i;
        const double v = B[(int64_t)w * ldb + i];
        c.rh[o] = v;
        c.xh[o] = 0.0;
        acc = fma(v, v, acc);
      }
      const double bn = sqrt(wsum(acc));
      if (lane == 0) {
        R->bn[w] = bn;
        R->rn[w] = bn;
        R->it[w] = 0;
        R->rel[w] = 0.0;
        R->done[w] = bn == 0.0 ? 4 : 0;
      }
    }
    __syncthreads();
    int it = 0, restarts = 0;
    bool fresh = true;
    while (true) {
      if (fresh) {
        level1(c, c.rh, c.ldn, c.P.refine_tol, R->done, false);
        if (w < c.k && R->done[w] == 0) {
          double acc = 0.0;
          _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
            const int64_t o = (int64_t)w * c.ldn + i;
            const double z = c.zh[o];
            c.ph[o] = z;
            acc = fma(c.rh[o], z, acc);
          }
          acc = wsum(acc);
          if (lane == 0) R->rz[w] = acc;
        }
        fresh = false;
      }
      __syncthreads();
      if (!any_active(R, c.k)) {
        op_hi(c, 1, c.xh, B, ldb, c.qh);
        if (w < c.k && R->done[w] == 1) {
          double acc = 0.0;
          _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
            const double v = c.qh[(int64_t)w * c.ldn + i];
            acc = fma(v, v, acc);
          }
          const double bn = R->bn[w];
          const double rel = bn > 0.0 ? sqrt(wsum(acc)) / bn : 0.0;
          const bool ok = rel <= c.P.tol;
          if (!ok)
            _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) c.rh[(int64_t)w * c.ldn + i] = c.qh[(int64_t)w * c.ldn + i];
          if (lane == 0) {
            R->rel[w] = rel;
            R->done[w] = ok ? 4 : 0;
          }
        }
        __syncthreads();
        if (!any_active(R, c.k)) break;
        if (restarts >= MAX_RESTARTS || it >= c.P.max_refine) {
          // capped after a failed confirmation: rel holds the recomputed residual
          if (w < c.k && lane == 0 && R->done[w] == 0) R->done[w] = 3;
          __syncthreads();
          break;
        }
        ++restarts;
        fresh = true;
        continue;
      }
      if (it >= c.P.max_refine) {
        if (w < c.k && lane == 0 && R->done[w] == 0) {
          R->done[w] = 3;  // capped: report the recurrence residual it stopped at
          R->rel[w] = R->bn[w] > 0.0 ? R->rn[w] / R->bn[w] : 0.0;
        }
        __syncthreads();
        break;
      }
      op_hi(c, 0, c.ph, nullptr, 0, c.qh);
      if (w < c.k && R->done[w] == 0) {
        const double pq = R->pq[w];
        const bool brk = !(pq > 0.0);
        const double al = brk ? 0.0 : R->rz[w] / pq;
        double acc = 0.0;
        _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
          const int64_t o = (int64_t)w * c.ldn + i;
          c.xh[o] = fma(al, c.ph[o], c.xh[o]);
          const double rv = c.rh[o];
          c.roh[o] = rv;
          const double rn = fma(-al, c.qh[o], rv);
          c.rh[o] = rn;
          acc = fma(rn, rn, acc);
        }
        const double rn = sqrt(wsum(acc));
        if (lane == 0) {
          const int itj = R->it[w] + 1;
          R->it[w] = itj;
          R->rn[w] = rn;
          if (brk || !(rn == rn)) R->done[w] = 2;
          else if (rn <= c.P.tol * R->bn[w]) R->done[w] = 1;
          else if (itj >= c.P.max_refine) {
            R->done[w] = 3;
            R->rel[w] = R->bn[w] > 0.0 ? rn / R->bn[w] : 0.0;
          }
        }
      }
      ++it;
      __syncthreads();
      level1(c, c.rh, c.ldn, c.P.refine_tol, R->done, false);
      if (w < c.k && R->done[w] == 0) {
        double zr = 0.0, zro = 0.0;
        _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
          const int64_t o = (int64_t)w * c.ldn + i;
          const double z = c.zh[o];
          zr = fma(z, c.rh[o], zr);
          zro = fma(z, c.roh[o], zro);
        }
        zr = wsum(zr);
        zro = wsum(zro);
        const double rzo = R->rz[w];
        if (rzo != 0.0 && isfinite(rzo)) {
          const double beta = (zr - zro) / rzo;
          _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) {
            const int64_t o = (int64_t)w * c.ldn + i;
            c.ph[o] = fma(beta, c.ph[o], c.zh[o]);
          }
          if (lane == 0) R->rz[w] = zr;
        } else if (lane == 0) {
          R->done[w] = 2;  // beta's denominator vanished: breakdown, the iterate is kept
        }
      }
    }
    if (threadIdx.x == 0) {
      c.refine += it;
      c.restarts += restarts;
    }
    __syncthreads();
  }
};


// ---- helpers: a workgroup whose system is finished serves other systems' sweeps ----
struct JobSh {  // the claimed job, broadcast through LDS
  const void* bv;
  const double* x;
  const double* rhs;
  double* out;
  int64_t ldb, ldr;
  double lam;
  int mode, ncols, nslice, epoch, state;
};

// serve slices of system S as helper h until it finishes or stays idle too long
template <class TLO, class THI, class TY>
__device__ void serve(const BatchSys& S, int h, int k, double* part, JobSh* js) {
  BatchTeam* T = S.team;
  const int nch = (S.n + CHR - 1) / CHR;
  int last = 0;
  if (threadIdx.x == 0) last = ld_acq(&T->epoch);  // epochs published before joining are not ours
  while (true) {
    if (threadIdx.x == 0) {
      int state = 0;  // 0 leave, 1 work, 2 nothing for this helper in this epoch
      const uint64_t t0 = wall_clock64();
      while (true) {
        if (ld_rlx(&T->finish)) break;
        const int e = ld_rlx(&T->epoch);
        if (e != last) {
          fence_acq();
          js->bv = T->bv;
          js->x = T->x;
          js->rhs = T->rhs;
          js->out = T->out;
          js->ldb = T->ldb;
          js->ldr = T->ldr;
          js->lam = T->lam;
          js->mode = T->mode;
          js->ncols = T->ncols;
          js->nslice = T->nslice;
          if (ld_acq(&T->epoch) != e) continue;  // republished while reading: read again
          last = e;
          js->epoch = e;
          state = (h < js->nslice && cas_claim(&T->claim[h], e)) ? 1 : 2;
          break;
        }
        if (wall_clock64() - t0 > IDLE_TICKS) break;
        __builtin_amdgcn_s_sleep(2);
      }
      js->state = state;
    }
    __syncthreads();
    const int state = js->state;
    if (state == 0) {
      __syncthreads();
      return;
    }
    if (state == 1) {
      const int ns = js->nslice, mode = js->mode;
      const bool yjob = mode >= 3;
      const Job J{mode == 0 ? S.A_lo : (yjob ? S.Y : S.A_hi),
                  yjob ? S.ldy : S.lda,
                  js->bv, js->ldb, js->x, js->rhs, js->ldr, js->out, S.cpart, js->lam, S.n, js->ncols, S.ldn, k, mode,
                  mode == 0 ? S.aln_lo : (yjob ? S.aln_y : S.aln_hi)};
      do_chunks<TLO, THI, TY>(J, slice_begin(h, ns, nch), slice_begin(h + 1, ns, nch), part);
      if (threadIdx.x == 0) st_rel(&T->done[h], js->epoch);  // after the barrier that ended the slice
    }
    __syncthreads();
  }
}

// pick the unfinished system with the most work per helper and serve it; leave when no
// system needs help or when some system has not started (its workgroup is waiting for a
// compute unit: this one is better given back)
template <class TLO, class THI, class TY>
__device__ void help(const BatchSys* __restrict__ sys, const BatchPrm& prm, int k, double* part, int* shi,
                     JobSh* js) {
  for (int round = 0; round < 4 * MAXH; ++round) {
    if (threadIdx.x == 0) {
      int target = -1, h = 0;
      double best = 0.0;
      for (int j = 0; j < prm.nsys; ++j) {
        BatchTeam* T = sys[j].team;
        if (!__hip_atomic_load(&T->started, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          target = -1;
          best = -1.0;
          break;
        }
        if (__hip_atomic_load(&T->finish, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) continue;
        const int nch = (sys[j].n + CHR - 1) / CHR;
        const int jn = __hip_atomic_load(&T->joined, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (jn >= MAXH || jn >= nch - 1) continue;
        const double score = (double)sys[j].n * (double)sys[j].n / (double)(jn + 2);
        if (score > best) {
          best = score;
          target = j;
        }
      }
      if (target >= 0) {
        h = __hip_atomic_fetch_add(&sys[target].team->joined, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (h > MAXH) target = -2;
      }
      shi[2] = target;
      shi[3] = h;
    }
    __syncthreads();
    const int target = shi[2], h = shi[3];
    __syncthreads();
    if (target == -1) return;
    if (target == -2) continue;
    serve<TLO, THI, TY>(sys[target], h, k, part, js);
  }
}

template <class TLO, class THI, class TY>
__global__ void __launch_bounds__(NTB) k_batch_psd(const BatchSys* __restrict__ sys, BatchPrm prm, int k,
                                                   BatchOut* __restrict__ out) {
  __shared__ Cols cH, c1, c2;
  __shared__ double red[NW * 256];
  __shared__ double part[NW * KB];
  __shared__ int shi[8];
  __shared__ JobSh js;
  Ctx c;
  c.S = sys[blockIdx.x];
  c.shi = shi;
  c.epoch = 0;
  c.team_err = 0;
  c.helped = 0;
  c.selfdone = 0;
  if (threadIdx.x == 0 && prm.teams)
    __hip_atomic_store(&c.S.team->started, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  c.P = prm;
  c.k = k;
  c.n = c.S.n;
  c.s = c.S.s;
  c.ldn = c.S.ldn;
  c.lds = c.S.lds;
  const int64_t vn = (int64_t)prm.kcap * c.ldn, vs = (int64_t)prm.kcap * c.lds;
  double* v = c.S.vec;
  c.xh = v;
  c.rh = v + vn;
  c.roh = v + 2 * vn;
  c.ph = v + 3 * vn;
  c.qh = v + 4 * vn;
  c.zh = v + 5 * vn;
  c.r1 = v + 6 * vn;
  c.ro1 = v + 7 * vn;
  c.z1 = v + 8 * vn;
  c.p1 = v + 9 * vn;
  c.q1 = v + 10 * vn;
  double* u = v + 11 * vn;
  c.r2 = u;
  c.ro2 = u + vs;
  c.z2 = u + 2 * vs;
  c.p2 = u + 3 * vs;
  c.q2 = u + 4 * vs;
  c.y2 = u + 5 * vs;
  c.b2 = u + 6 * vs;
  c.pf = c.S.pf;
  c.CH = &cH;
  c.C1 = &c1;
  c.C2 = &c2;
  c.red = red;
  c.part = part;
  c.outer = c.inner = c.refine = c.restarts = 0;
  for (int q = 0; q < BT_NPHASE; ++q) c.ticks[q] = 0;
  const uint64_t tstart = (prm.profile && threadIdx.x == 0) ? wall_clock64() : 0;
  using BT = Batch<TLO, THI, TY>;
  const bool do_refine = prm.refine != 0;
  // Under refinement the inner MSP sweeps A_lo + (lam + delta) I with
  // delta = u_lo ||A_hi||_inf >= ||A_lo - A_hi||_2 (elementwise rounding of a symmetric
  // matrix), so the inner operator dominates A_hi + lam I and stays positive definite.
  c.lam_lo = c.S.lam;
  if (do_refine) {
    const double u_lo = sizeof(TLO) == 2 ? 0x1p-8 : (sizeof(TLO) == 4 ? 0x1p-24 : 0.0);
    c.lam_lo = c.S.lam + u_lo * BT::norm_inf_hi(c);
  }
  if (do_refine) BT::refine(c);
  else BT::level1(c, c.S.B, c.S.ldb, prm.tol, nullptr, true);
  // solution out, per-system record
  const Cols* F = do_refine ? c.CH : c.C1;
  const double* xs = do_refine ? c.xh : c.zh;
  const int w = wave_id(), lane = lane_id();
  if (w < k)
    _Pragma("unroll 4") for (int i = lane; i < c.n; i += WAVE) c.S.X[(int64_t)w * c.S.ldx + i] = xs[(int64_t)w * c.ldn + i];
  if (threadIdx.x == 0) {
    BatchOut o;
    int worst = 0;  // 0 ok, 1 cap, 2 breakdown, 3 non-finite
    double rel = 0.0;
    for (int j = 0; j < k; ++j) {
      const int d = F->done[j];
      const double r = F->rel[j];
      if (!(r == r) || r > 1e300) worst = max(worst, 3);
      else rel = fmax(rel, r);
      if (d == 2) worst = max(worst, 2);
      else if (d != 4) worst = max(worst, 1);
    }
    if (c.team_err) worst = max(worst, 4);
    o.code = worst;
    o.outer = c.outer;
    o.inner = c.inner;
    o.refine = c.refine;
    o.restarts = c.restarts;
    o.helped = c.helped;
    o.selfdone = c.selfdone;
    o.relres = rel;
    if (prm.profile) c.ticks[BT_TOTAL] = wall_clock64() - tstart;
    for (int q = 0; q < BT_NPHASE; ++q) o.ticks[q] = c.ticks[q];
    out[c.S.id] = o;
  }
  if (!prm.teams) return;
  __syncthreads();
  if (threadIdx.x == 0) st_rel(&c.S.team->finish, 1);
  help<TLO, THI, TY>(sys, prm, k, part, shi, &js);
}

template <class TLO, class THI, class TY>
hipError_t launch_t(hipStream_t st, const BatchSys* sys, int nsys, const BatchPrm& prm, int k, BatchOut* out) {
  hipLaunchKernelGGL((k_batch_psd<TLO, THI, TY>), dim3((unsigned)nsys), dim3(NTB), 0, st, sys, prm, k, out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_batch_psd(hipStream_t st, msp_dtype lo_t, msp_dtype hi_t, msp_dtype y_t, const BatchSys* sys,
                            int nsys, const BatchPrm& prm, int k, BatchOut* out) {
  if (y_t == MSP_F64) {
    if (lo_t == MSP_F64 && hi_t == MSP_F64) return launch_t<double, double, double>(st, sys, nsys, prm, k, out);
    return hipErrorInvalidValue;
  }
  if (y_t == MSP_F32) {
    if (lo_t == MSP_F32 && hi_t == MSP_F32) return launch_t<float, float, float>(st, sys, nsys, prm, k, out);
    if (lo_t == MSP_F32 && hi_t == MSP_F64) return launch_t<float, double, float>(st, sys, nsys, prm, k, out);
    if (lo_t == MSP_BF16 && hi_t == MSP_F32) return launch_t<__hip_bfloat16, float, float>(st, sys, nsys, prm, k, out);
    if (lo_t == MSP_BF16 && hi_t == MSP_F64)
      return launch_t<__hip_bfloat16, double, float>(st, sys, nsys, prm, k, out);
  }
  return hipErrorInvalidValue;
}

bool batch_types_supported(msp_dtype lo_t, msp_dtype hi_t, msp_dtype y_t) {
  if (y_t == MSP_F64) return lo_t == MSP_F64 && hi_t == MSP_F64;
  if (y_t == MSP_F32) return (lo_t == MSP_F32 || lo_t == MSP_BF16) && (hi_t == MSP_F32 || hi_t == MSP_F64);
  return false;
}
