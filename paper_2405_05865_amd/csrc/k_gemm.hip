// Block A-sweep for many right-hand sides on the matrix cores:
//   Y[:, j] = A X[:, j] (+ lam X[:, j]) for j < k (k >= 8),
// the level-1 operator of Algorithms 1 and 3 applied to a block of k vectors at once
// (the block execution of the method for many right-hand sides or trace probes).
//
// Work unit: one wavefront computes a 16*RT-row x 16*KT-column output tile with
// 16x16x4 MFMA (F32 arithmetic for F32/BF16 storage, F64 for F64 storage and for the
// FP64-on-F32 residual form). Lane l supplies row (l % 16) of each 16-row tile and the
// reduction slice [c0 + E (l / 16), +E) of each step, for both operands (E = two 16-byte
// chunks), so the four lanes of a row read 128 contiguous bytes (a whole cache line) per
// step and one lane's loads feed E MFMAs. Neighbouring wavefronts take the column groups
// of the same rows, so A is read from HBM about once per 4*16*KT columns and reused
// from cache by the others. Per-column dot partials <X_j, Y_j> per row set feed the
// level-1 step length (the same layout as the single-vector sweep). When the row sets
// and column groups give too few wavefronts to keep HBM busy (a few right-hand sides),
// the reduction range is split into segments: each wavefront writes its partial tile and
// a second kernel adds the segments of every output in a fixed order, applies the shift
// and writes the dot partials.
#include "msp_internal.h"

#include <hip/hip_bf16.h>

#include <algorithm>

namespace {

constexpr int WAVE = 64;

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

// element e of lane l holds tile row out_row(l / 16, e), column l % 16
template <class TC>
__device__ __forceinline__ int out_row(int g, int e) {
  return sizeof(TC) == 4 ? 4 * g + e : 4 * e + g;
}

__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

template <class TA, class TC>
struct Ld;
template <>
struct Ld<double, double> {
  static constexpr int VEC = 2;
  __device__ static void vec(const double* p, double* o) {
    const nd2 v = __builtin_nontemporal_load(reinterpret_cast<const nd2*>(p));
    o[0] = v.x;
    o[1] = v.y;
  }
  __device__ static double one(const double* p) { return *p; }
};
template <>
struct Ld<float, float> {
  static constexpr int VEC = 4;
  __device__ static void vec(const float* p, float* o) {
    const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(p));
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
  __device__ static void vec(const float* p, double* o) {
    const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(p));
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
  __device__ static void vec(const __hip_bfloat16* p, float* o) {
    const nu4 v = __builtin_nontemporal_load(reinterpret_cast<const nu4*>(p));
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

// VEC consecutive FP64 vector entries (16-byte aligned when the vector's rows are),
// converted to the arithmetic type
template <class TC, int VEC, bool ALN>
__device__ __forceinline__ void ld_x(const double* p, TC* o) {
  if constexpr (ALN) {
#pragma unroll
    for (int q = 0; q < VEC / 2; ++q) {
      const nd2 v = *reinterpret_cast<const nd2*>(p + 2 * q);
      o[2 * q] = (TC)v.x;
      o[2 * q + 1] = (TC)v.y;
    }
  } else {
#pragma unroll
    for (int q = 0; q < VEC; ++q) o[q] = (TC)p[q];
  }
}

template <class TA, class TC, int RT, int KT, bool ALN>
__global__ void __launch_bounds__(256) k_gemm(const TA* __restrict__ A, int64_t lda, int rows, int cols,
                                             const double* __restrict__ X, int64_t ldx, double* __restrict__ Y,
                                             int64_t ldy, int k, double lam, int diag,
                                             const int32_t* __restrict__ skip, double* __restrict__ dot_part,
                                             int nrs, int ncs, int nseg, int seg_cols, double* __restrict__ part) {
  using L = Ld<TA, TC>;
  constexpr int VEC = L::VEC;
  constexpr int NCH = 2;          // 16-byte chunks per lane and step
  constexpr int E = NCH * VEC;    // reduction elements per lane and step
  constexpr int STEP = 4 * E;
  const int wg = blockIdx.x * 4 + threadIdx.x / WAVE;  // global wavefront index
  if (wg >= nrs * ncs * nseg) return;                    // whole wavefronts only
  // neighbouring wavefronts: column groups of the same rows and segment (A from cache)
  const int cs = wg % ncs, sg = (wg / ncs) % nseg, rs = wg / (ncs * nseg);
  const int cbeg = sg * seg_cols, cend = min(cols, cbeg + seg_cols);
  const int lane = threadIdx.x & (WAVE - 1), i = lane & 15, g = lane >> 4;
  const int r0 = rs * 16 * RT;
  const int gbase = cs * KT;  // first 16-column group of this wavefront
  // X is read in aligned pairs only when the vectors' rows are 16-byte aligned
  const TA* ap[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) ap[t] = A + (int64_t)min(r0 + 16 * t + i, rows - 1) * lda + E * g;
  const double* bp[KT];
#pragma unroll
  for (int q = 0; q < KT; ++q) {
    const int j = min(16 * (gbase + q) + i, k - 1);
    bp[q] = X + (int64_t)j * ldx + E * g;
  }
  typename V4<TC>::t acc[RT][KT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int q = 0; q < KT; ++q) acc[t][q] = typename V4<TC>::t{0, 0, 0, 0};
  int c0 = cbeg;
  if constexpr (ALN) {
#pragma unroll 2
    for (; c0 + STEP <= cend; c0 += STEP) {
      TC a[RT][E], b[KT][E];
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int h = 0; h < NCH; ++h) L::vec(ap[t] + c0 + h * VEC, a[t] + h * VEC);
#pragma unroll
      for (int q = 0; q < KT; ++q) ld_x<TC, E, true>(bp[q] + c0, b[q]);
#pragma unroll
      for (int m = 0; m < E; ++m)
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int q = 0; q < KT; ++q) acc[t][q] = mfma(a[t][m], b[q][m], acc[t][q]);
    }
  }
  for (; c0 < cend; c0 += STEP) {
    TC a[RT][E], b[KT][E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const bool ok = c0 + E * g + m < cend;
#pragma unroll
      for (int t = 0; t < RT; ++t) a[t][m] = ok ? L::one(ap[t] + c0 + m) : (TC)0;
#pragma unroll
      for (int q = 0; q < KT; ++q) b[q][m] = ok ? (TC)bp[q][c0 + m] : (TC)0;
    }
#pragma unroll
    for (int m = 0; m < E; ++m)
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int q = 0; q < KT; ++q) acc[t][q] = mfma(a[t][m], b[q][m], acc[t][q]);
  }
  if (nseg > 1) {  // partial tile of this segment: part[sg][j][row]
#pragma unroll
    for (int q = 0; q < KT; ++q) {
      const int j = 16 * (gbase + q) + i;
      if (j >= k || (skip && skip[j])) continue;
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = r0 + 16 * t + out_row<TC>(g, e);
          if (row < rows) part[((int64_t)sg * k + j) * rows + row] = (double)acc[t][q][e];
        }
    }
    return;
  }
  // epilogue: Y = acc (+ lam X), per-column dot partials over this row set
#pragma unroll
  for (int q = 0; q < KT; ++q) {
    const int j = 16 * (gbase + q) + i;
    const bool live = j < k && !(skip && skip[j]);
    double dp = 0.0;
    if (live) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = r0 + 16 * t + out_row<TC>(g, e);
          if (row < rows) {
            const double xr = (diag || dot_part) ? X[(int64_t)j * ldx + row] : 0.0;
            const double y = (double)acc[t][q][e] + (diag ? lam * xr : 0.0);
            Y[(int64_t)j * ldy + row] = y;
            dp = fma(xr, y, dp);
          }
        }
    }
    if (dot_part) {
      // the four lanes of column j (l / 16 = 0..3) hold disjoint rows
      dp += __shfl_xor(dp, 16, WAVE);
      dp += __shfl_xor(dp, 32, WAVE);
      if (g == 0 && j < k) dot_part[(int64_t)rs * k + j] = dp;
    }
  }
}

// Y[:, j] = sum over the segments (fixed order) (+ lam X[:, j]); dot partials per 64 rows
__global__ void __launch_bounds__(WAVE) k_gemm_sum(const double* __restrict__ part, int nseg, int rows, int k,
                                                  const double* __restrict__ X, int64_t ldx, double* __restrict__ Y,
                                                  int64_t ldy, double lam, int diag, const int32_t* __restrict__ skip,
                                                  double* __restrict__ dot_part) {
  const int row = blockIdx.x * WAVE + threadIdx.x, j = blockIdx.y;
  double dp = 0.0;
  if (!(skip && skip[j]) && row < rows) {
    double acc = 0.0;
    for (int s = 0; s < nseg; ++s) acc += part[((int64_t)s * k + j) * rows + row];
    const double xr = (diag || dot_part) ? X[(int64_t)j * ldx + row] : 0.0;
    const double y = acc + (diag ? lam * xr : 0.0);
    Y[(int64_t)j * ldy + row] = y;
    dp = xr * y;
  }
  if (dot_part) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dp += __shfl_xor(dp, off, WAVE);
    if (threadIdx.x == 0) dot_part[(int64_t)blockIdx.x * k + j] = dp;
  }
}

// segments of the reduction range: double until the launch has about 8 wavefronts per CU
// (measured at n = 32768, 16 RHS: 2048 wavefronts stream faster than 8192 once every step
// reads whole cache lines), each segment keeps >= min_seg columns and the partials fit the
// scratch. Products of cache-resident matrices (the s x s operators of the inner levels,
// min_seg = kSegSmall) stop at about 4 wavefronts per CU: at s = 1024 and 512 columns fewer,
// longer segments write and re-read fewer partials (a Schatten-1 block run 6% faster than
// with 2048 wavefronts; 512 and 256 were slower)
int gemm_segments(int64_t rows, int64_t cols, int k, int64_t waves, size_t scratch_doubles, int min_seg) {
  const int64_t target = min_seg <= kSegSmall ? 1024 : 2048;
  int nseg = 1;
  while (waves * nseg < target && nseg < 64 && cols / (2 * nseg) >= min_seg &&
         (size_t)(2 * nseg) * (size_t)k * (size_t)rows <= scratch_doubles)
    nseg *= 2;
  return nseg;
}

template <class TA, class TC, int RT, int KT>
hipError_t gemm_t(hipStream_t st, const TA* A, int64_t rows, int64_t cols, int64_t lda, const double* X,
                  int64_t ldx, double* Y, int64_t ldy, int k, double lam, bool diag, const int32_t* skip,
                  double* dot_part, int* nblocks, double* scratch, size_t scratch_doubles, int min_seg,
                  int force_nseg, int* nseg_out, bool defer_sum) {
  static_assert(16 * RT == WAVE, "the segment sum takes 64-row sets");
  const int nrs = (int)((rows + 16 * RT - 1) / (16 * RT));
  const int ngroups = (k + 15) / 16;
  const int ncs = (ngroups + KT - 1) / KT;
  // a forced count (the autotuner's) must fit the scratch; otherwise the built-in rule
  const bool forced = force_nseg == 1 || (force_nseg > 1 && scratch &&
                                          (size_t)force_nseg * (size_t)k * (size_t)rows <= scratch_doubles);
  const int nseg = forced ? force_nseg
                          : (scratch ? gemm_segments(rows, cols, k, (int64_t)nrs * ncs, scratch_doubles, min_seg) : 1);
  constexpr int STEP = 4 * 2 * Ld<TA, TC>::VEC;  // four lane groups x two 16-byte chunks
  const int seg_cols = (int)(((cols + nseg - 1) / nseg + STEP - 1) / STEP * STEP);
  const int64_t waves = (int64_t)nrs * ncs * nseg;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  const bool aln = ((uintptr_t)A % 16 == 0) && ((lda * (int64_t)sizeof(TA)) % 16 == 0) && ((uintptr_t)X % 16 == 0) &&
                   (ldx % 2 == 0);
  if (aln)
    hipLaunchKernelGGL((k_gemm<TA, TC, RT, KT, true>), dim3(blocks), dim3(256), 0, st, A, lda, (int)rows, (int)cols,
                       X, ldx, Y, ldy, k, lam, diag ? 1 : 0, skip, dot_part, nrs, ncs, nseg, seg_cols, scratch);
  else
    hipLaunchKernelGGL((k_gemm<TA, TC, RT, KT, false>), dim3(blocks), dim3(256), 0, st, A, lda, (int)rows, (int)cols,
                       X, ldx, Y, ldy, k, lam, diag ? 1 : 0, skip, dot_part, nrs, ncs, nseg, seg_cols, scratch);
  if (nseg > 1 && !defer_sum)
    hipLaunchKernelGGL(k_gemm_sum, dim3((unsigned)nrs, (unsigned)k), dim3(WAVE), 0, st, scratch, nseg, (int)rows, k, X,
                       ldx, Y, ldy, lam, diag ? 1 : 0, skip, dot_part);
  if (nblocks) *nblocks = nrs;
  if (nseg_out) *nseg_out = nseg;
  return hipGetLastError();
}

// column groups per wavefront: enough to cover k in one or two passes over A while
// keeping the accumulators in registers
template <class TA, class TC>
hipError_t gemm_k(hipStream_t st, const TA* A, int64_t rows, int64_t cols, int64_t lda, const double* X, int64_t ldx,
                  double* Y, int64_t ldy, int k, double lam, bool diag, const int32_t* skip, double* dot_part,
                  int* nblocks, double* scratch, size_t scratch_doubles, int min_seg = 1024, int force_nseg = 0,
                  int* nseg_out = nullptr, bool defer_sum = false) {
  if (k <= 16)
    return gemm_t<TA, TC, 4, 1>(st, A, rows, cols, lda, X, ldx, Y, ldy, k, lam, diag, skip, dot_part, nblocks, scratch,
                                scratch_doubles, min_seg, force_nseg, nseg_out, defer_sum);
  if (sizeof(TC) == 8 || k <= 32)
    return gemm_t<TA, TC, 4, 2>(st, A, rows, cols, lda, X, ldx, Y, ldy, k, lam, diag, skip, dot_part, nblocks, scratch,
                                scratch_doubles, min_seg, force_nseg, nseg_out, defer_sum);
  return gemm_t<TA, TC, 4, 4>(st, A, rows, cols, lda, X, ldx, Y, ldy, k, lam, diag, skip, dot_part, nblocks, scratch,
                              scratch_doubles, min_seg, force_nseg, nseg_out, defer_sum);
}

// column groups per wavefront as gemm_k picks them (KT)
int gemm_kt(int k, bool tc64) { return k <= 16 ? 1 : ((tc64 || k <= 32) ? 2 : 4); }

// Transposed block product Y[:, j] = A^T X[:, j] (A rows x cols row-major; the
// normal-equation operator of Algorithm 3). Lane l loads VEC consecutive columns
// [c0 + VEC (l % 16), +VEC) of row r + l / 16 in one 16-byte access; MFMA m takes
// element m, so output tile m holds the A-columns c0 + m + VEC * (0..15). A step covers
// 4 rows x 16 VEC columns. Waves with neighbouring indices share the same A columns and
// rows and differ in the right-hand-side group, so A is reused from cache. Row ranges
// are split when there are too few column tiles to fill the chip; the splits are summed
// in fixed order afterwards.
template <class TA, class TC, int KT, bool ALN>
__global__ void __launch_bounds__(256) k_gemm_t(const TA* __restrict__ A, int64_t lda, int rows, int cols,
                                               const double* __restrict__ X, int64_t ldx, int k, int nct, int ncs,
                                               int nsplit, int rows_per_split, double* __restrict__ out, int64_t ldo,
                                               const int32_t* __restrict__ skip, int direct) {
  using L = Ld<TA, TC>;
  constexpr int VEC = L::VEC;
  const int wg = blockIdx.x * 4 + threadIdx.x / WAVE;
  if (wg >= nct * ncs * nsplit) return;
  const int cs = wg % ncs, ct = (wg / ncs) % nct, sp = wg / (ncs * nct);
  const int lane = threadIdx.x & (WAVE - 1), i = lane & 15, g = lane >> 4;
  const int c0 = ct * 16 * VEC;
  const int cl = c0 + VEC * i;  // this lane's first A-column
  const int rb = sp * rows_per_split, re = min(rows, rb + rows_per_split);
  const bool full = ALN && (cl + VEC <= cols);
  const double* xp[KT];
#pragma unroll
  for (int q = 0; q < KT; ++q) xp[q] = X + (int64_t)min(16 * (cs * KT + q) + i, k - 1) * ldx;
  typename V4<TC>::t acc[VEC][KT];
#pragma unroll
  for (int m = 0; m < VEC; ++m)
#pragma unroll
    for (int q = 0; q < KT; ++q) acc[m][q] = typename V4<TC>::t{0, 0, 0, 0};
  for (int r = rb; r < re; r += 4) {
    const int row = r + g;
    const bool ok = row < re;
    TC a[VEC], b[KT];
    if (ok && full) {
      L::vec(A + (int64_t)row * lda + cl, a);
    } else {
#pragma unroll
      for (int m = 0; m < VEC; ++m) a[m] = (ok && cl + m < cols) ? L::one(A + (int64_t)row * lda + cl + m) : (TC)0;
    }
#pragma unroll
    for (int q = 0; q < KT; ++q) b[q] = ok ? (TC)xp[q][row] : (TC)0;
#pragma unroll
    for (int m = 0; m < VEC; ++m)
#pragma unroll
      for (int q = 0; q < KT; ++q) acc[m][q] = mfma(a[m], b[q], acc[m][q]);
  }
#pragma unroll
  for (int q = 0; q < KT; ++q) {
    const int j = 16 * (cs * KT + q) + i;
    if (j >= k) continue;
    if (direct && skip && skip[j]) continue;
#pragma unroll
    for (int m = 0; m < VEC; ++m)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int col = c0 + m + VEC * out_row<TC>(g, e);
        if (col >= cols) continue;
        if (direct) out[(int64_t)j * ldo + col] = (double)acc[m][q][e];
        else out[((int64_t)sp * k + j) * cols + col] = (double)acc[m][q][e];
      }
  }
}

__global__ void k_sum_splits_t(const double* __restrict__ part, int nsplit, int64_t cols, int k,
                               const int32_t* __restrict__ skip, double* __restrict__ Y, int64_t ldy) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t len = cols * k;
  if (idx >= len) return;
  const int j = (int)(idx / cols);
  const int64_t c = idx % cols;
  if (skip && skip[j]) return;
  double acc = 0.0;
  for (int t = 0; t < nsplit; ++t) acc += part[(int64_t)t * len + idx];
  Y[(int64_t)j * ldy + c] = acc;
}

// row splits of the transposed product: enough wavefronts to fill the chip
void gemmT_split(int64_t rows, int64_t cols, int k, int vec, int kt, int* nsplit_out, int* rps_out) {
  const int64_t nct = (cols + 16 * vec - 1) / (16 * vec);
  const int64_t ncs = ((k + 15) / 16 + kt - 1) / kt;
  int64_t nsplit = (2048 + nct * ncs - 1) / (nct * ncs);
  nsplit = std::max<int64_t>(1, std::min<int64_t>(nsplit, std::min<int64_t>(64, (rows + 255) / 256)));
  const int64_t rps = ((rows + nsplit - 1) / nsplit + 3) / 4 * 4;
  *nsplit_out = (int)((rows + rps - 1) / rps);
  *rps_out = (int)rps;
}

template <class TA, class TC, int KT>
hipError_t gemmT_t(hipStream_t st, const TA* A, int64_t rows, int64_t cols, int64_t lda, const double* X,
                   int64_t ldx, double* Y, int64_t ldy, int k, const int32_t* skip, double* part) {
  constexpr int VEC = Ld<TA, TC>::VEC;
  const int nct = (int)((cols + 16 * VEC - 1) / (16 * VEC));
  const int ncs = ((k + 15) / 16 + KT - 1) / KT;
  int nsplit = 1, rps = 4;
  gemmT_split(rows, cols, k, VEC, KT, &nsplit, &rps);
  const int64_t waves = (int64_t)nct * ncs * nsplit;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  const bool aln = ((uintptr_t)A % 16 == 0) && ((lda * (int64_t)sizeof(TA)) % 16 == 0);
  const int direct = nsplit == 1;
  double* out = direct ? Y : part;
  const int64_t ldo = direct ? ldy : 0;
  if (aln)
    hipLaunchKernelGGL((k_gemm_t<TA, TC, KT, true>), dim3(blocks), dim3(256), 0, st, A, lda, (int)rows, (int)cols, X,
                       ldx, k, nct, ncs, nsplit, rps, out, ldo, skip, direct);
  else
    hipLaunchKernelGGL((k_gemm_t<TA, TC, KT, false>), dim3(blocks), dim3(256), 0, st, A, lda, (int)rows, (int)cols, X,
                       ldx, k, nct, ncs, nsplit, rps, out, ldo, skip, direct);
  if (!direct) {
    const int64_t len = cols * k;
    hipLaunchKernelGGL(k_sum_splits_t, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, part, nsplit, cols, k,
                       skip, Y, ldy);
  }
  return hipGetLastError();
}

}  // namespace

int gemm_row_sets(int64_t rows) { return (int)((rows + 63) / 64); }

size_t gemm_t_part_doubles(int64_t rows, int64_t cols, int64_t k) {
  size_t worst = 0;
  for (int vec : {2, 4, 8}) {
    int ns = 1, rps = 4;
    gemmT_split(rows, cols, (int)k, vec, 2, &ns, &rps);
    if (ns > 1) worst = std::max(worst, (size_t)ns * k * cols);
  }
  return worst + 64;
}

hipError_t launch_gemm_t(hipStream_t st, const void* A, msp_dtype a_t, int64_t rows, int64_t cols, int64_t lda,
                         const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k, const int32_t* skip,
                         double* part) {
  const int kk = (int)k;
  switch (a_t) {
    case MSP_F64:
      return gemmT_t<double, double, 2>(st, (const double*)A, rows, cols, lda, X, ldx, Y, ldy, kk, skip, part);
    case MSP_F32:
      return gemmT_t<float, float, 2>(st, (const float*)A, rows, cols, lda, X, ldx, Y, ldy, kk, skip, part);
    case MSP_BF16:
      return gemmT_t<__hip_bfloat16, float, 2>(st, (const __hip_bfloat16*)A, rows, cols, lda, X, ldx, Y, ldy, kk,
                                                skip, part);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_t_f32_as_f64(hipStream_t st, const float* A, int64_t rows, int64_t cols, int64_t lda,
                                    const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k,
                                    const int32_t* skip, double* part) {
  return gemmT_t<float, double, 2>(st, A, rows, cols, lda, X, ldx, Y, ldy, (int)k, skip, part);
}

hipError_t launch_gemm_split(hipStream_t st, const void* A, msp_dtype a_t, bool fp64_arith, int64_t rows,
                             int64_t cols, int64_t lda, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k,
                             double lam, bool diag, const int32_t* skip, double* dot_part, int* nblocks,
                             double* scratch, size_t scratch_doubles, int nseg) {
  const int kk = (int)k;
  switch (a_t) {
    case MSP_F64:
      return gemm_k<double, double>(st, (const double*)A, rows, cols, lda, X, ldx, Y, ldy, kk, lam, diag, skip,
                                    dot_part, nblocks, scratch, scratch_doubles, 1024, nseg);
    case MSP_F32:
      if (fp64_arith)
        return gemm_k<float, double>(st, (const float*)A, rows, cols, lda, X, ldx, Y, ldy, kk, lam, diag, skip,
                                     dot_part, nblocks, scratch, scratch_doubles, 1024, nseg);
      return gemm_k<float, float>(st, (const float*)A, rows, cols, lda, X, ldx, Y, ldy, kk, lam, diag, skip, dot_part,
                                  nblocks, scratch, scratch_doubles, 1024, nseg);
    case MSP_BF16:
      return gemm_k<__hip_bfloat16, float>(st, (const __hip_bfloat16*)A, rows, cols, lda, X, ldx, Y, ldy, kk, lam,
                                           diag, skip, dot_part, nblocks, scratch, scratch_doubles, 1024, nseg);
  }
  return hipErrorInvalidValue;
}

int gemm_split_default(int64_t rows, int64_t cols, int64_t k, msp_dtype a_t, bool fp64_arith,
                       size_t scratch_doubles) {
  const bool tc64 = a_t == MSP_F64 || (a_t == MSP_F32 && fp64_arith);
  const int kt = gemm_kt((int)k, tc64);
  const int64_t nrs = (rows + 63) / 64;
  const int64_t ncs = (((k + 15) / 16) + kt - 1) / kt;
  return gemm_segments(rows, cols, (int)k, nrs * ncs, scratch_doubles, 1024);
}

hipError_t launch_gemm(hipStream_t st, const void* A, msp_dtype a_t, bool fp64_arith, int64_t rows, int64_t cols,
                       int64_t lda, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k, double lam,
                       bool diag, const int32_t* skip, double* dot_part, int* nblocks) {
  return launch_gemm_split(st, A, a_t, fp64_arith, rows, cols, lda, X, ldx, Y, ldy, k, lam, diag, skip, dot_part,
                           nblocks, nullptr, 0, 0);
}

size_t gemm_split_doubles(int64_t rows, int64_t k) { return (size_t)16 * rows * k + 64; }

hipError_t launch_gemm_seg(hipStream_t st, const double* M, int64_t rows, int64_t cols, const double* X,
                           int64_t ldx, double* Y, int64_t ldy, int64_t k, const int32_t* skip, double* scratch,
                           size_t scratch_doubles, int min_seg, int* nseg_out, bool defer_sum) {
  return gemm_k<double, double>(st, M, rows, cols, cols, X, ldx, Y, ldy, (int)k, 0.0, false, skip, nullptr, nullptr,
                                scratch, scratch_doubles, min_seg, 0, nseg_out, defer_sum);
}
