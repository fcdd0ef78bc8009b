// Symmetric A-sweep from the lower triangle: q = (A + lam I) p reads A[i][j] for j <= i
// only, so a sweep streams n(n+1)/2 elements instead of n^2 (the level-1 operator of
// Algorithm 1 is symmetric by the problem statement). Each element of the strict lower
// triangle is used twice from one load: in the row dot (A p)_i and, mirrored, in the
// column sum (A^T p)_j.
//
// The lower triangle is cut into 256 x 256 tiles (I, J), J <= I, one per block, numbered
// b = I (I + 1) / 2 + J. A block has four wavefronts; wavefront w takes the tile rows
// w + 4 (g + 4 t) (lane group g = lane / 16) and all 256 columns: 16 lanes share a row
// (16-byte chunks, 256 contiguous bytes per row and load), so the row dots reduce over 16
// lanes and the column sums over the 4 lane groups and then the 4 wavefronts (LDS). A
// tile writes its row partials (ypart) and column partials (zpart); a second kernel adds,
// for each row, the row partials of its tile row and the column partials of its tile
// column in a fixed order, applies the shift and writes the <p, q> partials of the
// level-1 update. Diagonal tiles mask the strict upper triangle (not loaded) and the
// diagonal from the column sums.
#include "msp_internal.h"

#include <hip/hip_bf16.h>

namespace {

constexpr int WAVE = 64;
constexpr int T = 256;          // tile edge
constexpr int NWV = 4;          // wavefronts per block (rows interleaved)
constexpr int LC = 16;          // lanes along a row
constexpr int LR = WAVE / LC;   // lane groups along a column
constexpr int NB = NWV * WAVE;  // threads per block
constexpr int NR = 64;          // rows per block of the reduction
constexpr int NG = 16;          // partial sums per row of the reduction (one wavefront each)

typedef double sd2 __attribute__((ext_vector_type(2)));
typedef float sf4 __attribute__((ext_vector_type(4)));
typedef uint32_t su4 __attribute__((ext_vector_type(4)));

template <class TA, class TC>
struct Chunk;  // one 16-byte chunk of a row as VEC values of the arithmetic type
template <>
struct Chunk<double, double> {
  static constexpr int VEC = 2;
  static __device__ __forceinline__ void load(const double* p, double* o) {
    const sd2 v = __builtin_nontemporal_load(reinterpret_cast<const sd2*>(p));
    o[0] = v.x;
    o[1] = v.y;
  }
  static __device__ __forceinline__ double one(const double* p) { return *p; }
};
template <>
struct Chunk<float, float> {
  static constexpr int VEC = 4;
  static __device__ __forceinline__ void load(const float* p, float* o) {
    const sf4 v = __builtin_nontemporal_load(reinterpret_cast<const sf4*>(p));
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
  static __device__ __forceinline__ float one(const float* p) { return *p; }
};
template <>
struct Chunk<__hip_bfloat16, float> {
  static constexpr int VEC = 8;
  static __device__ __forceinline__ void load(const __hip_bfloat16* p, float* o) {
    const su4 v = __builtin_nontemporal_load(reinterpret_cast<const su4*>(p));
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = __uint_as_float(w[i] << 16);
      o[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
    }
  }
  static __device__ __forceinline__ float one(const __hip_bfloat16* p) { return __bfloat162float(*p); }
};

template <class TC>
__device__ __forceinline__ TC xor_sum(TC v, int mask) {
  return v + __shfl_xor(v, mask, WAVE);
}

__device__ __forceinline__ int tile_row(int b) {
  int I = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((int64_t)(I + 1) * (I + 2) / 2 <= b) ++I;
  while ((int64_t)I * (I + 1) / 2 > b) --I;
  return I;
}

// the rows of one tile that belong to this wavefront. MASK: diagonal tile or a tile
// reaching past n (per-element checks); otherwise every chunk is whole and below the
// diagonal.
template <class TA, class TC, bool MASK>
__device__ __forceinline__ void tile_rows(const TA* __restrict__ A, int64_t lda, int64_t n,
                                          const double* __restrict__ x, int64_t r0, int64_t c0, bool diag,
                                          TC (&xj)[T / (LC * Chunk<TA, TC>::VEC)][Chunk<TA, TC>::VEC],
                                          TC (&za)[T / (LC * Chunk<TA, TC>::VEC)][Chunk<TA, TC>::VEC],
                                          double* ys) {
  constexpr int VEC = Chunk<TA, TC>::VEC;
  constexpr int M = T / (LC * VEC);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int kap = lane % LC, rho = lane / LC;
#pragma unroll 2
  for (int t = 0; t < T / (LR * NWV); ++t) {
    const int rl = w + NWV * (rho + LR * t);
    const int64_t gi = r0 + rl;
    TC ysum = (TC)0;
    if (!MASK || gi < n) {
      const TC xi = (TC)x[gi];
      const TA* arow = A + gi * lda;
      TC a[M][VEC];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int64_t col = c0 + m * (LC * VEC) + kap * VEC;
        if (!MASK) {
          Chunk<TA, TC>::load(arow + col, a[m]);
        } else if (col + VEC <= n && (!diag || col + VEC - 1 <= gi)) {
          Chunk<TA, TC>::load(arow + col, a[m]);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            const int64_t cc = col + v;
            a[m][v] = (cc < n && (!diag || cc <= gi)) ? Chunk<TA, TC>::one(arow + cc) : (TC)0;
          }
        }
      }
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          ysum = fma(a[m][v], xj[m][v], ysum);
          if (MASK && diag) {
            const int64_t cc = c0 + m * (LC * VEC) + kap * VEC + v;
            za[m][v] = fma((cc < gi) ? a[m][v] : (TC)0, xi, za[m][v]);
          } else {
            za[m][v] = fma(a[m][v], xi, za[m][v]);
          }
        }
    }
#pragma unroll
    for (int o = 1; o < LC; o <<= 1) ysum = xor_sum(ysum, o);
    if (kap == 0) ys[rl] = (double)ysum;
  }
}

template <class TA, class TC>
__global__ void __launch_bounds__(NB) k_symv_tiles(const TA* __restrict__ A, int64_t lda, int64_t n,
                                                  const double* __restrict__ x, const int32_t* __restrict__ skip,
                                                  double* __restrict__ ypart, double* __restrict__ zpart) {
  constexpr int VEC = Chunk<TA, TC>::VEC;
  constexpr int M = T / (LC * VEC);
  if (skip && skip[0]) return;
  __shared__ double ys[T];
  __shared__ double zs[NWV][T];
  const int b = blockIdx.x;
  const int I = tile_row(b);
  const int J = b - I * (I + 1) / 2;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int kap = lane % LC, rho = lane / LC;
  const int64_t r0 = (int64_t)I * T, c0 = (int64_t)J * T;
  TC xj[M][VEC], za[M][VEC];
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const int64_t col = c0 + m * (LC * VEC) + kap * VEC + v;
      xj[m][v] = (col < n) ? (TC)x[col] : (TC)0;
      za[m][v] = (TC)0;
    }
  const bool diag = I == J;
  const bool edge = r0 + T > n;  // the last tile row (and with it the last tile column)
  if (diag || edge)
    tile_rows<TA, TC, true>(A, lda, n, x, r0, c0, diag, xj, za, ys);
  else
    tile_rows<TA, TC, false>(A, lda, n, x, r0, c0, diag, xj, za, ys);
  // column sums over the 4 lane groups, then over the wavefronts in a fixed order
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      TC s = za[m][v];
      s = xor_sum(s, 16);
      s = xor_sum(s, 32);
      if (rho == 0) zs[w][m * (LC * VEC) + kap * VEC + v] = (double)s;
    }
  __syncthreads();
  for (int r = threadIdx.x; r < T; r += NB) {
    zpart[(int64_t)b * T + r] = (zs[0][r] + zs[1][r]) + (zs[2][r] + zs[3][r]);
    ypart[(int64_t)b * T + r] = ys[r];
  }
}

// q_i = sum_{J <= I} ypart(I, J)_i + sum_{I' >= I} zpart(I', I)_i (+ lam p_i), and the
// <p, q> partial of each block. A block takes 64 rows; wavefront q of 16 adds every 16th
// entry of the row's list (row partials of its tile row, then column partials of its tile
// column) and the 16 sums combine in a fixed order. Measured against 256 x 512 tiles with
// eight wavefronts on the same GPU, these tiles stream about 3% faster (699 against 720 us
// per n = 32768 sweep), and 16 wavefronts per row list cut the reduction from 14 to 6 us.
__global__ void __launch_bounds__(NG * NR) k_symv_reduce(const double* __restrict__ ypart,
                                                       const double* __restrict__ zpart, int64_t n, int N,
                                                       const double* __restrict__ x, double lam, int diag,
                                                       const int32_t* __restrict__ skip, double* __restrict__ y,
                                                       double* __restrict__ dot_part) {
  __shared__ double sh[NG][NR];
  const int lane = threadIdx.x % NR, q = threadIdx.x / NR;
  const int64_t r = (int64_t)blockIdx.x * NR + lane;
  const bool live = !(skip && skip[0]);
  double acc = 0.0;
  if (live && r < n) {
    const int I = (int)(r / T), rl = (int)(r % T);
    const int64_t rowb = (int64_t)I * (I + 1) / 2;
    for (int e = q; e <= N; e += NG) {
      // e <= I: row partial of tile (I, e); e > I: column partial of tile (e - 1, I)
      const int64_t tile = (e <= I) ? rowb + e : (int64_t)(e - 1) * e / 2 + I;
      acc += ((e <= I) ? ypart : zpart)[tile * T + rl];
    }
  }
  sh[q][lane] = acc;
  __syncthreads();
  if (q != 0) return;  // whole wavefronts leave; no barrier follows
  double prod = 0.0;
  if (live && r < n) {
    const double xr = x[r];
    double v = 0.0;
#pragma unroll
    for (int g = 0; g < NG; g += 2) v += sh[g][lane] + sh[g + 1][lane];
    if (diag) v += lam * xr;
    y[r] = v;
    prod = xr * v;
  }
  if (dot_part) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) prod += __shfl_xor(prod, off, WAVE);
    if (lane == 0) dot_part[blockIdx.x] = prod;
  }
}

template <class TA, class TC>
hipError_t symv_t(hipStream_t st, const TA* A, int64_t n, int64_t lda, const double* x, double* y, double lam,
                  bool diag, const int32_t* skip, double* part, double* dot_part, int* nblocks) {
  const int N = (int)((n + T - 1) / T);
  const int64_t tiles = (int64_t)N * (N + 1) / 2;
  double* ypart = part;
  double* zpart = part + tiles * T;
  hipLaunchKernelGGL((k_symv_tiles<TA, TC>), dim3((unsigned)tiles), dim3(NB), 0, st, A, lda, n, x, skip, ypart,
                     zpart);
  const unsigned rb = (unsigned)((n + NR - 1) / NR);
  hipLaunchKernelGGL(k_symv_reduce, dim3(rb), dim3(NG * NR), 0, st, ypart, zpart, n, N, x, lam, diag ? 1 : 0, skip, y,
                     dot_part);
  if (nblocks) *nblocks = (int)rb;
  return hipGetLastError();
}

}  // namespace

size_t symv_part_doubles(int64_t n) {
  const int64_t N = (n + T - 1) / T;
  return (size_t)(N * (N + 1)) * T + 64;  // row and column partials of every tile
}

bool symv_supported(const void* A, msp_dtype t, int64_t lda, int64_t k) {
  if (k != 1 || ((uintptr_t)A % 16) != 0) return false;
  const int64_t es = t == MSP_F64 ? 8 : (t == MSP_F32 ? 4 : 2);
  return (lda * es) % 16 == 0;
}

hipError_t launch_symv(hipStream_t st, const void* A, msp_dtype a_t, int64_t n, int64_t lda, const double* x,
                       double* y, double lam, bool diag_shift, const int32_t* skip, double* part, double* dot_part,
                       int* nblocks) {
  if (n < 1 || !symv_supported(A, a_t, lda, 1)) return hipErrorInvalidValue;
  switch (a_t) {
    case MSP_F64:
      return symv_t<double, double>(st, (const double*)A, n, lda, x, y, lam, diag_shift, skip, part, dot_part,
                                    nblocks);
    case MSP_F32:
      return symv_t<float, float>(st, (const float*)A, n, lda, x, y, lam, diag_shift, skip, part, dot_part, nblocks);
    case MSP_BF16:
      return symv_t<__hip_bfloat16, float>(st, (const __hip_bfloat16*)A, n, lda, x, y, lam, diag_shift, skip, part,
                                           dot_part, nblocks);
  }
  return hipErrorInvalidValue;
}
