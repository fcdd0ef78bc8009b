// Symmetric A-sweep from the lower triangle: q = (A + lam I) p reads A[i][j] for j <= i
// only, so a sweep streams n(n+1)/2 elements instead of n^2 (the level-1 operator of
// Algorithm 1 is symmetric by the problem statement). Each element of the strict lower
// triangle is used twice from one load: in the row dot (A p)_i and, mirrored, in the
// column sum (A^T p)_j.
//
// The lower triangle is cut into TH x TW tiles (TH = 256 rows, TW = 512 columns): row band
// I (rows I TH ..) holds the column chunks J = 0 .. floor(I / q), q = TW / TH, the last of
// which meets the diagonal; tiles are numbered band by band, so band I starts at
// tile_start(I) = I + q m (m - 1) / 2 + (I - q m) m with m = floor(I / q). A block has eight
// wavefronts; wavefront w takes the tile rows w, w + 8, ..., and all 64 lanes of a
// wavefront share a row (16-byte chunks, TW contiguous columns per row: 4 KB in FP64), so
// the row dot reduces over the wavefront and each lane keeps the column sums of its own
// columns in registers; the eight wavefronts' column sums add in LDS in a fixed order. A
// tile writes its row partials (ypart) and column partials (zpart); a second kernel adds,
// for each row, the row partials of its band and the column partials of its column chunk
// from the bands at and below it, in a fixed order, applies the shift and writes the
// <p, q> partials of the level-1 update. Tiles that reach the diagonal or the matrix edge
// mask per element (the strict upper triangle is not loaded; the diagonal is left out of
// the column sums). Measured on n = 32768 (FP64): 256 x 512 tiles with eight wavefronts
// stream about 3% faster than 256 x 256 tiles with four.
#include "msp_internal.h"

#include <hip/hip_bf16.h>

namespace {

constexpr int WAVE = 64;
constexpr int TH = 256;          // tile rows
constexpr int TW = 512;          // tile columns
constexpr int QT = TW / TH;      // column chunks per band step
constexpr int NWV = 8;           // wavefronts per block (rows interleaved)
constexpr int NB = NWV * WAVE;   // threads per block
constexpr int NR = 64;           // rows per block of the reduction
constexpr int NG = 16;           // partial sums per row of the reduction (one wavefront each)

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

__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// first tile of band I (tiles numbered band by band, band I has floor(I / QT) + 1 chunks)
__host__ __device__ __forceinline__ int64_t tile_start(int64_t I) {
  const int64_t m = I / QT, rem = I - m * QT;
  return I + QT * m * (m - 1) / 2 + rem * m;
}

// the band of tile b: the largest I with tile_start(I) <= b
__device__ __forceinline__ int tile_band(int64_t b, int nbands) {
  int lo = 0, hi = nbands - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_start(mid) <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// the rows of one tile that belong to this wavefront. MASK: a tile that reaches the
// diagonal or the matrix edge (per-element checks); otherwise every chunk is whole and
// strictly below the diagonal.
template <class TA, class TC, bool MASK>
__device__ __forceinline__ void tile_rows(const TA* __restrict__ A, int64_t lda, int64_t n,
                                          const double* __restrict__ x, int64_t r0, int64_t c0,
                                          TC (&xj)[TW / (WAVE * Chunk<TA, TC>::VEC)][Chunk<TA, TC>::VEC],
                                          TC (&za)[TW / (WAVE * Chunk<TA, TC>::VEC)][Chunk<TA, TC>::VEC],
                                          double* ys) {
  constexpr int VEC = Chunk<TA, TC>::VEC;
  constexpr int M = TW / (WAVE * VEC);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
#pragma unroll 2
  for (int t = 0; t < TH / NWV; ++t) {
    const int rl = w + NWV * t;
    const int64_t gi = r0 + rl;
    TC ysum = (TC)0;
    if (!MASK || gi < n) {
      const TC xi = (TC)x[gi];
      const TA* arow = A + gi * lda;
      TC a[M][VEC];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int64_t col = c0 + m * (WAVE * VEC) + lane * VEC;
        if (!MASK || (col + VEC <= n && col + VEC - 1 <= gi)) {
          Chunk<TA, TC>::load(arow + col, a[m]);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            const int64_t cc = col + v;
            a[m][v] = (cc < n && cc <= gi) ? Chunk<TA, TC>::one(arow + cc) : (TC)0;
          }
        }
      }
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          ysum = fma(a[m][v], xj[m][v], ysum);
          if (MASK) {
            const int64_t cc = c0 + m * (WAVE * VEC) + lane * VEC + v;
            za[m][v] = fma((cc < gi) ? a[m][v] : (TC)0, xi, za[m][v]);
          } else {
            za[m][v] = fma(a[m][v], xi, za[m][v]);
          }
        }
    }
    const double tot = wave_total((double)ysum);
    if (lane == 0) ys[rl] = tot;
  }
}

template <class TA, class TC>
__global__ void __launch_bounds__(NB) k_symv_tiles(const TA* __restrict__ A, int64_t lda, int64_t n, int nbands,
                                                  const double* __restrict__ x, const int32_t* __restrict__ skip,
                                                  double* __restrict__ ypart, double* __restrict__ zpart) {
  constexpr int VEC = Chunk<TA, TC>::VEC;
  constexpr int M = TW / (WAVE * VEC);
  if (skip && skip[0]) return;
  __shared__ double ys[TH];
  __shared__ double zs[NWV][TW];
  const int64_t b = blockIdx.x;
  const int I = tile_band(b, nbands);
  const int J = (int)(b - tile_start(I));
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int64_t r0 = (int64_t)I * TH, c0 = (int64_t)J * TW;
  TC xj[M][VEC], za[M][VEC];
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const int64_t col = c0 + m * (WAVE * VEC) + lane * VEC + v;
      xj[m][v] = (col < n) ? (TC)x[col] : (TC)0;
      za[m][v] = (TC)0;
    }
  const bool mask = (c0 + TW > r0) || (r0 + TH > n) || (c0 + TW > n);  // diagonal or edge
  if (mask)
    tile_rows<TA, TC, true>(A, lda, n, x, r0, c0, xj, za, ys);
  else
    tile_rows<TA, TC, false>(A, lda, n, x, r0, c0, xj, za, ys);
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int v = 0; v < VEC; ++v) zs[w][m * (WAVE * VEC) + lane * VEC + v] = (double)za[m][v];
  __syncthreads();
  // column sums over the wavefronts in a fixed order
  for (int c = threadIdx.x; c < TW; c += NB) {
    double t = 0.0;
#pragma unroll
    for (int ww = 0; ww < NWV; ++ww) t += zs[ww][c];
    zpart[b * TW + c] = t;
  }
  for (int r = threadIdx.x; r < TH; r += NB) ypart[b * TH + r] = ys[r];
}

// q_i = sum_J ypart(I, J)_i + sum_{I' >= I} zpart(I', i / TW)_i (+ lam p_i) for the row i of
// band I, and the <p, q> partial of each block. A block takes 64 rows; wavefront g adds
// every fourth entry of the row's list (row partials of its band, then column partials of
// its chunk from band I on) and the four sums combine in a fixed order.
__global__ void __launch_bounds__(NG * NR) k_symv_reduce(const double* __restrict__ ypart,
                                                        const double* __restrict__ zpart, int64_t n, int nbands,
                                                        const double* __restrict__ x, double lam, int diag,
                                                        const int32_t* __restrict__ skip, double* __restrict__ y,
                                                        double* __restrict__ dot_part) {
  __shared__ double sh[NG][NR];
  const int lane = threadIdx.x % NR, g = threadIdx.x / NR;
  const int64_t r = (int64_t)blockIdx.x * NR + lane;
  const bool live = !(skip && skip[0]);
  double acc = 0.0;
  if (live && r < n) {
    const int I = (int)(r / TH);
    const int nJ = I / QT + 1;
    const int Jc = (int)(r / TW);
    const int nt = nJ + (nbands - I);
    const int64_t oI = tile_start(I);
    const int rh = (int)(r % TH), rw = (int)(r % TW);
    for (int e = g; e < nt; e += NG) {
      if (e < nJ) acc += ypart[(oI + e) * TH + rh];
      else acc += zpart[(tile_start(I + (e - nJ)) + Jc) * TW + rw];
    }
  }
  sh[g][lane] = acc;
  __syncthreads();
  if (g != 0) return;  // whole wavefronts leave; no barrier follows
  double prod = 0.0;
  if (live && r < n) {
    const double xr = x[r];
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < NG; q += 2) v += sh[q][lane] + sh[q + 1][lane];
    if (diag) v += lam * xr;
    y[r] = v;
    prod = xr * v;
  }
  if (dot_part) {
    prod = wave_total(prod);
    if (lane == 0) dot_part[blockIdx.x] = prod;
  }
}

template <class TA, class TC>
hipError_t symv_t(hipStream_t st, const TA* A, int64_t n, int64_t lda, const double* x, double* y, double lam,
                  bool diag, const int32_t* skip, double* part, double* dot_part, int* nblocks) {
  const int nbands = (int)((n + TH - 1) / TH);
  const int64_t tiles = tile_start(nbands);
  double* ypart = part;
  double* zpart = part + tiles * TH;
  hipLaunchKernelGGL((k_symv_tiles<TA, TC>), dim3((unsigned)tiles), dim3(NB), 0, st, A, lda, n, nbands, x, skip,
                     ypart, zpart);
  const unsigned rb = (unsigned)((n + NR - 1) / NR);
  hipLaunchKernelGGL(k_symv_reduce, dim3(rb), dim3(NG * NR), 0, st, ypart, zpart, n, nbands, x, lam, diag ? 1 : 0,
                     skip, y, dot_part);
  if (nblocks) *nblocks = (int)rb;
  return hipGetLastError();
}

}  // namespace

size_t symv_part_doubles(int64_t n) {
  const int64_t tiles = tile_start((n + TH - 1) / TH);
  return (size_t)tiles * (TH + TW) + 64;  // row and column partials of every tile
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
