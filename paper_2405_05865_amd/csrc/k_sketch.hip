// Sparse embedding (Definition 2.1): index draw, bucket lists, and the two sparse
// products of the method: Y = A S^T (Algorithms 1 and 3) and
// row gathers S X / Phi X on a tall X (W = S C, C~ = Phi C, A^ = Phi A~).
#include "msp_internal.h"

#include <hip/hip_bf16.h>

#include <algorithm>

namespace {

constexpr int kMaxGamma = 32;

__device__ __forceinline__ uint64_t fmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// One thread per column i: the SplitMix64 counter-based draw, first gamma distinct rows.
__global__ void k_sketch_gen(uint64_t seed, int64_t n, uint64_t s, int gamma, int32_t* __restrict__ rows,
                             int8_t* __restrict__ signs) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t G = 0x9E3779B97F4A7C15ull;
  const uint64_t key = fmix64(seed + (uint64_t)(i + 1) * G);
  int got[kMaxGamma];
  int cnt = 0;
  uint64_t a = 0;
  while (cnt < gamma) {
    ++a;
    const uint64_t u = fmix64(key + a * G);
    const int r = (int)(((u >> 32) * s) >> 32);
    bool dup = false;
    for (int g = 0; g < cnt; ++g) dup |= (got[g] == r);
    if (dup) continue;
    got[cnt] = r;
    rows[i * gamma + cnt] = r;
    signs[i * gamma + cnt] = (u & 1ull) ? (int8_t)-1 : (int8_t)1;
    ++cnt;
  }
}

// Gaussian probes (Box-Muller over the same counter-based stream): probe j has key
// fmix(seed ^ kProbeDomain + (j+1) G); element i takes draws 2i+1 and 2i+2 of that key's
// stream as U1 = (hi53 + 1) 2^-53 in (0, 1] and U2 = hi53 2^-53 in [0, 1), and
// g = sqrt(-2 ln U1) cos(2 pi U2). One thread per element.
constexpr uint64_t kProbeDomain = 0xD1B54A32D192ED03ull;
__global__ void k_probes_off(uint64_t seed, int64_t n, int64_t j0, double* __restrict__ G, int64_t ldg) {
  const int64_t j = j0 + blockIdx.y;
  const uint64_t Gc = 0x9E3779B97F4A7C15ull;
  const uint64_t key = fmix64((seed ^ kProbeDomain) + (uint64_t)(j + 1) * Gc);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t u1 = fmix64(key + (uint64_t)(2 * i + 1) * Gc);
    const uint64_t u2 = fmix64(key + (uint64_t)(2 * i + 2) * Gc);
    const double U1 = ((double)(u1 >> 11) + 1.0) * 0x1p-53;
    const double U2 = (double)(u2 >> 11) * 0x1p-53;
    G[j * ldg + i] = sqrt(-2.0 * log(U1)) * cos(2.0 * M_PI * U2);
  }
}

// ---- deterministic counting sort of the n*gamma entries by sketch row -------------
constexpr int kChunk = 2048;  // entries per chunk

__global__ void k_bucket_hist(const int32_t* __restrict__ rows, int64_t E, int nrows, int32_t* __restrict__ H) {
  extern __shared__ int32_t hist[];
  for (int j = threadIdx.x; j < nrows; j += blockDim.x) hist[j] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * kChunk;
  const int64_t e1 = min(E, e0 + kChunk);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) atomicAdd(&hist[rows[e]], 1);
  __syncthreads();
  int32_t* out = H + (int64_t)blockIdx.x * nrows;
  for (int j = threadIdx.x; j < nrows; j += blockDim.x) out[j] = hist[j];
}

// per bucket: exclusive scan over chunks (in place), totals out
__global__ void k_bucket_colscan(int32_t* __restrict__ H, int nchunks, int nrows, int32_t* __restrict__ total) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrows) return;
  int32_t run = 0;
  for (int c = 0; c < nchunks; ++c) {
    const int32_t t = H[(int64_t)c * nrows + j];
    H[(int64_t)c * nrows + j] = run;
    run += t;
  }
  total[j] = run;
}

// exclusive scan of totals -> offsets[0..nrows]; single block of 1024 threads
__global__ void k_offsets_scan(const int32_t* __restrict__ total, int nrows, int32_t* __restrict__ offsets) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int per = (nrows + 1023) / 1024;
  const int j0 = t * per, j1 = min(nrows, j0 + per);
  int32_t sum = 0;
  for (int j = j0; j < j1; ++j) sum += total[j];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
    const int32_t v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = (t == 0) ? 0 : part[t - 1];
  for (int j = j0; j < j1; ++j) {
    offsets[j] = run;
    run += total[j];
  }
  if (t == 1023) offsets[nrows] = part[1023];
}

// place the entries of one chunk in entry order (stable): the chunk's rows are staged in
// LDS, then one wavefront walks its columns in order, lane g placing draw g of each column
// (the gamma rows of a column are distinct, so the lanes of one step never share a bucket)
__global__ void __launch_bounds__(256) k_bucket_place(const int32_t* __restrict__ rows,
                                                      const int8_t* __restrict__ signs, int64_t E, int gamma,
                                                      int nrows, const int32_t* __restrict__ H,
                                                      const int32_t* __restrict__ offsets,
                                                      int32_t* __restrict__ entries) {
  extern __shared__ int32_t base[];  // [nrows] bucket cursors, then [kChunk] staged rows
  int32_t* rw = base + nrows;
  const int32_t* h = H + (int64_t)blockIdx.x * nrows;
  const int64_t e0 = (int64_t)blockIdx.x * kChunk;
  const int64_t e1 = min(E, e0 + kChunk);
  for (int j = threadIdx.x; j < nrows; j += blockDim.x) base[j] = offsets[j] + h[j];
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x)
    rw[e - e0] = (rows[e] << 1) | (signs[e] < 0 ? 1 : 0);
  __syncthreads();
  const int g = threadIdx.x;
  if (g >= gamma) return;  // whole lanes of the first wavefront stay; no barrier follows
  // chunks start at multiples of kChunk entries; columns that straddle a chunk boundary
  // are walked by both chunks, each placing only its own entries
  const int64_t c_first = e0 / gamma, c_last = (e1 - 1) / gamma;
  for (int64_t c = c_first; c <= c_last; ++c) {
    const int64_t e = c * gamma + g;
    if (e >= e0 && e < e1) {
      const int32_t v = rw[e - e0];
      entries[base[v >> 1]++] = ((int32_t)c << 1) | (v & 1);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ---- tile-major lists of S for Y = A S^T --------------------------------------------
// The columns of A are cut into tiles of wc columns. For tile t, its wc * gamma entries
// are grouped by sketch row j (bucket), columns increasing inside a bucket, at
// tent[t * wc * gamma + ...]; toff[t * (s + 1) + j] is the absolute start of bucket j of
// tile t (toff[... + s] the end of the tile). Entry = (column within the tile << 1) | neg.
// One block per tile: rows staged in LDS, bucket counts by LDS integer atomics (the counts
// do not depend on their order), an exclusive scan, then one wavefront places the entries
// column by column (lane g places draw g; a column's gamma rows are distinct).
__global__ void __launch_bounds__(256) k_tile_lists(const int32_t* __restrict__ rows, const int8_t* __restrict__ signs,
                                                    int64_t n, int s, int gamma, int wc, int32_t* __restrict__ toff,
                                                    int32_t* __restrict__ tent) {
  extern __shared__ int32_t sh[];  // cnt[s], part[256], rw[wc * gamma]
  int32_t* cnt = sh;
  int32_t* part = sh + s;
  int32_t* rw = part + 256;
  const int64_t t = blockIdx.x;
  const int64_t c0 = t * wc;
  const int cols = (int)min<int64_t>(wc, n - c0);
  const int E = cols * gamma;
  const int64_t base = c0 * gamma;
  for (int j = threadIdx.x; j < s; j += 256) cnt[j] = 0;
  for (int e = threadIdx.x; e < E; e += 256) rw[e] = (rows[base + e] << 1) | (signs[base + e] < 0 ? 1 : 0);
  __syncthreads();
  for (int e = threadIdx.x; e < E; e += 256) atomicAdd(&cnt[rw[e] >> 1], 1);
  __syncthreads();
  // exclusive scan of cnt[0..s): each thread scans a contiguous run, then the run totals
  const int per = (s + 255) / 256;
  const int j0 = threadIdx.x * per, j1 = min(s, j0 + per);
  int32_t run = 0;
  for (int j = j0; j < j1; ++j) run += cnt[j];
  part[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele scan of the run totals
    const int32_t v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int32_t pos = threadIdx.x == 0 ? 0 : part[threadIdx.x - 1];
  int32_t* to = toff + t * (s + 1);
  for (int j = j0; j < j1; ++j) {
    const int32_t c = cnt[j];
    cnt[j] = pos;  // becomes the bucket's cursor
    to[j] = (int32_t)base + pos;
    pos += c;
  }
  if (threadIdx.x == 0) to[s] = (int32_t)base + E;
  __syncthreads();
  const int g = threadIdx.x;
  if (g >= gamma) return;  // lanes of the first wavefront stay; no barrier follows
  for (int c = 0; c < cols; ++c) {
    const int32_t v = rw[c * gamma + g];
    tent[base + cnt[v >> 1]++] = (c << 1) | (v & 1);
    __builtin_amdgcn_wave_barrier();
  }
}

// ---- Y = A S^T over the tile-major lists -------------------------------------------
// A block takes R rows of A and walks the column tiles. Tile t + 1 (its R x wc block of A,
// its entries and bucket starts) is loaded into registers while tile t is processed from
// LDS, then stored to the other LDS buffer: one barrier per tile. The tile is stored
// column-major, each column's R values contiguous (plus a 16-byte pad that spreads the
// columns over the LDS banks), so one entry costs R / (16 / sizeof(TA)) 16-byte LDS reads.
// Thread j owns sketch rows (buckets) j, j + 256, ...: it adds the columns of its bucket's
// entries, in column order, into R accumulators per bucket (the order of the old bucket
// walk, so the sums are the same bits).
template <class TA, int R>
struct TileCol;  // one column of the LDS tile: R values as 16-byte vectors
template <int R>
struct TileCol<double, R> {
  static constexpr int LDR = R + 2;  // doubles per column, 16-byte pad
  template <class TC>
  static __device__ __forceinline__ void add(const double* col, TC sgn, TC* acc) {
#pragma unroll
    for (int q = 0; q < R / 2; ++q) {
      const double2 v = *reinterpret_cast<const double2*>(col + 2 * q);
      acc[2 * q] = fma(sgn, v.x, acc[2 * q]);
      acc[2 * q + 1] = fma(sgn, v.y, acc[2 * q + 1]);
    }
  }
};
template <int R>
struct TileCol<float, R> {
  static constexpr int LDR = R + 4;
  template <class TC>
  static __device__ __forceinline__ void add(const float* col, TC sgn, TC* acc) {
#pragma unroll
    for (int q = 0; q < R / 4; ++q) {
      const float4 v = *reinterpret_cast<const float4*>(col + 4 * q);
      acc[4 * q] = fmaf(sgn, v.x, acc[4 * q]);
      acc[4 * q + 1] = fmaf(sgn, v.y, acc[4 * q + 1]);
      acc[4 * q + 2] = fmaf(sgn, v.z, acc[4 * q + 2]);
      acc[4 * q + 3] = fmaf(sgn, v.w, acc[4 * q + 3]);
    }
  }
};
template <int R>
struct TileCol<__hip_bfloat16, R> {
  static constexpr int LDR = R + 8;
  template <class TC>
  static __device__ __forceinline__ void add(const __hip_bfloat16* col, TC sgn, TC* acc) {
#pragma unroll
    for (int q = 0; q < R / 8; ++q) {
      const uint4 v = *reinterpret_cast<const uint4*>(col + 8 * q);
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float lo = __uint_as_float(w[i] << 16), hi = __uint_as_float(w[i] & 0xFFFF0000u);
        acc[8 * q + 2 * i] = fmaf(sgn, lo, acc[8 * q + 2 * i]);
        acc[8 * q + 2 * i + 1] = fmaf(sgn, hi, acc[8 * q + 2 * i + 1]);
      }
    }
  }
};

constexpr int kTileEntries = 1024;  // entries per tile: wc * gamma <= 1024 (sketch_tile_width)

// one element of A, streamed past the caches (it is read once)
template <class TA>
__device__ __forceinline__ TA load_stream(const TA* p) {
  return __builtin_nontemporal_load(p);
}
template <>
__device__ __forceinline__ __hip_bfloat16 load_stream<__hip_bfloat16>(const __hip_bfloat16* p) {
  const unsigned short u = __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p));
  return __builtin_bit_cast(__hip_bfloat16, u);
}

template <class TA, class TC, class TY, int R, int WC, int BPT>
__global__ void __launch_bounds__(256) k_sketch_tiles(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                      int s, const int32_t* __restrict__ toff,
                                                      const int32_t* __restrict__ tent, TC scale,
                                                      TY* __restrict__ Y, int64_t ldy, int ntiles) {
  constexpr int LDR = TileCol<TA, R>::LDR;
  constexpr int PER = (WC * R) / 256;              // elements of A per thread per tile
  constexpr int EPT = kTileEntries / 256;          // entries per thread per tile (bound)
  constexpr int NOFF = 256 * BPT + 1;
  constexpr int OPT = (NOFF + 255) / 256;
  __shared__ __align__(16) TA tile[2][WC * LDR];
  __shared__ int32_t ent[2][kTileEntries];
  __shared__ int32_t off[2][NOFF];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * R;
  TC acc[BPT][R];
#pragma unroll
  for (int b = 0; b < BPT; ++b)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[b][r] = (TC)0;
  TA v[PER];
  int32_t ev[EPT], ov[OPT];
  // tile t into registers: A (consecutive threads take consecutive columns of a row),
  // its entries (relative to the tile's first) and its bucket starts
  auto gload = [&](int t) {
    const int64_t c0 = (int64_t)t * WC;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * 256;
      const int c = idx % WC, rr = idx / WC;
      const int64_t row = r0 + rr, col = c0 + c;
      v[k] = (row < m && col < n) ? load_stream(A + row * lda + col) : TA(0);
    }
    const int32_t* to = toff + (int64_t)t * (s + 1);
    const int32_t b0 = to[0];
    const int cnt = to[s] - b0;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int i = tid + k * 256;
      ev[k] = i < cnt ? tent[b0 + i] : 0;
    }
#pragma unroll
    for (int k = 0; k < OPT; ++k) {
      const int j = tid + k * 256;
      ov[k] = j <= s ? to[j] - b0 : 0;
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * 256;
      tile[buf][(idx % WC) * LDR + idx / WC] = v[k];
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) ent[buf][tid + k * 256] = ev[k];
#pragma unroll
    for (int k = 0; k < OPT; ++k) {
      const int j = tid + k * 256;
      if (j < NOFF) off[buf][j] = ov[k];
    }
  };
  gload(0);
  lstore(0);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    const int buf = t & 1;
    if (t + 1 < ntiles) gload(t + 1);
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int j = tid + b * 256;
      if (j < s) {
        const int p1 = off[buf][j + 1];
        for (int p = off[buf][j]; p < p1; ++p) {
          const int32_t e = ent[buf][p];
          // the entry's sign as a factor: fma(-1, v, a) rounds exactly as a - v
          TileCol<TA, R>::add(&tile[buf][(e >> 1) * LDR], (e & 1) ? TC(-1) : TC(1), acc[b]);
        }
      }
    }
    if (t + 1 < ntiles) lstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = tid + b * 256;
    if (j >= s) continue;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r0 + r < m) Y[(r0 + r) * ldy + j] = (TY)(acc[b][r] * scale);
  }
}

// admissible rows per block: at most 32 (FP64) or 64 (FP32 accumulators) per thread over its
// BPT buckets, at least one 16-byte vector per tile column, at least one element of A per
// thread and tile
template <class TA, int WC, int BPT, int RR>
constexpr bool rows_ok() {
  return RR * BPT <= (sizeof(TA) == 8 ? 32 : 64) && RR * (int)sizeof(TA) >= 16 && (WC * RR) % 256 == 0;
}

template <class TA, class TC, class TY, int WC, int BPT, int RR>
hipError_t tiles_launch(hipStream_t st, const TA* A, int64_t m, int64_t n, int64_t lda, int s, TileLists L,
                        double scale, TY* Y, int64_t ldy) {
  if constexpr (rows_ok<TA, WC, BPT, RR>()) {
    hipLaunchKernelGGL((k_sketch_tiles<TA, TC, TY, RR, WC, BPT>), dim3((unsigned)((m + RR - 1) / RR)), dim3(256), 0,
                       st, A, lda, m, n, s, L.toff, L.tent, (TC)scale, Y, ldy, L.ntiles);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

// R: rows of A per block (accumulators R x BPT per thread); 0 picks the built-in rule: the
// largest admissible of 16, 8, 4, ...
template <class TA, class TC, class TY, int WC, int BPT>
hipError_t tiles_r(hipStream_t st, const TA* A, int64_t m, int64_t n, int64_t lda, int s, TileLists L, double scale,
                   TY* Y, int64_t ldy, int R) {
  if (R == 0) {
    R = rows_ok<TA, WC, BPT, 16>() ? 16
        : rows_ok<TA, WC, BPT, 8>() ? 8
        : rows_ok<TA, WC, BPT, 32>() ? 32
        : rows_ok<TA, WC, BPT, 4>() ? 4 : 2;
  }
  switch (R) {
    case 2: return tiles_launch<TA, TC, TY, WC, BPT, 2>(st, A, m, n, lda, s, L, scale, Y, ldy);
    case 4: return tiles_launch<TA, TC, TY, WC, BPT, 4>(st, A, m, n, lda, s, L, scale, Y, ldy);
    case 8: return tiles_launch<TA, TC, TY, WC, BPT, 8>(st, A, m, n, lda, s, L, scale, Y, ldy);
    case 16: return tiles_launch<TA, TC, TY, WC, BPT, 16>(st, A, m, n, lda, s, L, scale, Y, ldy);
    case 32: return tiles_launch<TA, TC, TY, WC, BPT, 32>(st, A, m, n, lda, s, L, scale, Y, ldy);
  }
  return hipErrorInvalidValue;
}

template <class TA, class TC, class TY, int WC>
hipError_t tiles_b(hipStream_t st, const TA* A, int64_t m, int64_t n, int64_t lda, int s, TileLists L, double scale,
                   TY* Y, int64_t ldy, int R) {
  const int bpt = (s + 255) / 256;
  if (bpt <= 1) return tiles_r<TA, TC, TY, WC, 1>(st, A, m, n, lda, s, L, scale, Y, ldy, R);
  if (bpt <= 2) return tiles_r<TA, TC, TY, WC, 2>(st, A, m, n, lda, s, L, scale, Y, ldy, R);
  if (bpt <= 4) return tiles_r<TA, TC, TY, WC, 4>(st, A, m, n, lda, s, L, scale, Y, ldy, R);
  if (bpt <= 8) return tiles_r<TA, TC, TY, WC, 8>(st, A, m, n, lda, s, L, scale, Y, ldy, R);
  return hipErrorInvalidValue;
}

template <class TA, class TC, class TY>
hipError_t tiles_dispatch(hipStream_t st, const TA* A, int64_t m, int64_t n, int64_t lda, int s, TileLists L,
                          double scale, TY* Y, int64_t ldy, int R) {
  if (L.wc == 128) return tiles_b<TA, TC, TY, 128>(st, A, m, n, lda, s, L, scale, Y, ldy, R);
  if (L.wc == 64) return tiles_b<TA, TC, TY, 64>(st, A, m, n, lda, s, L, scale, Y, ldy, R);
  if (L.wc == 32) return tiles_b<TA, TC, TY, 32>(st, A, m, n, lda, s, L, scale, Y, ldy, R);
  return hipErrorInvalidValue;
}

// ---- out[j, :] = scale * sum_{e in bucket j} sign(e) X[col(e), :] -----------------
template <class TX>
__global__ void __launch_bounds__(256) k_gather_rows(const TX* __restrict__ X, int64_t ldx, int64_t ncols,
                                                     const int32_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ entries, double scale,
                                                     double* __restrict__ out, int64_t ldo) {
  const int j = blockIdx.x;
  const int p0 = offsets[j], p1 = offsets[j + 1];
  for (int64_t c = threadIdx.x; c < ncols; c += blockDim.x) {
    double acc = 0.0;
    for (int p = p0; p < p1; ++p) {
      const int32_t ent = entries[p];
      const double v = (double)X[(int64_t)(ent >> 1) * ldx + c];
      acc += (ent & 1) ? -v : v;
    }
    out[(int64_t)j * ldo + c] = acc * scale;
  }
}

}  // namespace

hipError_t launch_sketch_gen(hipStream_t st, uint64_t seed, int64_t n, int64_t s, int32_t gamma, int32_t* rows,
                             int8_t* signs) {
  const int nt = 256;
  hipLaunchKernelGGL(k_sketch_gen, dim3((unsigned)((n + nt - 1) / nt)), dim3(nt), 0, st, seed, n, (uint64_t)s,
                     (int)gamma, rows, signs);
  return hipGetLastError();
}

hipError_t launch_probes(hipStream_t st, uint64_t seed, int64_t n, int64_t N, double* G, int64_t ldg) {
  const int64_t bx = std::min<int64_t>((n + 255) / 256, 64);
  for (int64_t j0 = 0; j0 < N; j0 += 65535) {
    const int64_t nj = std::min<int64_t>(65535, N - j0);
    hipLaunchKernelGGL(k_probes_off, dim3((unsigned)bx, (unsigned)nj), dim3(256), 0, st, seed, n, j0, G, ldg);
  }
  return hipGetLastError();
}

size_t bucket_scratch_bytes(int64_t n, int64_t nrows, int32_t gamma) {
  const int64_t E = n * gamma;
  const int64_t nchunks = (E + kChunk - 1) / kChunk;
  return (size_t)(nchunks * nrows + nrows) * sizeof(int32_t) + 512;
}

hipError_t build_buckets(hipStream_t st, const int32_t* rows, const int8_t* signs, int64_t n, int64_t nrows,
                         int32_t gamma, BucketLists out, void* scratch) {
  const int64_t E = n * gamma;
  const int nchunks = (int)((E + kChunk - 1) / kChunk);
  int32_t* H = (int32_t*)scratch;
  int32_t* total = H + (int64_t)nchunks * nrows;
  const size_t lds = (size_t)nrows * sizeof(int32_t);
  hipLaunchKernelGGL(k_bucket_hist, dim3(nchunks), dim3(256), lds, st, rows, E, (int)nrows, H);
  hipLaunchKernelGGL(k_bucket_colscan, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, st, H, nchunks,
                     (int)nrows, total);
  hipLaunchKernelGGL(k_offsets_scan, dim3(1), dim3(1024), 0, st, total, (int)nrows, out.offsets);
  hipLaunchKernelGGL(k_bucket_place, dim3(nchunks), dim3(256), lds + kChunk * sizeof(int32_t), st, rows, signs, E,
                     (int)gamma, (int)nrows, H, out.offsets, out.entries);
  return hipGetLastError();
}

int sketch_tile_width(int32_t gamma) { return gamma <= 8 ? 128 : (gamma <= 16 ? 64 : 32); }

size_t tile_lists_ints(int64_t n, int64_t s, int32_t gamma) {
  const int wc = sketch_tile_width(gamma);
  const int64_t ntiles = (n + wc - 1) / wc;
  return (size_t)(ntiles * (s + 1) + n * gamma);
}

TileLists carve_tile_lists(int32_t* base, int64_t n, int64_t s, int32_t gamma) {
  TileLists L;
  L.wc = sketch_tile_width(gamma);
  L.ntiles = (int)((n + L.wc - 1) / L.wc);
  L.toff = base;
  L.tent = base ? base + (int64_t)L.ntiles * (s + 1) : nullptr;
  return L;
}

hipError_t build_tile_lists(hipStream_t st, const int32_t* rows, const int8_t* signs, int64_t n, int64_t s,
                            int32_t gamma, TileLists L) {
  const size_t lds = (size_t)(s + 256 + L.wc * gamma) * sizeof(int32_t);
  hipLaunchKernelGGL(k_tile_lists, dim3((unsigned)L.ntiles), dim3(256), lds, st, rows, signs, n, (int)s, (int)gamma,
                     L.wc, L.toff, L.tent);
  return hipGetLastError();
}

hipError_t launch_sketch_apply(hipStream_t st, const void* A, msp_dtype a_t, int64_t m, int64_t n, int64_t lda,
                               int64_t s, TileLists L, double scale, void* Y, msp_dtype y_t, int64_t ldy, int R) {
  const int si = (int)s;
  if (y_t == MSP_F64) {
    if (a_t != MSP_F64) return hipErrorInvalidValue;
    return tiles_dispatch<double, double, double>(st, (const double*)A, m, n, lda, si, L, scale, (double*)Y, ldy, R);
  }
  if (a_t == MSP_F64) return hipErrorInvalidValue;
  if (a_t == MSP_F32)
    return tiles_dispatch<float, float, float>(st, (const float*)A, m, n, lda, si, L, scale, (float*)Y, ldy, R);
  return tiles_dispatch<__hip_bfloat16, float, float>(st, (const __hip_bfloat16*)A, m, n, lda, si, L, scale,
                                                      (float*)Y, ldy, R);
}

hipError_t launch_gather_rows(hipStream_t st, const void* X, msp_dtype x_t, int64_t ldx, int64_t ncols,
                              int64_t nrows, BucketLists b, double scale, double* out, int64_t ldo) {
  if (x_t == MSP_F64)
    hipLaunchKernelGGL(k_gather_rows<double>, dim3((unsigned)nrows), dim3(256), 0, st, (const double*)X, ldx, ncols,
                       b.offsets, b.entries, scale, out, ldo);
  else if (x_t == MSP_F32)
    hipLaunchKernelGGL(k_gather_rows<float>, dim3((unsigned)nrows), dim3(256), 0, st, (const float*)X, ldx, ncols,
                       b.offsets, b.entries, scale, out, ldo);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
