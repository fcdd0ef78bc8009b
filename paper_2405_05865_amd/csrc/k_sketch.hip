// Sparse embedding (Definition 2.1): index draw, bucket lists, and the two sparse
// products of the method: Y = A S^T (Algorithm 1 line 3, Algorithm 3 line 4) and
// row gathers S X / Phi X on a tall X (W = S C, C~ = Phi C, A^ = Phi A~).
#include "msp_internal.h"

#include <hip/hip_bf16.h>

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

// place entries of one chunk in entry order (stable): a single thread walks the chunk
__global__ void k_bucket_place(const int32_t* __restrict__ rows, const int8_t* __restrict__ signs, int64_t E,
                               int gamma, int nrows, const int32_t* __restrict__ H,
                               const int32_t* __restrict__ offsets, int32_t* __restrict__ entries) {
  extern __shared__ int32_t base[];
  const int32_t* h = H + (int64_t)blockIdx.x * nrows;
  for (int j = threadIdx.x; j < nrows; j += blockDim.x) base[j] = offsets[j] + h[j];
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int64_t e0 = (int64_t)blockIdx.x * kChunk;
  const int64_t e1 = min(E, e0 + kChunk);
  for (int64_t e = e0; e < e1; ++e) {
    const int j = rows[e];
    const int32_t col = (int32_t)(e / gamma);
    entries[base[j]++] = (col << 1) | (signs[e] < 0 ? 1 : 0);
  }
}

// ---- Y = A S^T: LDS-staged row tiles, one thread per sketch row (bucket) ----------
template <class TA, class TACC>
__device__ __forceinline__ TACC load_as(const TA v);
template <>
__device__ __forceinline__ double load_as<double, double>(const double v) { return v; }
template <>
__device__ __forceinline__ float load_as<float, float>(const float v) { return v; }
template <>
__device__ __forceinline__ float load_as<__hip_bfloat16, float>(const __hip_bfloat16 v) { return __bfloat162float(v); }

template <class TA, class TACC, class TY, int R, int BPT>
__global__ void __launch_bounds__(256) k_sketch_apply(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                      int s, const int32_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ entries, TACC scale,
                                                      TY* __restrict__ Y, int64_t ldy, int WC) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TA* tile = reinterpret_cast<TA*>(smem_raw);  // [R][WC]
  const int64_t r0 = (int64_t)blockIdx.x * R;
  const int nt = blockDim.x;
  TACC acc[BPT][R];
  int ptr[BPT], end[BPT];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = threadIdx.x + b * nt;
    ptr[b] = (j < s) ? offsets[j] : 0;
    end[b] = (j < s) ? offsets[j + 1] : 0;
#pragma unroll
    for (int r = 0; r < R; ++r) acc[b][r] = (TACC)0;
  }
  for (int64_t c0 = 0; c0 < n; c0 += WC) {
    const int cw = (int)min<int64_t>(WC, n - c0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = r0 + r;
      const TA* src = A + row * lda + c0;
      for (int c = threadIdx.x; c < cw; c += nt) tile[r * WC + c] = (row < m) ? src[c] : TA(0);
    }
    __syncthreads();
    const int32_t c1 = (int32_t)(c0 + cw);
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      int p = ptr[b];
      const int e = end[b];
      while (p < e) {
        const int32_t ent = entries[p];
        const int32_t col = ent >> 1;
        if (col >= c1) break;
        const int lc = col - (int32_t)c0;
        const bool neg = ent & 1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const TACC v = load_as<TA, TACC>(tile[r * WC + lc]);
          acc[b][r] += neg ? -v : v;
        }
        ++p;
      }
      ptr[b] = p;
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = threadIdx.x + b * nt;
    if (j >= s) continue;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = r0 + r;
      if (row < m) Y[row * ldy + j] = (TY)(acc[b][r] * scale);
    }
  }
}

template <class TA, class TACC, class TY, int R, int BPT>
hipError_t sketch_apply_t(hipStream_t st, const TA* A, int64_t m, int64_t n, int64_t lda, int s, BucketLists b,
                          double scale, TY* Y, int64_t ldy) {
  const int nt = (s >= 256) ? 256 : ((s + 63) / 64) * 64;
  const int lds_bytes = 64 * 1024;
  int WC = lds_bytes / (R * (int)sizeof(TA));
  WC = (WC / 64) * 64;
  const int64_t blocks = (m + R - 1) / R;
  hipLaunchKernelGGL((k_sketch_apply<TA, TACC, TY, R, BPT>), dim3((unsigned)blocks), dim3(nt),
                     (size_t)R * WC * sizeof(TA), st, A, lda, m, n, s, b.offsets, b.entries, (TACC)scale, Y, ldy,
                     WC);
  return hipGetLastError();
}

template <class TA, class TACC, class TY>
hipError_t sketch_apply_dispatch(hipStream_t st, const TA* A, int64_t m, int64_t n, int64_t lda, int s,
                                 BucketLists b, double scale, TY* Y, int64_t ldy) {
  const int bpt = (s + 255) / 256;
  if (bpt <= 1) return sketch_apply_t<TA, TACC, TY, 16, 1>(st, A, m, n, lda, s, b, scale, Y, ldy);
  if (bpt <= 2) return sketch_apply_t<TA, TACC, TY, 16, 2>(st, A, m, n, lda, s, b, scale, Y, ldy);
  if (bpt <= 4) return sketch_apply_t<TA, TACC, TY, 8, 4>(st, A, m, n, lda, s, b, scale, Y, ldy);
  return sketch_apply_t<TA, TACC, TY, 4, 8>(st, A, m, n, lda, s, b, scale, Y, ldy);
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
  hipLaunchKernelGGL(k_bucket_place, dim3(nchunks), dim3(256), lds, st, rows, signs, E, (int)gamma, (int)nrows, H,
                     out.offsets, out.entries);
  return hipGetLastError();
}

hipError_t launch_sketch_apply(hipStream_t st, const void* A, msp_dtype a_t, int64_t m, int64_t n, int64_t lda,
                               int64_t s, BucketLists b, double scale, void* Y, msp_dtype y_t, int64_t ldy) {
  const int si = (int)s;
  if (y_t == MSP_F64) {
    if (a_t != MSP_F64) return hipErrorInvalidValue;
    return sketch_apply_dispatch<double, double, double>(st, (const double*)A, m, n, lda, si, b, scale, (double*)Y,
                                                         ldy);
  }
  if (a_t == MSP_F64) return hipErrorInvalidValue;
  if (a_t == MSP_F32)
    return sketch_apply_dispatch<float, float, float>(st, (const float*)A, m, n, lda, si, b, scale, (float*)Y, ldy);
  return sketch_apply_dispatch<__hip_bfloat16, float, float>(st, (const __hip_bfloat16*)A, m, n, lda, si, b, scale,
                                                             (float*)Y, ldy);
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
