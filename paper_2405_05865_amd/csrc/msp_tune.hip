// Autotuners. (1) The level-1 block sweep Y = A X (k >= kGemmMinK right-hand sides on the
// matrix cores). The kernel's reduction range can be cut into 1..64 segments whose
// partials are summed afterwards; how many pay depends on the shape, the storage type and
// the number of right-hand sides (more wavefronts hide latency, more segments cost partial
// traffic and a summing pass). The built-in rule aims at about 2048 wavefronts; the tuner
// instead times every admissible count on the caller's matrix and keeps the fastest.
//
// (2) The sparse sketch Y = A S^T: the rows of A per block (R, each thread keeps R
// accumulators per sketch row it owns; more rows reuse each list entry more, fewer rows
// leave more blocks and registers), timed for every admissible R on the caller's matrix.
//
// Results are cached per shape for the life of the process (guarded by a mutex; tuning
// holds it, so concurrent tuners do not disturb each other's timings). When MSP_TUNE_CACHE
// names a file, earlier results are read from it at the first query and every new result
// is appended to it, one JSON object per line.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "msp_internal.h"

namespace {

using Key = std::tuple<int, int, int64_t, int64_t, int64_t, int64_t>;
// sketch: (A dtype, Y dtype, m, n, lda, s * 64 + gamma)
using SKey = std::tuple<int, int, int64_t, int64_t, int64_t, int64_t>;

std::mutex g_mu;
std::map<Key, int> g_cache;
std::map<SKey, int> g_sketch;
bool g_loaded = false;

const char* cache_path() {
  const char* p = getenv("MSP_TUNE_CACHE");
  return (p && p[0]) ? p : nullptr;
}

// the line format written by store(); other lines are skipped
void load_file() {
  g_loaded = true;
  const char* path = cache_path();
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    int dt = 0, f64 = 0, nseg = 0;
    long long rows = 0, cols = 0, lda = 0, k = 0;
    double ms = 0.0;
    if (sscanf(line,
               "{\"kernel\": \"block_sweep\", \"dtype\": %d, \"fp64_arith\": %d, \"rows\": %lld, \"cols\": %lld, "
               "\"lda\": %lld, \"k\": %lld, \"nseg\": %d, \"ms\": %lf}",
               &dt, &f64, &rows, &cols, &lda, &k, &nseg, &ms) == 8 &&
        nseg >= 1 && nseg <= 64)
      g_cache[Key(dt, f64, rows, cols, lda, k)] = nseg;
    int at = 0, yt = 0, R = 0, gam = 0;
    long long m = 0, n = 0, ld = 0, ss = 0;
    if (sscanf(line,
               "{\"kernel\": \"sketch_apply\", \"dtype\": %d, \"y_dtype\": %d, \"m\": %lld, \"n\": %lld, "
               "\"lda\": %lld, \"s\": %lld, \"gamma\": %d, \"rows_per_block\": %d, \"ms\": %lf}",
               &at, &yt, &m, &n, &ld, &ss, &gam, &R, &ms) == 9 &&
        R >= 1 && R <= 64)
      g_sketch[SKey(at, yt, m, n, ld, ss * 64 + gam)] = R;
  }
  fclose(f);
}

void store(const Key& key, int nseg, double ms) {
  g_cache[key] = nseg;
  const char* path = cache_path();
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f,
          "{\"kernel\": \"block_sweep\", \"dtype\": %d, \"fp64_arith\": %d, \"rows\": %lld, \"cols\": %lld, "
          "\"lda\": %lld, \"k\": %lld, \"nseg\": %d, \"ms\": %.6f}\n",
          std::get<0>(key), std::get<1>(key), (long long)std::get<2>(key), (long long)std::get<3>(key),
          (long long)std::get<4>(key), (long long)std::get<5>(key), nseg, ms);
  fclose(f);
}

}  // namespace

hipError_t tune_block_sweep(hipStream_t st, const void* A, msp_dtype a_t, bool fp64_arith, int64_t rows,
                            int64_t cols, int64_t lda, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k,
                            double* scratch, size_t scratch_doubles, int* nseg_out) {
  const bool f64 = fp64_arith && a_t == MSP_F32;
  const Key key((int)a_t, f64 ? 1 : 0, rows, cols, lda, k);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_loaded) load_file();
  auto it = g_cache.find(key);
  if (it != g_cache.end()) {
    *nseg_out = it->second;
    return hipSuccess;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int best = 0;
  float best_ms = 0.0f;
  constexpr int kReps = 3;
  for (int nseg = 1; nseg <= 64 && e == hipSuccess; nseg *= 2) {
    // admissible: partials fit the scratch and every segment keeps 64 columns or more
    if (nseg > 1 && ((size_t)nseg * (size_t)k * (size_t)rows > scratch_doubles || cols / nseg < 64)) break;
    int nb = 0;
    e = launch_gemm_split(st, A, a_t, f64, rows, cols, lda, X, ldx, Y, ldy, k, 0.0, false, nullptr, nullptr, &nb,
                          scratch, scratch_doubles, nseg);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < kReps && e == hipSuccess; ++r)
      e = launch_gemm_split(st, A, a_t, f64, rows, cols, lda, X, ldx, Y, ldy, k, 0.0, false, nullptr, nullptr, &nb,
                            scratch, scratch_doubles, nseg);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && (best == 0 || ms < best_ms)) {
      best = nseg;
      best_ms = ms;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  store(key, best, best_ms / kReps);
  *nseg_out = best;
  return hipSuccess;
}

int sketch_rows_choice(msp_dtype a_t, int64_t m, int64_t n, int64_t lda, int64_t s, int32_t gamma) {
  const msp_dtype y_t = a_t == MSP_F64 ? MSP_F64 : MSP_F32;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_loaded) load_file();
  auto it = g_sketch.find(SKey((int)a_t, (int)y_t, m, n, lda, s * 64 + gamma));
  return it == g_sketch.end() ? 0 : it->second;
}

hipError_t tune_sketch_apply(hipStream_t st, const void* A, msp_dtype a_t, int64_t m, int64_t n, int64_t lda,
                             int64_t s, int32_t gamma, const TileLists& L, void* Y, msp_dtype y_t, int64_t ldy,
                             int* rows_out) {
  const SKey key((int)a_t, (int)y_t, m, n, lda, s * 64 + gamma);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_loaded) load_file();
  auto it = g_sketch.find(key);
  if (it != g_sketch.end()) {
    *rows_out = it->second;
    return hipSuccess;
  }
  const double scale = 1.0 / std::sqrt((double)gamma);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int best = 0;
  float best_ms = 0.0f;
  for (int R = 2; R <= 32 && e == hipSuccess; R *= 2) {
    // candidates the kernel instantiates for this storage type and sketch size
    e = launch_sketch_apply(st, A, a_t, m, n, lda, s, L, scale, Y, y_t, ldy, R);  // warm-up
    if (e == hipErrorInvalidValue) {
      e = hipSuccess;
      (void)hipGetLastError();
      continue;
    }
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch_sketch_apply(st, A, a_t, m, n, lda, s, L, scale, Y, y_t, ldy, R);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && (best == 0 || ms < best_ms)) {
      best = R;
      best_ms = ms;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  g_sketch[key] = best;
  if (const char* path = cache_path()) {
    if (FILE* f = fopen(path, "a")) {
      fprintf(f,
              "{\"kernel\": \"sketch_apply\", \"dtype\": %d, \"y_dtype\": %d, \"m\": %lld, \"n\": %lld, "
              "\"lda\": %lld, \"s\": %lld, \"gamma\": %d, \"rows_per_block\": %d, \"ms\": %.6f}\n",
              (int)a_t, (int)y_t, (long long)m, (long long)n, (long long)lda, (long long)s, gamma, best, best_ms);
      fclose(f);
    }
  }
  *rows_out = best;
  return hipSuccess;
}
