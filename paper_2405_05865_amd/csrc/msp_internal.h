// Internal declarations shared by the HIP translation units of libmsp.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "msp.h"

#define MSP_CHECK_HIP(expr)                                                        \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) return msp_fail_hip(_e, #expr, __FILE__, __LINE__);      \
  } while (0)

msp_status msp_fail(msp_status st, const char* fmt, ...);
msp_status msp_fail_hip(hipError_t e, const char* what, const char* file, int line);

// ---------------------------------------------------------------------------------
// Workspace carving: 256-byte aligned bump allocator over a caller-owned buffer.
// ---------------------------------------------------------------------------------
struct WsCarver {
  char* base;
  size_t cap;
  size_t off = 0;
  bool dry;  // size query only
  WsCarver(void* b, size_t c) : base((char*)b), cap(c), dry(b == nullptr) {}
  template <class T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T* p = dry ? nullptr : (T*)(base + off);
    off += bytes;
    return p;
  }
  bool ok() const { return dry || off <= cap; }
};

// ---------------------------------------------------------------------------------
// Sketch kernels (k_sketch.hip)
// ---------------------------------------------------------------------------------
// Bucket lists of a sparse embedding: for each sketch row j, the (column, sign)
// entries with S[j, col] != 0 in increasing column order. Entry = (col << 1) | neg.
struct BucketLists {
  int32_t* offsets;  // [rows + 1]
  int32_t* entries;  // [n * gamma]
};
size_t bucket_scratch_bytes(int64_t n, int64_t rows, int32_t gamma);
hipError_t launch_sketch_gen(hipStream_t st, uint64_t seed, int64_t n, int64_t s, int32_t gamma,
                             int32_t* rows, int8_t* signs);
hipError_t build_buckets(hipStream_t st, const int32_t* rows, const int8_t* signs, int64_t n, int64_t nrows,
                         int32_t gamma, BucketLists out, void* scratch);
// Tile-major lists of S for Y = A S^T: the columns of A in tiles of wc (sketch_tile_width:
// wc * gamma <= 1024); for tile t and sketch row j, toff[t * (s + 1) + j] .. [.. + j + 1] index
// tent entries (column within the tile << 1) | neg, columns increasing.
struct TileLists {
  int32_t* toff;
  int32_t* tent;
  int wc;
  int ntiles;
};
int sketch_tile_width(int32_t gamma);
size_t tile_lists_ints(int64_t n, int64_t s, int32_t gamma);
TileLists carve_tile_lists(int32_t* base, int64_t n, int64_t s, int32_t gamma);
hipError_t build_tile_lists(hipStream_t st, const int32_t* rows, const int8_t* signs, int64_t n, int64_t s,
                            int32_t gamma, TileLists L);
// Y = A S^T with scale 1/sqrt(gamma): Y[r, j] = scale * sum_{entries of bucket j} sign * A[r, col],
// in column order; R = rows of A per block (0: built-in rule; the autotuner's choice otherwise)
hipError_t launch_sketch_apply(hipStream_t st, const void* A, msp_dtype a_t, int64_t m, int64_t n, int64_t lda,
                               int64_t s, TileLists L, double scale, void* Y, msp_dtype y_t, int64_t ldy, int R);
// N Gaussian probes of length n (probe j at G + j * ldg) from seed: Box-Muller over the
// counter-based SplitMix64 stream (msp_gaussian_probes)
hipError_t launch_probes(hipStream_t st, uint64_t seed, int64_t n, int64_t N, double* G, int64_t ldg);
// out[j, :] = scale * sum_{entries of bucket j} sign * X[col, :]   (out is F64, nrows x ncols)
hipError_t launch_gather_rows(hipStream_t st, const void* X, msp_dtype x_t, int64_t ldx, int64_t ncols,
                              int64_t nrows, BucketLists b, double scale, double* out, int64_t ldo);

// ---------------------------------------------------------------------------------
// Small dense FP64 kernels (k_dense.hip)
// ---------------------------------------------------------------------------------
// G = X^T X (X: rows x s row-major, F64), full symmetric result; the row range is split
// `splits` ways (part: splits*s*s doubles when splits > 1) and summed in fixed order.
int gram_splits(int64_t rows, int64_t s);
hipError_t launch_gram(hipStream_t st, const double* X, int64_t rows, int64_t s, int64_t ldx, double* G,
                       double* part, int splits);
// the same for an F32-stored X (FP64 arithmetic)
hipError_t launch_gram_f32(hipStream_t st, const float* X, int64_t rows, int64_t s, int64_t ldx, double* G,
                           double* part, int splits);
// out = sym(a*P + b*Q) + c*I  (P, Q may alias out; Q may be null)
hipError_t launch_combine_sym(hipStream_t st, int64_t s, double a, const double* P, double b, const double* Q,
                              double c, double* out);
hipError_t launch_symmetrize(hipStream_t st, int64_t s, double* Wm);
// trace(M) -> *out (device scalar)
hipError_t launch_trace(hipStream_t st, int64_t s, const double* M, double* out);
// *out = sum_i A[i, i] in FP64 for an F64, F32 or BF16 matrix (device scalar)
hipError_t launch_diag_sum(hipStream_t st, const void* A, msp_dtype t, int64_t n, int64_t lda, double* out);
// lam0 estimate from the trace deficit of the Nystrom approximation: with scal[0] = tr A,
// scal[1] <- <Winv, C^T C>_F = tr(Winv C^T C) and scal[2] <- (2/l) max(scal[0] - scal[1], 0)
hipError_t launch_lambda0_est(hipStream_t st, const double* Winv, const double* CtC, int64_t s, double l,
                              double* scal);
// In-place inverse of SPD M (s x s) by Gauss-Jordan sweeps, shifted by
// mu = shift_rel * trace / s; tmp: s*s doubles; status: device int (0 ok, 1 not PD).
// Result lands in M.
hipError_t spd_inverse(hipStream_t st, int64_t s, double* M, double* tmp, double shift_rel,
                       double* scal /*2 doubles*/, int32_t* status);

// ---------------------------------------------------------------------------------
// Sweep kernels (k_sweep.hip)
// ---------------------------------------------------------------------------------
// Y[:, j] = A X[:, j] + lam * X[:, j] (lam applied only if diag_shift) for j < k.
// `skip` (device, per column; may be null): columns with skip[j] != 0 are left alone.
// If dot_part != null, each block writes sum_r X[r,j] * Y[r,j] into dot_part[block*k + j]
// and the number of blocks is returned in *nblocks (host).
hipError_t launch_gemv(hipStream_t st, const void* A, msp_dtype a_t, int64_t rows, int64_t cols, int64_t lda,
                       const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k, double lam,
                       bool diag_shift, const int32_t* skip, double* dot_part, int* nblocks);
// the same with FP64 arithmetic on an FP32-stored A
hipError_t launch_gemv_f32_as_f64(hipStream_t st, const float* A, int64_t rows, int64_t cols, int64_t lda,
                                  const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k, double lam,
                                  bool diag_shift, const int32_t* skip, double* dot_part, int* nblocks);
// Blocks of k >= kGemmMinK vectors take the matrix-core block sweep (k_gemm.hip) with the
// same contract; its dot partials come per 64-row set (gemm_row_sets(rows) of them).
constexpr int64_t kGemmMinK = 8;
int gemm_row_sets(int64_t rows);
hipError_t launch_gemm(hipStream_t st, const void* A, msp_dtype a_t, bool fp64_arith, int64_t rows, int64_t cols,
                       int64_t lda, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k, double lam,
                       bool diag, const int32_t* skip, double* dot_part, int* nblocks);
// y = (A + lam I) x (lam only if diag_shift) for symmetric A from its lower triangle
// (k_symv.hip), one vector; part: symv_part_doubles(n); dot_part: one <x, y> partial per
// reduction block (count in *nblocks). Needs 16-byte aligned A and lda (symv_supported).
size_t symv_part_doubles(int64_t n);
bool symv_supported(const void* A, msp_dtype t, int64_t lda, int64_t k);
hipError_t launch_symv(hipStream_t st, const void* A, msp_dtype a_t, int64_t n, int64_t lda, const double* x,
                       double* y, double lam, bool diag_shift, const int32_t* skip, double* part, double* dot_part,
                       int* nblocks);
// the same with a scratch of segment partials (k_gemm splits the reduction range when the
// launch would have too few wavefronts; gemm_split_doubles(rows, k) allows up to 16
// segments)
size_t gemm_split_doubles(int64_t rows, int64_t k);
// nseg > 0 forces that many segments (the autotuner's choice; it must fit the scratch,
// nseg * k * rows doubles, or the built-in rule is used); 0 = built-in rule
hipError_t launch_gemm_split(hipStream_t st, const void* A, msp_dtype a_t, bool fp64_arith, int64_t rows,
                             int64_t cols, int64_t lda, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k,
                             double lam, bool diag, const int32_t* skip, double* dot_part, int* nblocks,
                             double* scratch, size_t scratch_doubles, int nseg);
// the segment count the built-in rule picks for that launch
int gemm_split_default(int64_t rows, int64_t cols, int64_t k, msp_dtype a_t, bool fp64_arith,
                       size_t scratch_doubles);
// autotuner of the level-1 block sweep (msp_tune.hip): times every admissible segment
// count of launch_gemm_split on this matrix (Y is overwritten) and returns the fastest,
// cached per (dtype, arithmetic, rows, cols, lda, k) for the process and, when the
// environment names a file in MSP_TUNE_CACHE, across processes (JSON lines)
hipError_t tune_block_sweep(hipStream_t st, const void* A, msp_dtype a_t, bool fp64_arith, int64_t rows,
                            int64_t cols, int64_t lda, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k,
                            double* scratch, size_t scratch_doubles, int* nseg_out);
// autotuner of the sparse sketch (msp_tune.hip): rows of A per block, timed for every
// admissible value on this matrix (Y is overwritten) and cached per shape;
// sketch_rows_choice returns the cached value or 0 (built-in rule)
hipError_t tune_sketch_apply(hipStream_t st, const void* A, msp_dtype a_t, int64_t m, int64_t n, int64_t lda,
                             int64_t s, int32_t gamma, const TileLists& L, void* Y, msp_dtype y_t, int64_t ldy,
                             int* rows_out);
int sketch_rows_choice(msp_dtype a_t, int64_t m, int64_t n, int64_t lda, int64_t s, int32_t gamma);
// Y[:, j] = M X[:, j] for an FP64 row-major M (ld = cols) with few rows: the same
// matrix-core product, its reduction range cut into segments of at least min_seg columns
// until about 2048 wavefronts run (scratch of at least gemm_split_doubles(rows, k)
// doubles). The level-1 sweep keeps min_seg = 1024 (long streams from HBM); the s x s
// inner operators, which stay in cache, take 64; the s x n level-2 factor takes 256.
// With defer_sum and more than one segment the segment partials stay in the scratch
// (layout [segment][column][row], *nseg_out segments) for the consumer to add in order.
hipError_t launch_gemm_seg(hipStream_t st, const double* M, int64_t rows, int64_t cols, const double* X,
                           int64_t ldx, double* Y, int64_t ldy, int64_t k, const int32_t* skip, double* scratch,
                           size_t scratch_doubles, int min_seg, int* nseg_out = nullptr, bool defer_sum = false);
constexpr int kSegSmall = 64;
constexpr int kSegWide = 256;
// Y[:, j] = A^T X[:, j] on the matrix cores for k >= kGemmMinK (same contract as
// launch_gemv_t; part: gemv_t_part_doubles(rows, cols, k) doubles)
size_t gemm_t_part_doubles(int64_t rows, int64_t cols, int64_t k);  // its split partials
hipError_t launch_gemm_t(hipStream_t st, const void* A, msp_dtype a_t, int64_t rows, int64_t cols, int64_t lda,
                         const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k, const int32_t* skip,
                         double* part);
// Y[:, j] = A^T X[:, j]  (A rows x cols row-major; X length rows; Y length cols)
// part: scratch of gemv_t_part_doubles(rows, cols, k) doubles
size_t gemv_t_part_doubles(int64_t rows, int64_t cols, int64_t k);
hipError_t launch_gemv_t(hipStream_t st, const void* A, msp_dtype a_t, int64_t rows, int64_t cols, int64_t lda,
                         const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k, const int32_t* skip,
                         double* part);
// both transposed products with FP64 arithmetic on an FP32-stored A (same contracts)
hipError_t launch_gemm_t_f32_as_f64(hipStream_t st, const float* A, int64_t rows, int64_t cols, int64_t lda,
                                    const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k,
                                    const int32_t* skip, double* part);
hipError_t launch_gemv_t_f32_as_f64(hipStream_t st, const float* A, int64_t rows, int64_t cols, int64_t lda,
                                    const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t k,
                                    const int32_t* skip, double* part);

// ---------------------------------------------------------------------------------
// Tall-skinny kernels on Y (n x s) and reductions (k_tall.hip)
// ---------------------------------------------------------------------------------
int tall_blocks(int64_t rows);
// part[blk][j][c] = sum_{rows r of blk} Y[r, c] * V[r, j]   (Y^T V partials), V n x k (ld ldv)
hipError_t launch_yt_v(hipStream_t st, const void* Y, msp_dtype y_t, int64_t n, int64_t s, int64_t ldy,
                       const double* V, int64_t ldv, int64_t k, const int32_t* skip, double* part);
// part[blk][j][c] = sum_r Y[r, c] * (Y[r, :] . Z[:, j])       (Y^T Y Z partials), Z s x k (ld s)
hipError_t launch_yty_z(hipStream_t st, const void* Y, msp_dtype y_t, int64_t n, int64_t s, int64_t ldy,
                        const double* Z, int64_t k, const int32_t* skip, double* part);
// out[:, j] = (a * V[:, j] + b * Y Z[:, j]) for j < k (Z s x k, ld s); out n x k (ld ldo)
hipError_t launch_y_z(hipStream_t st, const void* Y, msp_dtype y_t, int64_t n, int64_t s, int64_t ldy,
                      const double* Z, int64_t k, double a, const double* V, int64_t ldv, double b,
                      const int32_t* skip, double* out, int64_t ldo);
// out[j][c] = sum_b part[b][j][c]  (fixed order)
hipError_t launch_reduce_parts(hipStream_t st, const double* part, int nparts, int64_t len, double* out);
// out[i, j] = sum_c M[i, c] * V[c, j] for s x s M (row-major), V s x k (ld s)
hipError_t launch_small_mv(hipStream_t st, int64_t s, const double* M, const double* V, int64_t k,
                           const int32_t* skip, double* out);

// ---------------------------------------------------------------------------------
// Flexible-PCG state machine kernels (k_fcg.hip). A level works on k columns of
// vectors of length len stored contiguously (column j at ptr + j*len). Per-column
// scalars live in device arrays; reductions use per-block partials summed in fixed
// block order by the last block to finish (deterministic).
// done[j]: 0 active, 1 converged (recurrence), 2 breakdown, 3 iteration cap,
//          4 converged and confirmed on the recomputed residual.
// ---------------------------------------------------------------------------------
struct FcgState {
  double* rz;
  double* alpha;
  double* beta;
  double* bnorm;
  double* rnorm;
  int32_t* done;
  int32_t* iters;
  int32_t* active;   // [1]
  int32_t* counter;  // [1] last-block ticket (reset by the last block)
  double* part;      // per-block partials, >= fcg_part_doubles(len, k)
  int32_t* brk;      // [k] breakdown marker written by block 0 of each column
  int32_t* done_next;   // [k] decision taken inside a multi-block kernel, committed by the next
  int32_t* iters_next;  // [k] single-block kernel (so no block reads a value another block rewrites)
  int64_t k;
};
size_t fcg_part_doubles(int64_t len, int64_t k);
FcgState carve_fcg_state(WsCarver& w, int64_t len, int64_t k);
// r = b, x = 0, bnorm; done = parent_done || |b| == 0; mirror <- active count
hipError_t fcg_init(hipStream_t st, FcgState S, int64_t len, const double* b, int64_t ldb, double* r, double* x,
                    const int32_t* parent_done, int32_t* mirror);
// p = z, rz = <r, z>   (columns not done)
hipError_t fcg_first_dir(hipStream_t st, FcgState S, int64_t len, const double* r, const double* z, double* p);
// alpha = rz / pq with pq = sum of nparts per-block partials (layout part[b*k + j])
hipError_t fcg_alpha_parts(hipStream_t st, FcgState S, const double* pq_part, int nparts);
// alpha = rz / <p, q> computed directly (short vectors)
hipError_t fcg_alpha_dot(hipStream_t st, FcgState S, int64_t len, const double* p, const double* q);
// x += alpha p; r_old = r; r -= alpha q; |r| -> done by tol / max_iter; mirror <- active.
// With pq_part (nparts per-block partials of <p, q>, layout [b][k]) every block forms
// alpha = rz / <p, q> itself; otherwise alpha is read from S.alpha.
hipError_t fcg_update(hipStream_t st, FcgState S, int64_t len, double* x, double* r, double* r_old,
                      const double* p, const double* q, double tol, int32_t max_iter, int32_t* mirror,
                      const double* pq_part = nullptr, int nparts = 0);
hipError_t fcg_update_nodecide(hipStream_t st, FcgState S, int64_t len, double* x, double* r, double* r_old,
                               const double* p, const double* q);
// rho -= alpha t with the stop decision on |rho| (A x = b through the normal equations)
hipError_t fcg_rho_update(hipStream_t st, FcgState S, int64_t len, double* rho, const double* t, double tol,
                          int32_t max_iter, int32_t* mirror);
// S.done = src (or 0 when src is null)
hipError_t fcg_copy_done(hipStream_t st, FcgState S, const int32_t* src);
// beta = <z, r - r_old> / rz ; rz = <r, z> ; p = z + beta p
hipError_t fcg_direction(hipStream_t st, FcgState S, int64_t len, const double* r, const double* r_old,
                         const double* z, double* p);
// confirmation on rtrue = b - op(x) for columns with done == 1: done -> 4 if |rtrue| <= tol |b|,
// else r = rtrue, done -> 0 (restart). relres[j] (device) receives |rtrue| / |b|; mirror <- active
hipError_t fcg_confirm(hipStream_t st, FcgState S, int64_t len, const double* rtrue, double* r, double tol,
                       double* relres, int32_t* mirror);
// out = a*x + b*y on len x k blocks (each with its own ld); skip columns flagged in skip
hipError_t launch_axpby(hipStream_t st, int64_t len, int64_t k, double a, const double* x, int64_t ldx, double b,
                        const double* y, int64_t ldy, double* out, int64_t ldo, const int32_t* skip);
// dev_out[j] = <x_j, y_j>
hipError_t launch_coldots(hipStream_t st, int64_t len, int64_t k, const double* x, int64_t ldx, const double* y,
                          int64_t ldy, double* dev_out);
// dA = -dB X^T (n x n dense, ld ldda)
hipError_t launch_outer_neg(hipStream_t st, int64_t n, int64_t k, const double* dB, int64_t lddb, const double* X,
                            int64_t ldx, double* dA, int64_t ldda);
// out[0] = max_i sum_j |A[i, j]| for an F64 or F32 matrix (device scalar): a grid of blocks
// (at most part_doubles, each writing its maximum to part) and a one-block maximum
hipError_t launch_row_abs_max(hipStream_t st, const void* A, msp_dtype t, int64_t rows, int64_t cols, int64_t lda,
                              double* part, int64_t part_doubles, double* out);
// out (cols x rows, FP64, ld ldo) = transpose of X (rows x cols, F64 or F32, ld ldx)
hipError_t launch_transpose_f64(hipStream_t st, const void* X, msp_dtype x_t, int64_t rows, int64_t cols,
                                int64_t ldx, double* out, int64_t ldo);
// copy len x k block between leading dimensions
hipError_t launch_copy_block(hipStream_t st, int64_t len, int64_t k, const double* x, int64_t ldx, double* y,
                             int64_t ldy);

// ---------------------------------------------------------------------------------
// Fused inner-iteration kernels on the sketch Y (k_level2.hip): one flexible-PCG step
// for q = Y^T Y p + wscale W p + sigma p with preconditioner Minv. Vectors are s x k.
// ---------------------------------------------------------------------------------
struct L2Step {
  int64_t s = 0, k = 0;
  int nbC = 0;                 // blocks of the Y pass (l2_blocks(n))
  double* part = nullptr;      // [nbC][k][s]
  double* pqpart = nullptr;    // [nbC][k]
  double* wp = nullptr;        // [k][s] (null without W)
  double* pqw = nullptr;       // [k][s] (null without W)
  double wscale = 0.0, sigma = 0.0;
  double *y = nullptr, *r = nullptr, *ro = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  const double* Minv = nullptr;
  FcgState S{};
  double* bpart = nullptr;     // l2_bpart_doubles(s, k)
  double tol = 0.0;
  int max_iter = 0;
  int32_t* mirror = nullptr;
  const int32_t* parent_done = nullptr;
  const double* rhs = nullptr; // l2_init: right-hand side given directly (s x k), else Y^T v partials
  // with k >= kGemmMinK: z = Minv r (and an explicit operator's M p) as matrix-core block
  // products through this scratch (gemm_split_doubles(s, k) doubles or more)
  double* gscratch = nullptr;
  size_t gscratch_n = 0;
};
int l2_blocks(int64_t n);
size_t l2_bpart_doubles(int64_t s, int64_t k);
// sizes of the Y-pass partial buffers (block partials, group sums and group counters);
// the counters must be zero before the first pass (l2_op_counters)
size_t l2_op_part_doubles(int64_t n, int64_t s, int64_t k);
size_t l2_op_pq_doubles(int64_t n, int64_t k);
// Y pass: rhs_mode=false: partials of Y^T Y v (v: s x k) and <v, Y^T Y v>, plus W v rows;
//         rhs_mode=true : partials of Y^T v (v: n x k, ld ldv) for the right-hand side.
hipError_t l2_op(hipStream_t st, const void* Y, msp_dtype y_t, int64_t n, int64_t s, int64_t ldy, const double* v,
                 int64_t ldv, int64_t k, const int32_t* done, double* part, double* pqpart, const double* W,
                 double* wp, double* pqw, bool rhs_mode);
// the same step input from an explicit s x s operator M (steps then run with nbC = 0 and
// wscale = 1): wp = M p, pqw = p .* (M p). With a scratch and k >= kGemmMinK, wp comes
// from launch_gemm_seg and pqw is not written (the step then takes <p, M p> from wp
// and must run with pqw = null)
hipError_t l2_op_matrix(hipStream_t st, const double* M, int64_t s, const double* v, int64_t k, const int32_t* done,
                        double* wp, double* pqw, double* scratch, size_t scratch_n);
// right-hand side (after l2_op in rhs mode): y = 0, r = rhs, |rhs|, z = Minv r, p = z
hipError_t l2_init(hipStream_t st, const L2Step& a);
// the first kernel of l2_init alone: y = 0, r = rhs (0 where parent_done)
hipError_t l2_rhs(hipStream_t st, const L2Step& a);
// one step after l2_op(p): alpha, y/r update, convergence decision, z = Minv r, p = z + beta p
// publish = false skips the host mirror of the active count for more than 16 columns (the
// caller publishes with the last step before it reads the mirror)
hipError_t l2_step(hipStream_t st, const L2Step& a, bool publish = true);
// out[j][c] = sum of the group partials of the last rhs-mode l2_op (Y^T v), s x k
hipError_t l2_reduce_to(hipStream_t st, const L2Step& a, double* out, const int32_t* skip);

// ---------------------------------------------------------------------------------
// Inner iterations with an explicit operator H and preconditioner Minv, one kernel per
// step (k_l2x.hip). G = H Minv (row-major s x s). Vectors are [k][s]; arrays indexed
// [2] alternate by step parity. The right-hand side goes into r[0] and y must be zero
// before l2x_start; the solution accumulates in y.
// ---------------------------------------------------------------------------------
constexpr int kL2xMaxS = 2048;
constexpr int kL2xMaxK = 16;
struct L2xArgs {
  int s, k;
  const double* Minv;
  const double* G;
  double *r[2], *z[2], *g[2], *p[2], *u[2];
  double* y;
  double *rz[2], *al[2];
  double* bn;
  int32_t *done[2], *it[2];
  double tol;
  int max_iter;
  int32_t* mirror;               // [2] host-mapped: active columns, largest iteration count
  const int32_t* parent_done;    // columns already finished one level up (or null)
};
size_t l2x_doubles(int64_t s, int64_t k);
L2xArgs l2x_carve(WsCarver& w, int64_t s, int64_t k);
// |b|, the first decision, z_0 = Minv r_0 and g_0 = G r_0
hipError_t l2x_start(hipStream_t st, const L2xArgs& a);
// one step reading parity par; first = 1 for the step after l2x_start (par 0)
hipError_t l2x_step(hipStream_t st, const L2xArgs& a, int par, int first);
// host mirror (active columns, largest iteration count) of the state at parity par, for
// k > 1 (with one column the step and start kernels publish it themselves)
hipError_t l2x_publish(hipStream_t st, const L2xArgs& a, int par);

// ---------------------------------------------------------------------------------
// Inner iterations with an explicit operator H (+ sigma I) and preconditioner Minv by
// direct products, two kernels per step (k_l2f.hip): the level-3 solves of the general
// path (s <= kL2fMaxS). The state after l2_init (y = 0, r_0, z_0 = Minv r_0, p_0 = z_0, S.rz, S.done,
// S.bnorm, S.iters = 0) is the input: r[0] = that r, p[0] = that p; r[1] and p[1] alternate
// with them by step parity. The solution accumulates in y; z and q exist only as the sums of
// their column-segment partials.
// ---------------------------------------------------------------------------------
constexpr int kL2fMaxK = 16;
constexpr int kL2fMaxS = 2048;
constexpr int kL2fRows = 8;     // wavefronts per block
constexpr int kL2fSegW = 512;       // operator columns per block
constexpr int kL2fSegWSmall = 128;  // the same for s <= kL2fSegW (more blocks)
struct L2fArgs {
  int s, k, nb;
  int nseg, rpw, segw;  // column segments of segw columns; rows per wavefront (l2f_shape)
  const double* H;
  const double* Minv;
  double sigma;
  FcgState S;
  double* y;
  double *r[2], *p[2];
  double *rz[2];
  double* alpha;
  double* ppart;   // [nb][k]     <p, q> partials
  double* dpart;   // [nb][k][3]  <z, r_new>, <z, r_old>, |r_new|^2 partials
  double* qpart;   // [nseg][k][s] (H + sigma I) p by column segment (sigma p in segment 0)
  double* zpart;   // [nseg][k][s] Minv r by column segment
  int32_t *done[2], *iters[2];
  int32_t* brk;
  double tol;
  int max_iter;
  int32_t* mirror;  // [2] host-mapped: active columns, largest iteration count
};
// the launch shape for s: column segments, rows per wavefront, blocks (row blocks x
// segments), segment width
void l2f_shape(int64_t s, int* nseg, int* rpw, int* nb, int* segw);
// carves p[1], rz, alpha, the partials and the int state; the caller sets the rest
L2fArgs l2f_carve(WsCarver& w, int64_t s, int64_t k);
// step t: decision on the previous step (fresh = 1 for t = 0: the l2_init state), p_t,
// q_t = (H + sigma I) p_t and <p_t, q_t> partials; publishes the host mirror
hipError_t l2f_op(hipStream_t st, const L2fArgs& a, int t, int fresh);
// step t: alpha_t, y, r_{t+1}, z_{t+1} = Minv r_{t+1} and the dot partials
hipError_t l2f_prec(hipStream_t st, const L2fArgs& a, int t);

// ---------------------------------------------------------------------------------
// The preconditioner handle
// ---------------------------------------------------------------------------------
struct msp_precond {
  msp_structure structure;
  int64_t m, n, s, phi;
  int32_t gamma, phi_gamma;
  const int32_t* S_rows;
  const int8_t* S_signs;
  const void* Y;      // C (PSD) or A-tilde (general), m x s
  msp_dtype y_t;
  int64_t ldy;
  double lam, lam0, lt;
  double trace_a = 0.0, trace_nys = 0.0;  // lam0 estimated: tr A and tr(W^+ C^T C)
  double shift_rel;
  // device data carved from the nystrom workspace
  double* Wm;         // PSD: W = S C (symmetrised)
  double* G;          // PSD: C~^T C~ ; general: A^^T A^ (M3a)
  double* Minv;       // PSD: M2^{-1} ; general: M3a^{-1}
  double* Minv2;      // general: M3b^{-1}
  double* tmp;        // s*s scratch for refactoring
  double* scal;       // small device scalars
  int32_t* status;    // device status word
  int32_t* host_flags;  // pinned, mapped host memory (mirrors of device counters)
  int32_t* dev_view_flags;
  double* host_d;     // pinned scratch doubles
  int device;
  void* events;       // pool of hipEvent_t pairs for profiled sweeps (std::vector)
};
