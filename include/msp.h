/*
 * msp.h -- C-ABI of libmsp, a gfx950 (MI355X) implementation of the hot path of
 * Multi-level Sketched Preconditioning (Derezinski, Musco, Yang, "Faster Linear
 * Systems and Matrix Norm Approximation via Multi-level Sketched Preconditioning").
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers unless marked [host].
 *   - Matrices are row-major with an explicit leading dimension (in elements).
 *   - Blocks of k vectors (right-hand sides, solutions, probes) are stored as k
 *     contiguous vectors: vector j starts at ptr + j * ld (ld >= vector length).
 *   - Every call enqueues its device work on `stream` (hipStream_t passed as void*);
 *     calls that fill [host] outputs synchronise the stream before returning.
 *   - The caller owns all device memory, including the workspaces whose sizes the
 *     *_workspace queries return; the library never allocates device memory, apart
 *     from the fixed static scratch of msp_sketch_noalloc. On the host, msp_nystrom
 *     allocates one 4 KiB page of pinned, device-mapped memory per handle (the mirror
 *     through which solves read convergence flags), solves with profile != 0 create HIP
 *     events (kept in the handle), and solves with use_graph != 0 create a capture stream
 *     and graphs (freed at return); msp_precond_destroy frees the rest.
 *   - Errors: every call returns an msp_status; no call throws or aborts.
 *     Arguments are validated before any device work is enqueued. msp_last_error()
 *     returns a thread-local message describing the last failure.
 *   - Determinism: identical inputs, seeds and device give bitwise-identical results
 *     (all reductions run in a fixed order; no floating-point atomics).
 */
#ifndef MSP_H
#define MSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MSP_OK = 0,
  MSP_ERR_INVALID_ARG = 1,   /* bad size, pointer, dtype or parameter */
  MSP_ERR_NOT_POSDEF = 2,    /* a pivot of an SPD inverse was <= 0 */
  MSP_ERR_BREAKDOWN = 3,     /* p^T A p <= 0 in a Krylov iteration */
  MSP_ERR_NO_CONVERGENCE = 4,/* iteration cap reached; best iterate returned */
  MSP_ERR_NONFINITE = 5,     /* NaN/Inf in an input scalar or a residual */
  MSP_ERR_WORKSPACE = 6,     /* workspace too small or misaligned */
  MSP_ERR_UNSUPPORTED = 7,   /* valid request outside what the library implements */
  MSP_ERR_HIP = 8            /* a HIP runtime call failed */
} msp_status;

typedef enum { MSP_F64 = 0, MSP_F32 = 1, MSP_BF16 = 2 } msp_dtype;

typedef enum {
  MSP_SYM_PSD = 0,  /* (A + lam I) x = b with A symmetric PSD: Algorithms 1-2 (two levels) */
  MSP_GENERAL = 1   /* (A^T A + lam I) x = c, or A x = b via c = A^T b: Algorithms 3-5 */
} msp_structure;

/* Opaque preconditioner handle (host memory). Its device data lives in the caller's
 * sketch output Y and nystrom workspace, which must outlive the handle. */
typedef struct msp_precond msp_precond;

/* ---------------------------------------------------------------------------------
 * msp_sketch -- sketch generation and the sparse sketch of A.
 *
 * Definition 2.1 (sparse embedding matrix): S in R^{s x n}; column i of S holds
 * +-1/sqrt(gamma) in gamma distinct rows chosen uniformly without replacement, with
 * independent signs. Algorithm 1 (PSD) and Algorithm 3 (general) form
 * Y = A S^T (the paper's C, resp. A-tilde), one pass over A.
 *
 * The index draw is counter-based SplitMix64: column key k_i = fmix(seed + (i+1)G),
 * draw a >= 0 u = fmix(k_i + (a+1)G) with G = 0x9E3779B97F4A7C15; candidate row
 * floor(hi32(u) s / 2^32), sign -1 iff bit 0 of u is set; the first gamma distinct
 * candidates are kept in draw order.
 *
 *   A        m x n, row-major, leading dim lda >= n, dtype a_t (F64 | F32 | BF16)
 *   s, gamma sketch rows and nonzeros per column, 1 <= gamma <= s <= n
 *   S_rows   out, int32 [n][gamma]     S_signs  out, int8 [n][gamma] (+1 / -1)
 *   Y        out, m x s row-major, leading dim ldy >= s, dtype y_t (F64 | F32);
 *            F64 Y requires F64 A. Sums run in y_t precision.
 *   ws       device workspace of at least msp_sketch_workspace(...) bytes, 256-B aligned
 * Asynchronous: returns after enqueueing.
 * ------------------------------------------------------------------------------ */
msp_status msp_sketch_workspace(int64_t m, int64_t n, int64_t s, int32_t gamma, size_t* bytes /*host*/);
msp_status msp_sketch(void* stream, const void* A, msp_dtype a_t, int64_t m, int64_t n, int64_t lda,
                      int64_t s, int32_t gamma, uint64_t seed,
                      int32_t* S_rows, int8_t* S_signs, void* Y, msp_dtype y_t, int64_t ldy,
                      void* ws, size_t ws_bytes);

/* msp_sketch_autotune -- msp_sketch that first times every admissible number of rows of A
 * per block of the sketch kernel (the shape of its register tile) on this matrix, keeps the
 * fastest for this (A dtype, Y dtype, m, n, lda, s, gamma) for the process (and in the file
 * named by MSP_TUNE_CACHE, one JSON object per line), and writes S and Y with it; later
 * msp_sketch calls with that shape use it. Same arguments and outputs as msp_sketch, plus
 *   rows_per_block [host] out (may be NULL): the chosen value.
 * Synchronises the stream. */
msp_status msp_sketch_autotune(void* stream, const void* A, msp_dtype a_t, int64_t m, int64_t n, int64_t lda,
                               int64_t s, int32_t gamma, uint64_t seed, int32_t* S_rows, int8_t* S_signs,
                               void* Y, msp_dtype y_t, int64_t ldy, void* ws, size_t ws_bytes,
                               int32_t* rows_per_block /*host*/);

/* ---------------------------------------------------------------------------------
 * msp_sketch_noalloc -- msp_sketch without a workspace, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation. Same arguments, kernels, results (bit for bit) and asynchrony as msp_sketch,
 * minus ws / ws_bytes; calls no allocating routine and no memset.
 *
 * The sketch's scratch (bucket lists and sort counts, msp_sketch_workspace bytes) lives in
 * a static device array of MSP_NOALLOC_SCRATCH_BYTES that each GPU the library runs on
 * holds until the process ends; its device address is looked up on the first call on
 * each device. A sketch whose msp_sketch_workspace exceeds that size returns
 * MSP_ERR_WORKSPACE before any device work. Every call on one GPU shares the array, so
 * calls that overlap on one GPU (different streams or threads without ordering) race.
 * ------------------------------------------------------------------------------ */
#define MSP_NOALLOC_SCRATCH_BYTES (16u << 20)
msp_status msp_sketch_noalloc(void* stream, const void* A, msp_dtype a_t, int64_t m, int64_t n, int64_t lda,
                              int64_t s, int32_t gamma, uint64_t seed, int32_t* S_rows, int8_t* S_signs, void* Y,
                              msp_dtype y_t, int64_t ldy);

/* ---------------------------------------------------------------------------------
 * msp_nystrom -- the Nystrom factor and the inner-level preconditioners.
 *
 * MSP_SYM_PSD (Algorithm 1; Section 4): lam~ = lam + lam0, W = S C
 *   (symmetrised), C~ = Phi C with Phi a second sparse embedding (phi rows,
 *   phi_gamma nonzeros per column, seed phi_seed), M2 = C~^T C~ + lam~ W, and the
 *   explicit inverse M2^{-1} that Algorithm 1 precomputes.
 * MSP_GENERAL (Algorithm 3; Section 5): A^ = Phi A~ (Phi over the m rows),
 *   M3a = A^^T A^, M3b = M3a + lam~ I and their explicit inverses.
 * Every inverse is of (M + mu I), mu = 1e-12 tr(M)/s, by Gauss-Jordan elimination
 * without pivoting (valid for SPD M: each pivot is a positive Schur-complement
 * diagonal; a pivot <= 0 returns MSP_ERR_NOT_POSDEF).
 *
 *   m, n, s, gamma, S_rows, S_signs, Y, y_t, ldy   as produced by msp_sketch
 *            (MSP_SYM_PSD needs m == n)
 *   A, a_t, lda  the matrix Y was sketched from; read only when lambda0 < 0 (its diagonal),
 *            may be NULL otherwise
 *   lambda   regulariser lam >= 0 of the user's system
 *   lambda0  lam0 of Theorems 3.1/4.1 (the paper's value is (2/l) sum_{i>l} lambda_i, an
 *            explicit input as in the algorithms' input lists), lam + lam0 > 0; or, for
 *            MSP_SYM_PSD, any value < 0 to estimate it on the GPU when the tail spectrum is
 *            unknown: lam0 = (2/l) max(tr A - tr(W^+ C^T C), 0) with l = s/2, the trace
 *            deficit of the Nystrom approximation C W^+ C^T (at least sum_{i>s} lambda_i,
 *            0 when rank(A) <= s; W^+ taken as (W + mu I)^{-1}, mu = 1e-9 tr(W)/s; a deficit
 *            below 1e-6 tr A counts as the rounding of an exact recovery, 0). The value used is returned
 *            by msp_precond_params. An estimate of 0 with lam = 0 returns
 *            MSP_ERR_INVALID_ARG; MSP_GENERAL with lambda0 < 0 returns MSP_ERR_UNSUPPORTED.
 *   phi, phi_gamma, phi_seed   the level-2/3 embedding, 1 <= phi_gamma <= phi
 *   ws       device workspace of msp_nystrom_workspace(...) bytes; it holds the factors
 *            and must outlive the handle
 *   P        [host] out: the handle; free with msp_precond_destroy
 * Synchronises once (to report MSP_ERR_NOT_POSDEF), twice when estimating lam0.
 * ------------------------------------------------------------------------------ */
msp_status msp_nystrom_workspace(msp_structure structure, int64_t m, int64_t n, int64_t s, int64_t phi,
                                 int32_t phi_gamma, size_t* bytes /*host*/);
msp_status msp_nystrom(void* stream, msp_structure structure, int64_t m, int64_t n, int64_t s, int32_t gamma,
                       const int32_t* S_rows, const int8_t* S_signs, const void* Y, msp_dtype y_t, int64_t ldy,
                       const void* A, msp_dtype a_t, int64_t lda,
                       double lambda, double lambda0, int64_t phi, int32_t phi_gamma, uint64_t phi_seed,
                       void* ws, size_t ws_bytes, msp_precond** P /*host out*/);
msp_status msp_precond_destroy(msp_precond* P);
/* The handle's lam and lam0 (the estimate when msp_nystrom was given lambda0 < 0). Host only. */
msp_status msp_precond_params(const msp_precond* P, double* lambda /*host*/, double* lambda0 /*host*/);
/* Copy the handle's s x s factors into caller buffers (device, s*s doubles each, any may
 * be NULL): W = S C (PSD) and M2^{-1} (PSD) or M3a^{-1} (general), and M3b^{-1}
 * (general). For inspection and tests; asynchronous. */
msp_status msp_precond_factors(void* stream, const msp_precond* P, double* W, double* Minv, double* Minv2);
/* Change lam (and hence lam~ = lam + lam0) of an existing handle. For MSP_GENERAL this
 * refactors M3b = M3a + lam~ I (the nodes of msp_schatten); for MSP_SYM_PSD it refactors M2. */
msp_status msp_precond_set_lambda(void* stream, msp_precond* P, double lambda);

/* ---------------------------------------------------------------------------------
 * msp_solve -- the preconditioned iteration (the level-1 iteration of Algorithm 1 with Algorithm 2;
 * that of Algorithm 3 with Algorithms 4-5).
 *
 * Level 1 is flexible PCG (Polak-Ribiere beta) on (A + lam I) (PSD) or A^T A + lam I
 * (general); with an exact preconditioner it coincides with Algorithm 6 (Section 6).
 * SolveM1 (Algorithms 2/4) runs a level-2 flexible PCG to relative residual inner_tol
 * (at most max_inner steps) and returns (r - C y)/lam~; for MSP_GENERAL its
 * preconditioner SolveM2 (Algorithm 5) runs two level-3 PCGs in the product form
 * W^{-1}((W + lam~ I)^{-1} r), each to level3_tol.
 * Stop: per right-hand side, |b - (A + lam I) x| <= tol |b| (PSD) or |b - A x| <= tol |b|
 * (general, lam == 0 and `normal` == 0) or |c - (A^T A + lam I) x| <= tol |c| (general,
 * `normal` != 0), taken on the recurrence residual and confirmed on the residual
 * recomputed in FP64 from A_hi (restart from it if the confirmation fails).
 *
 * Mixed precision: A_lo (dtype lo_t) is the matrix swept inside MSP with accumulation
 * in FP64 (lo_t F64) or FP32 (lo_t F32/BF16); A_hi (hi_t) is used for the FP64
 * residuals. If refine != 0 and lo_t != F64, the solve runs FP64 iterative refinement:
 * x += MSP_lo(b - (A_hi + lam I) x) with each inner MSP solve to refine_inner_tol;
 * after two steps that fail to halve the residual it switches to Krylov refinement
 * (flexible PCG on A_hi with MSP_lo as preconditioner). A_hi may equal A_lo.
 *
 *   lambda   lam >= 0 of the system solved: (A + lam I) (PSD) or A^T A + lam I (general with
 *            normal != 0; A x = b needs lam = 0). The preconditioner is the handle's, built
 *            for lam~ = lam_P + lam0 (msp_nystrom / msp_precond_set_lambda); with lam != lam_P
 *            it is reused as it is (still symmetric positive definite, so the iteration
 *            converges; the step count grows as lam moves away from lam_P).
 *   B        k right-hand sides (PSD: n each, general: m each), ld ldb, FP64
 *   X        out, k solutions of length n, ld ldx, FP64
 *   info     [host] out, may be NULL
 * Under refinement, max_outer caps the level-1 steps of all inner solves together. A
 * refinement step "stalls" when it fails to halve some unconverged residual; after two
 * stalled steps the PSD path switches to Krylov refinement and the general path tightens
 * refine_inner_tol by 100x (floor 1e-12) once per stall; it stops with
 * MSP_ERR_NO_CONVERGENCE and the best iterate seen when the step after a tightening also
 * stalls, at the floor, or (level2_form 2, no inner level to tighten) at the first stall.
 * Synchronises the stream before returning.
 * ------------------------------------------------------------------------------ */
typedef struct {
  double tol;              /* level-1 relative residual target (default 1e-8) */
  int32_t max_outer;       /* level-1 iteration cap (default 5000) */
  double inner_tol;        /* level-2 relative residual target (default 1e-10) */
  int32_t max_inner;       /* level-2 iteration cap per SolveM1 (default 200) */
  double level3_tol;       /* level-3 relative residual target (default 1e-10) */
  int32_t max_level3;      /* level-3 iteration cap (default 200) */
  int32_t normal;          /* general only: solve (A^T A + lam I) x = B instead of A x = B */
  int32_t refine;          /* FP64 iterative refinement around a low-precision sweep */
  double refine_inner_tol; /* inner MSP target per refinement step (default 1e-4) */
  int32_t max_refine;      /* refinement step cap (default 30) */
  int32_t profile;         /* record HIP events around every level-1 sweep (sweep_ms in info) */
  int32_t level2_form;     /* how the inner operators are applied (default 1):
                              0: through the sketch each inner step (PSD: C^T (C y) + lam~ W y;
                                 general: passes over A~ and two A-sweeps), the paper's cost model;
                              1: through matrices formed once per solve: PSD: the s x s
                                 C^T C + lam~ W (s^2 instead of n s work per inner step);
                                 general: level 2 as B^T (B y) + lam~ A~^T A~ y with the n x s
                                 B = A^T A~ (two passes over B instead of two A-sweeps) and
                                 level 3 through the s x s A~^T A~. The same operators and
                                 iterations. Forming C^T C squares the conditioning of C;
                                 form 0 avoids that for very ill-conditioned A;
                              2: one-level variant: SolveM1 solved exactly through the explicit
                                 inverse of the level-2 matrix of form 1 (the standard Nystrom
                                 preconditioner of Section 2, no level-2/3 iteration; for
                                 comparison with the multi-level method). */
  int32_t sym_sweep;       /* MSP_SYM_PSD, one right-hand side: sweep the level-1 operator from the
                              lower triangle of A_lo only (n(n+1)/2 elements per sweep instead of
                              n^2; A is symmetric by the problem statement). The FP64 confirmation
                              and refinement residuals still use all of A_hi. Default 1. */
  int32_t use_graph;       /* level2_form 1: issue the predicted steps of every inner solve on a
                              formed operator (the PSD level 2, the general level 3) as one HIP
                              graph, captured once per solve, operator and chunk length and
                              replayed on the solve's stream. Same kernels and results as the
                              eager launches. Default 0. */
  int32_t batch_teams;     /* msp_solve_batched: a workgroup whose system is finished helps the
                              A-sweeps of a larger unfinished system (same results bit for bit;
                              chunked partials in a fixed order). Default 1. */
  int32_t autotune;        /* k >= 8 (level-1 sweeps on the matrix cores): before the first step,
                              time every admissible count of reduction segments (1..64) of the
                              block sweep on A_lo and keep the fastest. Cached per (dtype,
                              arithmetic, rows, cols, lda, k) for the process, and in the file
                              named by the environment variable MSP_TUNE_CACHE (one JSON object
                              per line) when set. The sweep's output scratch is overwritten
                              while timing; results differ from the built-in choice only by
                              summation order. Default 0 (built-in rule: about 2048
                              wavefronts). */
  int32_t level3_kernels;  /* general, level2_form 1, k <= 16: kernels per level-3 step. 2 (default):
                              the step as two kernels (decision, direction and operator product;
                              step length, residual, preconditioner product and dots), every
                              product a direct FP64 row dot over the formed s x s matrices;
                              0: the generic inner step (an operator product, a residual update,
                              a preconditioner product and a direction kernel). The same
                              iteration; results differ only in summation order. */
} msp_solve_opts;

typedef struct {
  msp_status status;
  int32_t outer_iters;      /* level-1 iterations (max over right-hand sides) */
  int64_t inner_iters;      /* level-2 iterations, summed over SolveM1 calls */
  int64_t level3_iters;     /* level-3 iterations, summed */
  int32_t refine_steps;     /* FP64 refinement steps taken (0 without refinement) */
  int32_t krylov_refine;    /* 1 if refinement switched to its Krylov form */
  int32_t restarts;         /* confirmation failures that restarted level 1 */
  double rel_residual_max;  /* max over RHS of the FP64 relative residual at exit */
  double sweep_bytes;       /* algorithmic bytes of A read by all level-1/2 sweeps */
  int64_t sweeps;           /* number of passes over A (per block of k RHS) */
  double sweep_ms;          /* profile != 0: summed duration of the timed level-1 sweeps */
  int64_t timed_sweeps;     /* profile != 0: number of sweeps in sweep_ms */
  int32_t sweep_segments;   /* k >= 8: reduction segments of the level-1 block sweep (tuned with
                               autotune, else the built-in rule); 0 for the other sweeps */
  double seconds;           /* host wall-clock time of the call, entry to return (the call
                               synchronises before returning, so this includes the device work) */
  int32_t trace_nodes;      /* msp_schatten / msp_orlicz: ridge-solve nodes taken (0 otherwise) */
} msp_solve_info;

void msp_solve_opts_default(msp_solve_opts* o /*host*/);
msp_status msp_solve_workspace(const msp_precond* P, int64_t k, const msp_solve_opts* opts, size_t* bytes /*host*/);
msp_status msp_solve(void* stream, const msp_precond* P,
                     const void* A_hi, msp_dtype hi_t, const void* A_lo, msp_dtype lo_t, int64_t lda,
                     double lambda, const double* B, int64_t ldb, int64_t k, double* X, int64_t ldx,
                     const msp_solve_opts* opts, void* ws, size_t ws_bytes, msp_solve_info* info /*host*/);

/* ---------------------------------------------------------------------------------
 * msp_solve_batched -- many independent PSD systems (A_i + lam_i I) X_i = B_i of
 * uneven size in one launch (Algorithm 1 with Algorithm 2 applied to each system;
 * the preconditioner of each system is built once and reused for all of its
 * right-hand sides, as Section 3 does for repeated solves).
 *
 * Each system brings its own MSP_SYM_PSD handle (from msp_nystrom on its own sketch;
 * n_i, s_i, lam_i and lam0_i come from the handle). All handles must store Y in the
 * same dtype. One workgroup solves one system: level-1 flexible PCG, SolveM1 with the
 * level-2 flexible PCG preconditioned by M2^{-1}, where the level-2 operator
 * (C^T C + lam~ W) is applied as one s x s matrix formed once per call (the same
 * operator; s^2 instead of n s work per inner step).
 * Supported (lo_t, hi_t, Y dtype): (F64, F64, F64), (F32 or BF16, F32 or F64, F32).
 * Without refinement (or lo_t == F64) the level-1 stop |B - (A + lam I) X| <= tol |B| is
 * confirmed on A_hi in FP64 (restart otherwise). With refine != 0 and lo_t != F64 the
 * solve is FP64 Krylov refinement on A_hi (flexible PCG) whose preconditioner is the
 * MSP solve on A_lo to refine_inner_tol; the refinement stops on the residual of A_hi,
 * confirmed by a recomputation.
 * Options used: tol, max_outer, inner_tol, max_inner, refine, refine_inner_tol,
 * max_refine. Right-hand sides are processed 16 per launch.
 *
 *   sys      [host] nsys descriptors; matrices row-major, vectors contiguous
 *   info     [host] out, nsys records (may be NULL): status, outer_iters (level-1 steps
 *            summed over inner solves), inner_iters, refine_steps, restarts,
 *            rel_residual_max (confirmed FP64 residual on A_hi)
 * Returns MSP_OK when every system met tol, else the first failure's status.
 * Synchronises the stream before returning.
 * ------------------------------------------------------------------------------ */
typedef struct {
  const msp_precond* P;  /* MSP_SYM_PSD handle of this system */
  const void* A_hi;      /* n x n, ld lda, dtype hi_t */
  const void* A_lo;      /* n x n, ld lda, dtype lo_t (may equal A_hi) */
  int64_t lda;
  const double* B;       /* n x k, vector j at B + j * ldb */
  int64_t ldb;
  double* X;             /* out, n x k, vector j at X + j * ldx */
  int64_t ldx;
} msp_system;

msp_status msp_solve_batched_workspace(int32_t nsys, const msp_system* sys /*host*/, int64_t k,
                                       const msp_solve_opts* opts, size_t* bytes /*host*/);
msp_status msp_solve_batched(void* stream, int32_t nsys, const msp_system* sys /*host*/, msp_dtype hi_t,
                             msp_dtype lo_t, int64_t k, const msp_solve_opts* opts, void* ws, size_t ws_bytes,
                             msp_solve_info* info /*host, nsys records*/);

/* ---------------------------------------------------------------------------------
 * msp_solve_batched_backward -- adjoints of many batched PSD solves X_i = (A_i + lam_i I)^{-1} B_i
 * in one launch: for each system, given G_i = dL/dX_i,
 *   dB_i = (A_i + lam_i I)^{-1} G_i           (A_i symmetric, so the transpose is itself;
 *                                             solved by msp_solve_batched with the same handles)
 *   dlambda_i = -sum_j <dB_ij, X_ij>
 *   dA_i = -dB_i X_i^T                        (dense n x n, only when dA != NULL)
 * Options, supported dtypes and processing as msp_solve_batched; X_i must be the forward
 * solutions. The workspace query includes the batched solve's workspace.
 *   sys      [host] nsys descriptors (matrices row-major, vectors contiguous, k each)
 *   dlambda  [host] out, nsys values (may be NULL)
 *   info     [host] out, nsys records of the adjoint solves (may be NULL)
 * Returns MSP_OK when every adjoint solve met tol, else the first failure's status (the
 * outputs of the other systems are still written). Synchronises the stream.
 * ------------------------------------------------------------------------------ */
typedef struct {
  const msp_precond* P;  /* MSP_SYM_PSD handle of this system */
  const void* A_hi;      /* n x n, ld lda, dtype hi_t */
  const void* A_lo;      /* n x n, ld lda, dtype lo_t (may equal A_hi) */
  int64_t lda;
  const double* X;       /* forward solutions, vector j at X + j * ldx */
  int64_t ldx;
  const double* G;       /* dL/dX, vector j at G + j * ldg */
  int64_t ldg;
  double* dB;            /* out, vector j at dB + j * lddb */
  int64_t lddb;
  double* dA;            /* out (may be NULL): n x n, ld ldda */
  int64_t ldda;
} msp_system_grad;

msp_status msp_solve_batched_backward_workspace(int32_t nsys, const msp_system_grad* sys /*host*/, int64_t k,
                                                const msp_solve_opts* opts, size_t* bytes /*host*/);
msp_status msp_solve_batched_backward(void* stream, int32_t nsys, const msp_system_grad* sys /*host*/,
                                      msp_dtype hi_t, msp_dtype lo_t, int64_t k, const msp_solve_opts* opts,
                                      void* ws, size_t ws_bytes, double* dlambda /*host, nsys*/,
                                      msp_solve_info* info /*host, nsys records*/);

/* ---------------------------------------------------------------------------------
 * msp_solve_backward -- adjoint of X = (A + lam I)^{-1} B for symmetric PSD A.
 *
 * Given G = dL/dX: dB = (A + lam I)^{-T} G = (A + lam I)^{-1} G (A symmetric), solved
 * with the same handle, lam and iteration as msp_solve; dlambda = -sum_j <dB_j, X_j>;
 * dA = -dB X^T, written densely (n x n, ld ldda) only when dA != NULL.
 *   dlambda  [host] out, may be NULL
 * MSP_GENERAL handles return MSP_ERR_UNSUPPORTED.
 * ------------------------------------------------------------------------------ */
msp_status msp_solve_backward(void* stream, const msp_precond* P,
                              const void* A_hi, msp_dtype hi_t, const void* A_lo, msp_dtype lo_t, int64_t lda,
                              double lambda, const double* X, int64_t ldx, const double* G, int64_t ldg, int64_t k,
                              double* dB, int64_t lddb, double* dlambda /*host*/, double* dA, int64_t ldda,
                              const msp_solve_opts* opts, void* ws, size_t ws_bytes, msp_solve_info* info /*host*/);

/* ---------------------------------------------------------------------------------
 * msp_schatten -- spectral sums through ridge solves (Section 3.2, Theorem 3.3).
 *
 * MSP_TRACE_SCHATTEN_P: ||A||_p^p = tr((A^T A)^{p/2}), 0 < p < 2, from
 *   (sin(pi p/2)/pi) int_0^inf t^{p/2-1} tr(A^T A (A^T A + t I)^{-1}) dt with t = e^u,
 *   the trapezoid rule with step h, and Hutchinson's estimator over the probe block G:
 *   per probe and node <A g, A x>, x = (A^T A + t_j I)^{-1} g solved by the three-level
 *   MSP of P (an MSP_GENERAL handle; lam~ = t_j + lam0 per node).
 *   Nodes: u_lo finite: u_j = u_lo + j h <= u_hi. u_lo NaN: u_j = u_hi - j h going down,
 *   the nodes below the last one taken at their t -> 0 value |g|^2 (a geometric series);
 *   since t <g, x> is nondecreasing in t, after node j that replacement is off by at most
 *   t_j <g, x_j> times the remaining weight per probe, and the descent stops when the mean
 *   of that bound is at most 1e-4 of the estimate (at most 400 nodes). u_hi NaN: from a
 *   30-step power iteration on A^T A, u_hi = 2 ln(1.01 |A|) + (2/(2-p)) ln 1e4.
 * MSP_TRACE_EFFDIM: d_lam = tr(A (A + lam I)^{-1}) = mean_k (g^T g - lam g^T x),
 *   x = (A + lam I)^{-1} g by the two-level MSP of P (an MSP_SYM_PSD handle); `p` is lam.
 *   G        N probes of length n, ld ldg, FP64; or NULL: the N probes msp_gaussian_probes
 *            draws from probe_seed (generated into the workspace; probe_seed ignored
 *            otherwise)
 *   estimate, std_err  [host] out (std_err: standard error over probes)
 * Returns MSP_ERR_NO_CONVERGENCE, with the estimate and info still written, when some
 * ridge solve stopped at its iteration cap; other failures return before any output.
 * Synchronises the stream before returning.
 * ------------------------------------------------------------------------------ */
typedef enum { MSP_TRACE_SCHATTEN_P = 0, MSP_TRACE_EFFDIM = 1 } msp_trace_kind;
msp_status msp_schatten_workspace(const msp_precond* P, int64_t nprobes, const msp_solve_opts* opts,
                                  size_t* bytes /*host*/);
msp_status msp_schatten(void* stream, msp_trace_kind kind, msp_precond* P,
                        const void* A_hi, msp_dtype hi_t, const void* A_lo, msp_dtype lo_t, int64_t lda,
                        double p, const double* G, int64_t ldg, int64_t nprobes, uint64_t probe_seed,
                        double h, double u_lo, double u_hi, const msp_solve_opts* opts,
                        void* ws, size_t ws_bytes, double* estimate /*host*/, double* std_err /*host*/,
                        msp_solve_info* info /*host*/);

/* ---------------------------------------------------------------------------------
 * msp_orlicz -- the Orlicz norm |A|_g = inf { r > 0 : sum_i g(sigma_i(A) / r) <= 1 } for
 * g(s) = sum_q c_q s^{p_q}, c_q > 0, 0 < p_q < 2 (a norm when every p_q >= 1), through the
 * spectral sums of Section 3.2: sum_i g(sigma_i / r) = sum_q c_q r^{-p_q} ||A||_{p_q}^{p_q},
 * every Schatten sum from the same ridge solves (the quadrature nodes do not depend on p,
 * only the weights do), nodes going down from u_hi as in msp_schatten with u_lo NaN (the
 * descent stops when every sum's tail bound is at most eps_q of that sum; eps_q NaN: 1e-4;
 * u_hi NaN: from |A| for the largest p_q). The root r is found by bisection on ln r.
 *   coefs, powers  [host] nterms (1..16) values each
 *   G, ldg, nprobes, probe_seed   the probe block, as for msp_schatten
 *   estimate   [host] out: r;  std_err [host] out: the delta-method standard error of r
 *   sums       [host] out, may be NULL: the nterms Schatten sum estimates
 * Workspace: msp_schatten_workspace. Returns MSP_ERR_NO_CONVERGENCE, with every output
 * written, when some ridge solve stopped at its iteration cap. Synchronises the stream.
 * ------------------------------------------------------------------------------ */
msp_status msp_orlicz(void* stream, msp_precond* P, const void* A_hi, msp_dtype hi_t, const void* A_lo,
                      msp_dtype lo_t, int64_t lda, const double* coefs /*host*/, const double* powers /*host*/,
                      int64_t nterms, const double* G, int64_t ldg, int64_t nprobes, uint64_t probe_seed,
                      double h, double u_hi, double eps_q, const msp_solve_opts* opts, void* ws,
                      size_t ws_bytes, double* estimate /*host*/, double* std_err /*host*/,
                      double* sums /*host*/, msp_solve_info* info /*host*/);

/* ---------------------------------------------------------------------------------
 * msp_kyfan -- the Ky Fan k-norm ||A||_(k) = sum_{i<=k} sigma_i(A) (Section 3.2 names Ky Fan
 * norms beside the Orlicz norms). A sum of the top k singular values needs the top of the
 * spectrum itself, which ridge solves (A^T A + t I)^{-1} do not isolate, so it is taken from
 * the top singular subspace: Z_0 = the b >= k Gaussian vectors msp_gaussian_probes draws from
 * seed, Q_0 = orth(Z_0), Q_i = orth(A^T A Q_{i-1}) for i = 1..q, and the Rayleigh-Ritz values of
 * A on Q_q (square roots of the eigenvalues of (A Q_q)^T (A Q_q)); orth(Z) = Z V Lambda^{-1/2}
 * from the eigenpairs of Z^T Z, dropping directions with eigenvalue <= 1e-13 of the largest.
 * Ritz values interlace, so the estimate is at most ||A||_(k) and converges to it; with
 * rank(A) <= b one step is exact. 2q + 1 block products with A and q with A^T, FP64
 * arithmetic; the b x b eigenproblems by cyclic Jacobi rotations in one workgroup.
 *   A        m x n, F64 or F32, ld lda >= n
 *   k, b, q  1 <= k <= b <= min(64, m, n), 0 <= q
 *   estimate [host] out; sigma [host] out, may be NULL: the b Ritz values, decreasing
 * Synchronises the stream before returning.
 * ------------------------------------------------------------------------------ */
msp_status msp_kyfan_workspace(int64_t m, int64_t n, int64_t b, size_t* bytes /*host*/);
msp_status msp_kyfan(void* stream, const void* A, msp_dtype a_t, int64_t m, int64_t n, int64_t lda, int64_t k,
                     int64_t b, int32_t q, uint64_t seed, void* ws, size_t ws_bytes, double* estimate /*host*/,
                     double* sigma /*host*/);

/* ---------------------------------------------------------------------------------
 * msp_gaussian_probes -- the Gaussian probe vectors of Hutchinson's estimator (Section
 * 3.2 draws them; the paper fixes no generator): Box-Muller (1958) over the counter-based
 * SplitMix64 stream of msp_sketch. Probe j has key k_j = fmix((seed ^ 0xD1B54A32D192ED03)
 * + (j+1)G); element i takes outputs u1, u2 number 2i+1 and 2i+2 of the stream started
 * at k_j, U1 = (hi53(u1) + 1) 2^-53 in (0, 1], U2 = hi53(u2) 2^-53 in [0, 1), and
 * g = sqrt(-2 ln U1) cos(2 pi U2) in FP64.
 *   G        out, N probes of length n, probe j at G + j * ldg (ldg >= n)
 * Asynchronous.
 * ------------------------------------------------------------------------------ */
msp_status msp_gaussian_probes(void* stream, int64_t n, int64_t N, uint64_t seed, double* G, int64_t ldg);

/* ---------------------------------------------------------------------------------
 * Least squares min |A x - b| for a tall A (n x d, n >= d): sketch-and-precondition with
 * MSP as the inner solver (Section 3, the least-squares corollary).
 *
 * msp_left_sketch -- Psi, a Definition 2.1 sketch with q rows over the n rows of A
 *   (gamma nonzeros +-1/sqrt(gamma) per column, from seed), and A~ = Psi A (q x d, FP64,
 *   ld ldat), a subspace embedding of A for q of a few times d.
 *   A          n x d row-major (lda >= d), F64 or F32
 *   Psi_rows   [n][gamma] int32 out; Psi_signs [n][gamma] int8 out (+1 / -1)
 *   ws         msp_left_sketch_workspace(n, q, gamma) bytes, 256-B aligned; caller-owned
 *
 * msp_lstsq -- flexible PCG on A^T A x = A^T b (k right-hand sides) whose preconditioner
 *   applies (A~^T A~)^{-1} by msp_solve on P, an MSP_GENERAL handle of A~ with lambda = 0
 *   (msp_sketch and msp_nystrom on A~), in normal mode to the relative accuracy
 *   opts->refine_inner_tol (a constant suffices; default 1e-4). The products with A use
 *   FP64 arithmetic on F64 or F32 storage. Stops when |A^T (b - A x)| <= opts->tol |A^T b|
 *   per right-hand side (confirmed on the recomputed residual) or after opts->max_outer
 *   steps.
 *   At         A~ (P->m x d, FP64, ld ldat), the matrix P was built from
 *   B          k columns of length n (ld ldb); X: k columns of length d (ld ldx), out
 *   ws         msp_lstsq_workspace(P, n, k, opts) bytes, 256-B aligned (holds the inner
 *              solve's workspace)
 *   info       outer_iters: steps of the outer iteration; inner_iters: level-1 steps of the
 *              inner solves; level3_iters: their level-2 and level-3 steps; rel_residual_max:
 *              max_j |A^T (b_j - A x_j)| / |A^T b_j| in FP64; sweeps, sweep_bytes: passes
 *              over A.
 *   Returns MSP_ERR_NO_CONVERGENCE (X still written) when the tolerance was not reached.
 * ------------------------------------------------------------------------------ */
msp_status msp_left_sketch_workspace(int64_t n, int64_t q, int32_t gamma, size_t* bytes /*host*/);
msp_status msp_left_sketch(void* stream, const void* A, msp_dtype a_t, int64_t n, int64_t d, int64_t lda, int64_t q,
                           int32_t gamma, uint64_t seed, int32_t* Psi_rows, int8_t* Psi_signs, double* At,
                           int64_t ldat, void* ws, size_t ws_bytes);
msp_status msp_lstsq_workspace(const msp_precond* P, int64_t n, int64_t k, const msp_solve_opts* opts,
                               size_t* bytes /*host*/);
msp_status msp_lstsq(void* stream, const msp_precond* P, const double* At, int64_t ldat, const void* A,
                     msp_dtype a_t, int64_t n, int64_t lda, const double* B, int64_t ldb, int64_t k, double* X,
                     int64_t ldx, const msp_solve_opts* opts, void* ws, size_t ws_bytes,
                     msp_solve_info* info /*host*/);

/* Thread-local description of the last failure (empty string if none). */
const char* msp_last_error(void);
/* Library version string. */
const char* msp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MSP_H */
