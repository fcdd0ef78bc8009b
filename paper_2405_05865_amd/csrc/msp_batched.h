// Internal declarations of the batched PSD solve (k_batched.hip, msp_batch.hip).
#pragma once
#include "msp_internal.h"

#define MSP_BATCH_KMAX 16  // right-hand sides per launch (the N dimension of the 16x16 tiles)
#define MSP_BATCH_MAXH 31  // helper workgroups per system
#define MSP_BATCH_CHR 512  // rows per sweep chunk (16 wavefronts x 32-row tiles)

// Cooperation record of one system (device memory, zeroed before the launch). The
// system's own workgroup (the leader) publishes each A-sweep as an epoch; workgroups
// whose systems are finished join as helpers and claim slices of its row chunks.
struct BatchTeam {
  int32_t epoch, nslice, mode, finish;
  int32_t joined, started, ncols, pad;
  int32_t claim[MSP_BATCH_MAXH + 1];  // slice s claimed for epoch claim[s]
  int32_t done[MSP_BATCH_MAXH + 1];   // slice s completed for epoch done[s]
  // the published job: 0 q = (A_lo + lam I) x, 1 q = (A_hi + lam I) x, 2 out = rhs - (A_hi +
  // lam I) x, 3 out = (rhs - Y x) lam (x s-vectors), 4 chunk partials of Y^T rhs
  const void* bv;     // x in the arithmetic type of the product
  const double* x;
  const double* rhs;
  double* out;
  int64_t ldb, ldr;
  double lam;
};

// One system as the kernel sees it (host-filled, copied to the device)
struct BatchSys {
  const void* A_lo;   // n x n, row-major, ld lda (swept inside MSP)
  const void* A_hi;   // n x n, ld lda (FP64 residuals)
  int64_t lda;
  const void* Y;      // C = A S^T, n x s, ld ldy
  int64_t ldy;
  const double* H;    // s x s: C^T C + lam~ W (the level-2 operator)
  const double* Minv; // s x s: M2^{-1}
  const double* B;    // n x k, vector j at B + j * ldb
  int64_t ldb;
  double* X;          // n x k, vector j at X + j * ldx
  int64_t ldx;
  double* vec;        // 11 n-vectors (ld ldn) and 7 s-vectors (ld lds), kcap columns each
  float* pf;          // F32 copy of the level-1 direction, kcap x ldn
  int32_t n, s, ldn, lds;
  double lam, lt;     // lambda and lambda~ = lambda + lambda0
  int32_t aln_lo, aln_hi, aln_y, aln_m;  // rows of A_lo / A_hi / Y / the s x s matrices are 16-byte aligned
  BatchTeam* team;    // cooperation record
  double* cpart;      // per-chunk partials of <x, A x>: [ceil(n / MSP_BATCH_CHR)][MSP_BATCH_KMAX]
  double* ypart;      // per-chunk partials of Y^T r: [ceil(n / MSP_BATCH_CHR)][MSP_BATCH_KMAX][s]
  int32_t id;         // position in the caller's array
  int32_t pad;
};

struct BatchPrm {
  double tol, inner_tol, refine_tol;
  int32_t max_outer, max_inner, max_refine, refine;
  int32_t kcap;       // columns allocated per vector
  int32_t profile;    // record wall-clock time per phase (BatchOut.ticks)
  int32_t teams;      // finished workgroups help the remaining systems' sweeps
  int32_t nsys;       // systems in the launch (helpers scan their records)
};

enum { BT_SWEEP_LO = 0, BT_SWEEP_HI, BT_YT, BT_LEVEL2, BT_YZ, BT_TOTAL, BT_NPHASE };

struct BatchOut {
  int32_t code;       // 0 ok, 1 tolerance not reached, 2 breakdown, 3 non-finite,
                      // 4 a helper's slice did not complete in time
  int32_t outer, inner, refine, restarts;
  int32_t helped, selfdone;  // sweep slices done by helpers / taken back by the leader
  int32_t pad;
  double relres;      // largest confirmed relative residual on A_hi
  uint64_t ticks[BT_NPHASE];  // profile: wall-clock ticks per phase (thread 0's view)
};

bool batch_types_supported(msp_dtype lo_t, msp_dtype hi_t, msp_dtype y_t);
hipError_t launch_batch_psd(hipStream_t st, msp_dtype lo_t, msp_dtype hi_t, msp_dtype y_t, const BatchSys* sys,
                            int nsys, const BatchPrm& prm, int k, BatchOut* out);
