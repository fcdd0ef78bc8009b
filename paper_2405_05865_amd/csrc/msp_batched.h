// Internal declarations of the batched PSD solve (k_batched.hip, msp_batch.hip).
#pragma once
#include "msp_internal.h"

#define MSP_BATCH_KMAX 16  // right-hand sides per launch (the N dimension of the 16x16 tiles)

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
  int32_t id;         // position in the caller's array
  int32_t pad;
};

struct BatchPrm {
  double tol, inner_tol, refine_tol;
  int32_t max_outer, max_inner, max_refine, refine;
  int32_t kcap;       // columns allocated per vector
  int32_t profile;    // record wall-clock time per phase (BatchOut.ticks)
};

enum { BT_SWEEP_LO = 0, BT_SWEEP_HI, BT_YT, BT_LEVEL2, BT_YZ, BT_TOTAL, BT_NPHASE };

struct BatchOut {
  int32_t code;       // 0 ok, 1 tolerance not reached, 2 breakdown, 3 non-finite
  int32_t outer, inner, refine, restarts, pad;
  double relres;      // largest confirmed relative residual on A_hi
  uint64_t ticks[BT_NPHASE];  // profile: wall-clock ticks per phase (thread 0's view)
};

bool batch_types_supported(msp_dtype lo_t, msp_dtype hi_t, msp_dtype y_t);
hipError_t launch_batch_psd(hipStream_t st, msp_dtype lo_t, msp_dtype hi_t, msp_dtype y_t, const BatchSys* sys,
                            int nsys, const BatchPrm& prm, int k, BatchOut* out);
