// FP64 complex dense linear algebra used by the ACE build and apply.
#pragma once

#include "common.hpp"

namespace fx {

// C = alpha op(A) op(B) + beta C (complex double, column-major), op 0 = N,
// 1 = conjugate transpose; `batch` independent products with element strides
// sA, sB, sC.  nsplit_hint > 0 fixes the number of K splits (1 = none);
// 0 chooses one.  Split partial sums are reduced in FP64 in a fixed order.
fx_status zgemm(fx_ctx* ctx, Workspace* ws, hipStream_t st, int opa, int opb, int M, int N, int K, cpx<double> alpha,
                const void* A, int64_t lda, const void* B, int64_t ldb, cpx<double> beta, void* C, int64_t ldc,
                int batch, int64_t sA, int64_t sB, int64_t sC, int nsplit_hint);

// In-place blocked Cholesky A = L L^H (lower; the strict upper part is
// zeroed).  *info_dev (device int, must start at 0) receives 1 + the first
// column whose pivot was not positive, or stays 0.
fx_status zpotrf(fx_ctx* ctx, Workspace* ws, hipStream_t st, int n, void* A, int64_t lda, int* info_dev);

// In-place inverse of a lower triangular n x n matrix.
fx_status ztrinv(fx_ctx* ctx, Workspace* ws, hipStream_t st, int n, void* A, int64_t lda);

// H = (M + M^H)/2 (n x n, ld n), Aneg = -H, *ex_dev = 1/2 Re tr H (nullable).
fx_status zherm(hipStream_t st, int n, const void* M, int64_t ldm, void* H, void* Aneg, double* ex_dev);

// B = A^H (n x n).
fx_status zconj_transpose(hipStream_t st, int n, const void* A, int64_t lda, void* B, int64_t ldb);

}  // namespace fx
