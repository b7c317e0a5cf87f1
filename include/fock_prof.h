/*
 * libfock profiling extension: per-kernel durations measured with HIP events
 * recorded on the stream each kernel is launched on.  Meant for benchmarks
 * and roofline accounting; costs two event records per timed launch.
 */
#ifndef LIBFOCK_FOCK_PROF_H
#define LIBFOCK_FOCK_PROF_H

#include "fock.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fx_kernel_id {
  FX_K_VX_PLANE_FWD = 0, /* pair product + forward FFT along x and y */
  FX_K_VX_PENCIL_Z = 1,  /* forward FFT z, kernel multiply, inverse FFT z */
  FX_K_VX_PLANE_INV = 2, /* inverse FFT y and x, times psi_j, j-sum */
  FX_K_CONVERT = 3,      /* precision conversion of inputs */
  FX_K_GEMM_CN = 4,      /* complex GEMM C = A^H B (split over the long dimension) */
  FX_K_GEMM_NN = 5,      /* complex GEMM Y = A C (tall) */
  FX_K_REDUCE = 6,       /* FP64 reduction of split partial products */
  FX_K_SPLIT = 7,        /* residual split X -> (X_p, r_X) */
  FX_K_LINALG = 8,       /* Cholesky / triangular inverse / Hermitisation */
  FX_K_COUNT = 16
} fx_kernel_id;

/* Turn timing on (on != 0) or off; either way the accumulated records are cleared. */
fx_status fx_prof_enable(fx_ctx* ctx, int on);

/* Wait for the recorded events and return, for kernel `id`, the number of timed
 * launches, their summed duration in milliseconds and their summed algorithmic
 * work: HBM bytes the launch must move as designed (FFT passes, conversions,
 * splits, reductions) or floating-point operations it executes (GEMMs; the
 * residual products included).  Any output pointer may be NULL. */
fx_status fx_prof_read(fx_ctx* ctx, int id, int64_t* launches, double* total_ms, double* work);

#ifdef __cplusplus
}
#endif

#endif /* LIBFOCK_FOCK_PROF_H */
