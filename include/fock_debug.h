/*
 * libfock debug extension: host execution of the device pass code, for
 * checking FFT plans, digit-reversed spectra and kernel tables without a GPU;
 * and forced allocation failures, for tests of the error paths.
 */
#ifndef LIBFOCK_FOCK_DEBUG_H
#define LIBFOCK_FOCK_DEBUG_H

#include "fock.h"

#ifdef __cplusplus
extern "C" {
#endif

/* v = (-scale/Omega) IFFT_u[ K FFT_u( conj(psi_j) phi_k ) ] for one pair, computed
 * on the host by the same pass code the kernels run (Eq. applyVX, one term).
 * psi_j, phi_k, v: host arrays of N_r interleaved complex doubles; prec 0 runs
 * the FP64 instantiation, 1 the FP32 one (inputs rounded, result widened).
 * Errors: FX_ERR_INVALID, FX_ERR_UNSUPPORTED. */
fx_status fx_debug_host_pair(const fx_cell* cell, const fx_kernel* kernel, int prec, const double* psi_j,
                             const double* phi_k, double* v);

/* As fx_debug_host_pair, with the radix schedule of each axis given as in
 * fx_vx_config.radix: `radix` points to 3 rows of 4 int32 (x, y, z), stages
 * in order, 0-terminated, an all-zero row meaning the default schedule;
 * NULL means all defaults.  Errors: FX_ERR_INVALID (a row that is not a
 * schedule of its edge), FX_ERR_UNSUPPORTED. */
fx_status fx_debug_host_pair_plan(const fx_cell* cell, const fx_kernel* kernel, int prec, const int32_t* radix,
                                  const double* psi_j, const double* phi_k, double* v);

/* The radix schedules the autotuner considers for edge n (at most three
 * stages, radices from {2,3,4,6,8,9,12}, the default first): up to
 * max_plans rows of 4 int32 written to radix_out (0-terminated), their
 * number to *count.  Errors: FX_ERR_INVALID, FX_ERR_UNSUPPORTED. */
fx_status fx_debug_axis_plans(int32_t n, int32_t max_plans, int32_t* radix_out, int32_t* count);

/* Make the k-th device allocation of the library after this call (k >= 1,
 * counted over all contexts of the process) fail once with FX_ERR_OOM, as if
 * the HBM budget were exhausted; k = 0 cancels a pending failure.  A call that
 * meets the failure returns FX_ERR_OOM and leaves its context usable.  The
 * environment variable FX_FAULT_INJECT=k does the same for the k-th
 * allocation of the process.  Errors: FX_ERR_INVALID (k < 0). */
fx_status fx_debug_fail_alloc(int64_t k);

/* Bandwidth probe: `iters` passes (after one warm-up pass) of a stream over
 * the device buffer buf of `bytes` bytes (16-byte aligned, a multiple of 16,
 * at least 4096), 16 bytes per lane with non-temporal hints, on `stream`:
 * mode 0 reads it (its first 4 KiB may be overwritten), 1 writes it, 2 reads
 * and writes it in place (adding 1 to every 32-bit word).  *gbps receives the bytes moved (2 x bytes per pass
 * in place) per second, timed with events on the stream; the call waits for
 * the passes.  These are the DRAM rates the pass kernels' rates are read
 * against.  Errors: FX_ERR_INVALID, FX_ERR_DEVICE. */
fx_status fx_debug_stream(fx_ctx* ctx, int32_t mode, void* buf, size_t bytes, int32_t iters, void* stream,
                          double* gbps);

#ifdef __cplusplus
}
#endif

#endif /* LIBFOCK_FOCK_DEBUG_H */
