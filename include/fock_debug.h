/*
 * libfock debug extension: host execution of the device pass code, for
 * checking FFT plans, digit-reversed spectra and kernel tables without a GPU.
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

#ifdef __cplusplus
}
#endif

#endif /* LIBFOCK_FOCK_DEBUG_H */
