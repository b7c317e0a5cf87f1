// Internal interface of the V_X pair path (used by fx_apply_vx, the ACE
// build and the serving loop).
#pragma once

#include "common.hpp"

namespace fx {

struct VxArgs {
  const fx_cell* cell = nullptr;
  const fx_kernel* kern = nullptr;
  const void* psi = nullptr;
  int n_psi = 0;
  int64_t ld_psi = 0;
  const void* phi = nullptr;
  int n_phi = 0;
  int64_t ld_phi = 0;
  void* out = nullptr;
  int64_t ld_out = 0;
  fx_dtype in_dtype = FX_C128;
  fx_dtype out_dtype = FX_C128;
  fx_prec prec = FX_PREC_FP64;
  double* ex_dev = nullptr;
  // tuning (0 = automatic)
  size_t work_cap = 0;  // bytes of pair work volume per batch
  int force_nj = 0;     // orbitals per batch
  int nthr_a = 0, nthr_b = 0;
};

struct VxStats {
  int nk = 0, nj = 0;
  int64_t launches = 0;
};

fx_status check_vx_args(const VxArgs& a);
// Copy ncols columns of nr complex values between dtypes (strided).
fx_status convert_cols(const void* in, fx_dtype din, int64_t ld_in, void* out, fx_dtype dout, int64_t ld_out,
                       int64_t nr, int ncols, hipStream_t st);
fx_status vx_apply(fx_ctx* ctx, Workspace* ws, const VxArgs& a, hipStream_t st, VxStats* stats);

}  // namespace fx
