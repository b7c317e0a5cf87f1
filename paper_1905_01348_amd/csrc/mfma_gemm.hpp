// ACE projections on the matrix cores (FP32 or BF16 inputs, FP32
// accumulation, optional residual step combined in FP64).
#pragma once

#include "ace.hpp"

namespace fx {
// Create the split copies of xi used by `prec` (no-op when present).
fx_status ace_prepare_split(fx_ace* a, fx_prec prec, hipStream_t st);
// K_ACE phi with FX_PREC_ACE_{FP32R,BF16R,FP32,BF16}.
fx_status ace_apply_mfma(fx_ctx* ctx, Workspace* ws, fx_ace* a, const void* phi, int nphi, int64_t ld_phi, void* out,
                         int64_t ld_out, fx_dtype in_dtype, fx_dtype out_dtype, fx_prec prec, hipStream_t st);
}  // namespace fx
