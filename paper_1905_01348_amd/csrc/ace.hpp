// ACE handle and internal entry points.
#pragma once

#include <utility>
#include <vector>

#include "common.hpp"

// Split (low-precision) copies of xi for one GEMM precision, padded along
// the reduction dimension to a multiple of the GEMM K tile:
//   col: N rows of Kc = roundup(2 N_r) values, row m = interleaved column m of xi
//        (operand A of C = xi^H phi);
//   row: N_r rows of Kn = roundup(2 N) values, row r = interleaved row r of xi
//        (operand A of y = -xi C).
// p = round(xi), r = round(xi - p).
struct AceSplit {
  bool ready = false;
  int64_t kc = 0, kn = 0;
  void *col_p = nullptr, *col_r = nullptr, *row_p = nullptr, *row_r = nullptr;
  void* smax = nullptr;  // FP16 forms: largest |xi| as FP32 bits (its power-of-two factor)
};

struct fx_ace {
  fx_ctx* ctx = nullptr;
  int n = 0;
  int64_t nr = 0;
  fx_cell cell;
  fx_kernel kern;
  fx_prec prec = FX_PREC_ACE_FP64;
  double ex = 0.0;
  void* xi = nullptr;  // complex double, N_r x N, ld N_r
  void* L = nullptr;   // complex double, N x N, column-major (lower Cholesky factor of -M)
  void* M = nullptr;   // complex double, N x N, Hermitised Psi^H W
  AceSplit f32, b16, f16;  // split forms for FP32, BF16 and FP16 matrix cores
  fx::Workspace ws;
  std::vector<std::pair<void*, size_t>> owned;
};

namespace fx {
fx_status ace_alloc(fx_ace* a, size_t bytes, void** out);
fx_status ace_build_impl(fx_ctx* ctx, Workspace* ws, const fx_cell* cell, const fx_kernel* kern, const void* psi,
                         int n, int64_t ld, fx_dtype in_dtype, fx_prec vx_prec, fx_prec ace_prec, hipStream_t st,
                         fx_ace** out, double* ex_host, double* ex_dev_out = nullptr);
fx_status ace_apply_impl(fx_ctx* ctx, Workspace* ws, const fx_ace* a, const void* phi, int nphi, int64_t ld_phi,
                         void* out, int64_t ld_out, fx_dtype in_dtype, fx_dtype out_dtype, fx_prec prec,
                         hipStream_t st);
}  // namespace fx
