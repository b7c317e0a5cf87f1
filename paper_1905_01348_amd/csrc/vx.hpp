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
  int nthr_b = 0;  // threads of the pencil pass
  int xtile = 0;   // x columns per pencil-pass workgroup
  int pipe = -1;   // plane-inverse pass prefetches the next plane: 1 yes, 0 no, -1 automatic
  int halve = -1;  // phi == psi: solve each unordered pair once (1 yes, 0 no, -1 automatic)
};

struct VxStats {
  int nk = 0, nj = 0;
  int64_t launches = 0;
  int64_t solves = 0;  // pair Poisson solves run (N*N_t, or N(N+1)/2 when halved)
};

// One batch of the pair passes for the compile-time-specialised kernels
// (cubic grids of edge 24, 48, 72 or 96; vx_ct.hip).
template <typename T>
struct CtBatch {
  const cpx<T>* psi;
  int64_t ld_psi;
  const cpx<T>* phi;
  int64_t ld_phi;
  cpx<T>* work;
  int j0, nj, k0, nk, npairs;
  const cpx<T>* tw;  // twiddles of the edge (all three axes share them)
  const T* kfold;
  const int* fold;  // folded frequency per digit-reversed position
  int tri;          // diagonal batch of a halved apply: pairs jj <= kk only, packed
};
template <typename A>
struct CtAcc {
  cpx<A>* acc;
  int64_t ld_acc;
  int first;
  void* out;
  int64_t ld_out;
  int out_c64, last, pipe;
};
bool ct_supported(const fx_cell* cell);
template <typename T>
fx_status ct_pass_a(fx_ctx* ctx, hipStream_t st, int n, const CtBatch<T>& b);
template <typename T>
fx_status ct_pass_b(fx_ctx* ctx, hipStream_t st, int n, const CtBatch<T>& b);
// role 0: targets are the batch's k; role 1: targets are its j (halved apply)
template <typename T, typename A>
fx_status ct_pass_c(fx_ctx* ctx, hipStream_t st, int n, const CtBatch<T>& b, const CtAcc<A>& c, int role);

fx_status check_vx_args(const VxArgs& a);
// Copy ncols columns of nr complex values between dtypes (strided).
fx_status convert_cols(const void* in, fx_dtype din, int64_t ld_in, void* out, fx_dtype dout, int64_t ld_out,
                       int64_t nr, int ncols, hipStream_t st);
fx_status vx_apply(fx_ctx* ctx, Workspace* ws, const VxArgs& a, hipStream_t st, VxStats* stats);

}  // namespace fx
