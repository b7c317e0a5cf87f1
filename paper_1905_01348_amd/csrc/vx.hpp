// Internal interface of the V_X pair path (used by fx_apply_vx, the ACE
// build and the serving loop).
#pragma once

#include "common.hpp"

namespace fx {

// Orbital blocks of a multi-trajectory launch (served V_X requests of several
// trajectories on one grid): targets [start[s], start[s+1]) of the launch
// pair with the n_psi orbitals at psi[s] (same count and stride for every
// block).  n == 0: one block, the launch's psi.
constexpr int kMaxTrajSegs = 8;
struct TrajSegs {
  int n = 0;
  int start[kMaxTrajSegs + 1] = {0};
  const void* psi[kMaxTrajSegs] = {nullptr};
};

// The orbital block of target k (device and host).
template <typename T>
__host__ __device__ inline const cpx<T>* seg_psi(const TrajSegs& s, const cpx<T>* dflt, int k) {
  if (s.n == 0) return dflt;
  int g = 0;
#pragma unroll
  for (int i = 1; i < kMaxTrajSegs; ++i)
    if (i < s.n && k >= s.start[i]) g = i;
  return reinterpret_cast<const cpx<T>*>(s.psi[g]);
}

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
  bool internal_kernel = false;  // kern may be the library's own kinetic kind
  // launch configuration (0 / -1 = automatic: the context's tuned
  // configuration for this grid and form if there is one, else defaults)
  size_t work_cap = 0;  // bytes of pair work volume per batch
  int force_nj = 0;     // orbitals per batch
  int nthr_b = 0;  // generic z pass: threads per workgroup
  int xtile = 0;   // generic z pass: x columns per workgroup
  int pipe = -1;   // generic plane-inverse pass prefetches the next plane: 1 yes, 0 no, -1 automatic
  int halve = -1;  // phi == psi: solve each unordered pair once (1 yes, 0 no, -1 automatic)
  int kernels = 0;  // 1 specialised (cubic workload edges only), 2 generic, 0 automatic
  int a_pipe = -1;  // specialised plane-forward pass: 1 register prefetch, 0 two workgroups per CU
  int b_var = 0;    // specialised z pass tile: 1 default, 2 half, 3 whole rows, 4 persistent, 0 automatic
  int c_var = 0;    // specialised plane-inverse form: 1 default, 2 second thread count, 3/4 those with the
                    // next plane staged in LDS, 0 automatic
  int a_var = 0;    // specialised plane-forward threads: 1 default, 2 second count, 3 that with the
                    // wave-level x transform (72 and 96), 0 automatic
  int nt_hint = -1;  // specialised kernels: non-temporal hints on the pair volume (1, 0, -1 automatic = 1)
  int c_split = 0;   // specialised plane-inverse pass: j-sum groups (1, 2, 4 or 8; 0 automatic = 1)
  bool plans_set = false;  // generic kernels: radix schedules in `plans`
  PlanSet plans;
  // several trajectories' orbital blocks (specialised kernels, phi != psi);
  // psi is then the first block's
  TrajSegs segs;
  // allocation-free form: `ws` carves from a fixed scratch region, the grid
  // tables are built there on the device, no conversion, no pair halving
  bool no_alloc = false;
};

// Radix rows (0-terminated, all-zero row = default) to plans; false if a row
// is not a valid schedule of its edge.  *any: some row was given.
bool plans_from_radix(const fx_cell* cell, const int32_t radix[3][4], PlanSet* ps, bool* any);
std::array<int, 5> vx_tune_key(const fx_cell* cell, fx_prec prec, bool square);
// Fill the automatic fields of `a` from the environment (FX_VX_* overrides,
// for experiments), then from the context's tuned configuration.
void resolve_vx_config(fx_ctx* ctx, VxArgs* a);
// The autotuner (tune.hip): tunes and stores the configuration of one shape.
fx_status vx_autotune_impl(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel, int n_psi, int n_phi,
                           bool square, fx_prec prec, hipStream_t st, fx_vx_config* best, double* ms_per_kpair);
// Whether a call is the phi == psi form (all targets are the orbitals).
inline bool vx_square_form(const VxArgs& a) {
  return a.phi == a.psi && a.ld_phi == a.ld_psi && a.n_phi == a.n_psi;
}

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
  int a_pipe;       // plane-forward pass: register prefetch of the next plane
  int b_var;        // z pass: 1 default x tile, 2 half tile, 3 whole x rows, 4 persistent (default tile)
  int c_var;        // plane-inverse pass: 1 default threads, 2 the second thread count, 3/4 staged
  int a_var;        // plane-forward pass: 1 default threads, 2 the second thread count, 3 wave-level x,
                    // 0 automatic (3 in FP64 where the wave-level form exists, else 1)
  int nts;          // the pair volume is read and written with non-temporal hints
  int zsplit = 0;   // plane passes split over the XCDs by z (bit 0: forward, bit 1: inverse) or by unit;
                    // bit 2: the forward pass walks its pairs in 4 x 16 blocks (FP32, not the
                    // wave-level form)
  TrajSegs segs;    // per-target orbital blocks (multi-trajectory launches; n == 0: psi for all)
  int jsplit = 1;   // plane-inverse pass: terms of orbital j go to sum group j mod jsplit
};
// Partial sums of the plane-inverse pass.  With jsplit groups, group g of
// target t lives at acc + g * gstride + t * ld_acc and `last` is never set:
// the groups are added afterwards (vx_combine_groups).
template <typename A>
struct CtAcc {
  cpx<A>* acc;
  int64_t ld_acc;
  int first;
  void* out;
  int64_t ld_out;
  int out_c64, last, pipe;
  int64_t gstride = 0;
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
// Grid tables (twiddles, fold maps, the kernel on the folded grid) for one
// cell, kernel and table precision (0 FP64, 1 FP32), carved from the arena
// of `ws` and filled on `st` by a device kernel (noalloc.hip).
fx_status scratch_tables(Workspace* ws, const fx_cell* cell, const fx_kernel* kern, int prec, const PlanSet* plans,
                         hipStream_t st, GridTables* out);

}  // namespace fx
