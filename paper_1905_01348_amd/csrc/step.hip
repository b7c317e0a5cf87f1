// The operations at the end of a PT-CN step: the residual of the fixed-point
// equation (the residual algorithm of Sec. 3.3), the Cholesky-QR
// re-orthonormalisation of the orbitals and the electron density (Sec. 3.4);
// and the kinetic operator -(1/2) Laplacian of the Hamiltonian (Sec. 2),
// which a residual may add to H.  All arithmetic is FP64; complex64 blocks
// are widened on the way in and rounded on the way out.
#include <algorithm>

#include "common.hpp"
#include "linalg.hpp"
#include "vx.hpp"

namespace fx {

// r = psi - half + (i hdt) hpsi, all FP64, column c at base + c*ld.
__global__ void __launch_bounds__(256) k_residual_init(const cpx<double>* __restrict__ psi, int64_t ldp,
                                                       const cpx<double>* __restrict__ hpsi, int64_t ldh,
                                                       const cpx<double>* __restrict__ half, int64_t ldf,
                                                       cpx<double>* __restrict__ r, int64_t ldr, int64_t nr, int n,
                                                       double hdt) {
  const int64_t total = nr * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = i / nr, e = i - c * nr;
    const cpx<double> p = psi[c * ldp + e], h = hpsi[c * ldh + e], f = half[c * ldf + e];
    r[c * ldr + e] = cpx<double>{p.x - f.x - hdt * h.y, p.y - f.y + hdt * h.x};
  }
}

// dst += src, n columns of nr FP64 complex values.
__global__ void __launch_bounds__(256) k_add_cols(cpx<double>* __restrict__ dst, int64_t ldd,
                                                  const cpx<double>* __restrict__ src, int64_t lds, int64_t nr, int n) {
  const int64_t total = nr * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = i / nr, e = i - c * nr;
    const cpx<double> a = dst[c * ldd + e], b = src[c * lds + e];
    dst[c * ldd + e] = cpx<double>{a.x + b.x, a.y + b.y};
  }
}

// the constant 1 at nr points
template <typename T>
__global__ void __launch_bounds__(256) k_fill_one(cpx<T>* __restrict__ p, int64_t nr) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nr; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = cpx<T>{(T)1, (T)0};
}

// rho[e] = sum_c f_c |psi_c[e]|^2 over c ascending, FP64 (f = 1 if occ is null).
template <typename T>
__global__ void __launch_bounds__(256) k_density(const cpx<T>* __restrict__ psi, int64_t ld, int n, int64_t nr,
                                                 const double* __restrict__ occ, double* __restrict__ rho) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nr; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < n; ++c) {
      const cpx<T> v = psi[c * ld + e];
      const double m = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
      acc += occ ? occ[c] * m : m;
    }
    rho[e] = acc;
  }
}

static int grid_for(int64_t total) { return (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 16384)); }

// A block as FP64: the input itself, or a widened copy in workspace `name`.
static fx_status as_c128(fx_ctx* ctx, Workspace* ws, const char* name, const void* p, int64_t ld, fx_dtype dt,
                         int64_t nr, int n, hipStream_t st, const void** out, int64_t* ld_out) {
  if (dt == FX_C128) {
    *out = p;
    *ld_out = ld;
    return FX_OK;
  }
  void* q = nullptr;
  FX_TRY(ws_get(ctx, ws, name, (size_t)16 * nr * n, &q));
  FX_TRY(convert_cols(p, FX_C64, ld, q, FX_C128, nr, nr, n, st));
  *out = q;
  *ld_out = nr;
  return FX_OK;
}

static fx_status check_block(const void* p, int n, int64_t ld, int64_t nr, fx_dtype dt, const char* what) {
  if (!p) FX_FAIL(FX_ERR_INVALID, "%s is NULL", what);
  if (n <= 0 || nr <= 0) FX_FAIL(FX_ERR_INVALID, "%s: n = %d and N_r = %lld must be positive", what, n, (long long)nr);
  if (ld < nr) FX_FAIL(FX_ERR_INVALID, "%s: leading dimension %lld < N_r = %lld", what, (long long)ld, (long long)nr);
  if (dt != FX_C128 && dt != FX_C64) FX_FAIL(FX_ERR_UNSUPPORTED, "%s: unknown dtype %d", what, dt);
  return FX_OK;
}

static bool overlaps(const void* a, int n, int64_t lda, const void* b, int m, int64_t ldb, int64_t nr, size_t esz) {
  const char* a0 = (const char*)a;
  const char* a1 = a0 + ((size_t)(n - 1) * lda + nr) * esz;
  const char* b0 = (const char*)b;
  const char* b1 = b0 + ((size_t)(m - 1) * ldb + nr) * esz;
  return a0 < b1 && b0 < a1;
}

// out = -(1/2) Laplacian phi on the periodic grid: each planewave coefficient
// times |G|^2/2 (Sec. 2).  It is the pair path with the constant orbital 1 as
// its only psi and |G|^2/(2 N_r) as its kernel, in FP64: conj(1) phi = phi,
// the FFT, the symbol, the inverse FFT, times 1.
static fx_status apply_kinetic(fx_ctx* ctx, Workspace* ws, const fx_cell* cell, const void* phi, int n,
                               int64_t ld, fx_dtype din, void* out, int64_t ld_out, fx_dtype dout, hipStream_t st) {
  FX_TRY(check_cell(cell));
  if (din != FX_C128 && din != FX_C64) FX_FAIL(FX_ERR_UNSUPPORTED, "unknown in_dtype %d", din);
  const int64_t nr = (int64_t)cell->n[0] * cell->n[1] * cell->n[2];
  void* ones = nullptr;
  FX_TRY(ws_get(ctx, ws, "kin_ones", dtype_size(din) * (size_t)nr, &ones));
  if (din == FX_C128)
    hipLaunchKernelGGL(k_fill_one<double>, dim3(grid_for(nr)), dim3(256), 0, st, (cpx<double>*)ones, nr);
  else
    hipLaunchKernelGGL(k_fill_one<float>, dim3(grid_for(nr)), dim3(256), 0, st, (cpx<float>*)ones, nr);
  FX_LAUNCH_CHECK();
  const fx_kernel kk{kKineticKind, 0.0, 1.0};
  VxArgs va;
  va.cell = cell;
  va.kern = &kk;
  va.internal_kernel = true;
  va.psi = ones;
  va.n_psi = 1;
  va.ld_psi = nr;
  va.phi = phi;
  va.n_phi = n;
  va.ld_phi = ld;
  va.out = out;
  va.ld_out = ld_out;
  va.in_dtype = din;
  va.out_dtype = dout;
  va.prec = FX_PREC_FP64;
  return vx_apply(ctx, ws, va, st, nullptr);
}

static fx_status pt_residual(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kern, const void* psi,
                             const void* hpsi, const void* half, int n, int64_t ld, fx_dtype dt, double dtime,
                             fx_prec vx_prec, int kinetic, void* r, int64_t ldr, void* s_out, hipStream_t st) {
  FX_TRY(check_cell(cell));
  const int64_t nr = (int64_t)cell->n[0] * cell->n[1] * cell->n[2];
  FX_TRY(check_block(psi, n, ld, nr, dt, "psi"));
  FX_TRY(check_block(half, n, ld, nr, dt, "psi_half"));
  FX_TRY(check_block(r, n, ldr, nr, dt, "r_out"));
  if (hpsi) FX_TRY(check_block(hpsi, n, ld, nr, dt, "hpsi"));
  const size_t esz = dtype_size(dt);
  for (const void* in : {psi, hpsi, half})
    if (in && overlaps(r, n, ldr, in, n, ld, nr, esz)) FX_FAIL(FX_ERR_INVALID, "r_out overlaps an input block");
  if (!(dtime == dtime)) FX_FAIL(FX_ERR_INVALID, "dt is NaN");
  Workspace* ws = &ctx->ws;
  const void *p64, *h64, *f64;
  int64_t ldp, ldh, ldf;
  FX_TRY(as_c128(ctx, ws, "pt_psi", psi, ld, dt, nr, n, st, &p64, &ldp));
  FX_TRY(as_c128(ctx, ws, "pt_half", half, ld, dt, nr, n, st, &f64, &ldf));
  if (hpsi) {
    FX_TRY(as_c128(ctx, ws, "pt_hpsi", hpsi, ld, dt, nr, n, st, &h64, &ldh));
  } else {
    // H = V_X: H Psi by the pair path (phi == psi, FP64 output)
    FX_TRY(check_kernel(kern));
    void* w = nullptr;
    FX_TRY(ws_get(ctx, ws, "pt_hpsi", (size_t)16 * nr * n, &w));
    VxArgs va;
    va.cell = cell;
    va.kern = kern;
    va.psi = psi;
    va.n_psi = n;
    va.ld_psi = ld;
    va.phi = psi;
    va.n_phi = n;
    va.ld_phi = ld;
    va.out = w;
    va.ld_out = nr;
    va.in_dtype = dt;
    va.out_dtype = FX_C128;
    va.prec = vx_prec;
    FX_TRY(vx_apply(ctx, ws, va, st, nullptr));
    h64 = w;
    ldh = nr;
  }
  if (kinetic) {
    // H Psi + T Psi in a buffer of the library's (hpsi may be the caller's)
    void* kin = nullptr;
    FX_TRY(ws_get(ctx, ws, "pt_kin", (size_t)16 * nr * n, &kin));
    FX_TRY(apply_kinetic(ctx, ws, cell, psi, n, ld, dt, kin, nr, FX_C128, st));
    hipLaunchKernelGGL(k_add_cols, dim3(grid_for(nr * n)), dim3(256), 0, st, (cpx<double>*)kin, nr,
                       (const cpx<double>*)h64, ldh, nr, n);
    FX_LAUNCH_CHECK();
    h64 = kin;
    ldh = nr;
  }
  // S = Psi^H (H Psi), N x N, FP64 (split over N_r with a fixed-order reduction)
  void* S = s_out;
  if (!S) FX_TRY(ws_get(ctx, ws, "pt_S", (size_t)16 * n * n, &S));
  FX_TRY(zgemm(ctx, ws, st, 1, 0, n, n, (int)nr, cpx<double>{1, 0}, p64, ldp, h64, ldh, cpx<double>{0, 0}, S, n, 1, 0,
               0, 0, 0));
  // R = Psi - Psi_half + (i dt/2) H Psi, then R += (-i dt/2) Psi S
  void* r64 = r;
  int64_t ldr64 = ldr;
  if (dt == FX_C64) {
    FX_TRY(ws_get(ctx, ws, "pt_r64", (size_t)16 * nr * n, &r64));
    ldr64 = nr;
  }
  const double hdt = 0.5 * dtime;
  hipLaunchKernelGGL(k_residual_init, dim3(grid_for(nr * n)), dim3(256), 0, st, (const cpx<double>*)p64, ldp,
                     (const cpx<double>*)h64, ldh, (const cpx<double>*)f64, ldf, (cpx<double>*)r64, ldr64, nr, n, hdt);
  FX_LAUNCH_CHECK();
  FX_TRY(zgemm(ctx, ws, st, 0, 0, (int)nr, n, n, cpx<double>{0, -hdt}, p64, ldp, S, n, cpx<double>{1, 0}, r64, ldr64,
               1, 0, 0, 0, 1));
  if (dt == FX_C64) FX_TRY(convert_cols(r64, FX_C128, ldr64, r, FX_C64, ldr, nr, n, st));
  return FX_OK;
}

static fx_status orthonormalize(fx_ctx* ctx, void* psi, int n, int64_t ld, int64_t nr, fx_dtype dt, hipStream_t st) {
  FX_TRY(check_block(psi, n, ld, nr, dt, "psi"));
  Workspace* ws = &ctx->ws;
  const size_t zsz = 16;
  const void* p64;
  int64_t ldp;
  FX_TRY(as_c128(ctx, ws, "on_psi", psi, ld, dt, nr, n, st, &p64, &ldp));
  void *S = nullptr, *L = nullptr, *scratch = nullptr, *LinvH = nullptr, *Q = nullptr, *scal = nullptr;
  FX_TRY(ws_get(ctx, ws, "on_S", zsz * n * n, &S));
  FX_TRY(ws_get(ctx, ws, "on_L", zsz * n * n, &L));
  FX_TRY(ws_get(ctx, ws, "on_neg", zsz * n * n, &scratch));
  FX_TRY(ws_get(ctx, ws, "on_LinvH", zsz * n * n, &LinvH));
  FX_TRY(ws_get(ctx, ws, "on_Q", zsz * nr * n, &Q));
  FX_TRY(ws_get(ctx, ws, "on_scal", 64, &scal));
  // S = Psi^H Psi, Hermitised into L, Cholesky S = L L^H in place
  FX_TRY(zgemm(ctx, ws, st, 1, 0, n, n, (int)nr, cpx<double>{1, 0}, p64, ldp, p64, ldp, cpx<double>{0, 0}, S, n, 1, 0,
               0, 0, 0));
  FX_TRY(zherm(st, n, S, n, L, scratch, nullptr));
  int* info_dev = (int*)scal;
  // the info flag must start at zero; this call waits on the host below and
  // is never captured
  FX_HIP(hipMemsetAsync(info_dev, 0, sizeof(int), st));
  FX_TRY(zpotrf(ctx, ws, st, n, L, n, info_dev));
  int info = 0;
  FX_HIP(hipMemcpyAsync(&info, info_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  FX_HIP(hipStreamSynchronize(st));
  if (info != 0)
    FX_FAIL(FX_ERR_NOT_POSDEF, "the overlap Psi^H Psi is not positive definite (pivot %d of %d): the orbitals are "
            "linearly dependent", info, n);
  // Q = Psi L^{-H}, then back into psi
  FX_TRY(ztrinv(ctx, ws, st, n, L, n));
  FX_TRY(zconj_transpose(st, n, L, n, LinvH, n));
  FX_TRY(zgemm(ctx, ws, st, 0, 0, (int)nr, n, n, cpx<double>{1, 0}, p64, ldp, LinvH, n, cpx<double>{0, 0}, Q, nr, 1,
               0, 0, 0, 1));
  FX_TRY(convert_cols(Q, FX_C128, nr, psi, dt, ld, nr, n, st));
  return FX_OK;
}

static fx_status density(const void* psi, int n, int64_t ld, int64_t nr, fx_dtype dt, const double* occ, double* rho,
                         hipStream_t st) {
  FX_TRY(check_block(psi, n, ld, nr, dt, "psi"));
  if (!rho) FX_FAIL(FX_ERR_INVALID, "rho is NULL");
  const int g = grid_for(nr);
  if (dt == FX_C128)
    hipLaunchKernelGGL(k_density<double>, dim3(g), dim3(256), 0, st, (const cpx<double>*)psi, ld, n, nr, occ, rho);
  else
    hipLaunchKernelGGL(k_density<float>, dim3(g), dim3(256), 0, st, (const cpx<float>*)psi, ld, n, nr, occ, rho);
  FX_LAUNCH_CHECK();
  return FX_OK;
}

}  // namespace fx

using namespace fx;

extern "C" {

fx_status fx_apply_kinetic(fx_ctx* ctx, const fx_cell* cell, const void* phi, int32_t n_phi, int64_t ld_phi,
                           void* out, int64_t ld_out, fx_dtype in_dtype, fx_dtype out_dtype, void* stream) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  FX_TRY(note_capture(ctx, st));
  return apply_kinetic(ctx, &ctx->ws, cell, phi, n_phi, ld_phi, in_dtype, out, ld_out, out_dtype, st);
}

fx_status fx_pt_residual(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel, const void* psi, const void* hpsi,
                         const void* psi_half, int32_t n, int64_t ld, fx_dtype dtype, double dt, fx_prec vx_prec,
                         int32_t kinetic, void* r_out, int64_t ld_r, void* s_out, void* stream) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  FX_TRY(note_capture(ctx, st));
  return pt_residual(ctx, cell, kernel, psi, hpsi, psi_half, n, ld, dtype, dt, vx_prec, kinetic, r_out, ld_r, s_out,
                     st);
}

fx_status fx_orthonormalize(fx_ctx* ctx, void* psi, int32_t n, int64_t ld, int64_t nr, fx_dtype dtype, void* stream) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  FX_TRY(note_capture(ctx, st));
  if (ctx->capturing) FX_FAIL(FX_ERR_INVALID, "fx_orthonormalize waits on its stream and cannot be captured");
  return orthonormalize(ctx, psi, n, ld, nr, dtype, st);
}

fx_status fx_density(fx_ctx* ctx, const void* psi, int32_t n, int64_t ld, int64_t nr, fx_dtype dtype,
                     const double* occ, double* rho, void* stream) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
  return density(psi, n, ld, nr, dtype, occ, rho, (hipStream_t)stream);
}

}  // extern "C"
