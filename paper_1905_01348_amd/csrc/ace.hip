// ACE operator: build from W = V_X Psi and apply K_ACE phi = -xi (xi^H phi).
// (ACE is cited in the paper's introduction as an alternative to applying
// V_X directly; the factorisation follows its standard definition: M = Psi^H W,
// -M = L L^H, xi = W L^{-H}.)
#include <algorithm>
#include <cstring>

#include "ace.hpp"
#include "linalg.hpp"
#include "mfma_gemm.hpp"
#include "vx.hpp"

using namespace fx;

namespace fx {

static void ace_release(fx_ace* a) {
  fx_ctx* ctx = a->ctx;
  for (auto& b : a->owned) ctx_free(ctx, b.first, b.second);
  a->owned.clear();
  ws_release(ctx, &a->ws);
}

void ace_detach_all(fx_ctx* ctx) {
  for (fx_ace* a : ctx->aces) {
    ace_release(a);
    a->ctx = nullptr;
  }
  ctx->aces.clear();
}

fx_status ace_alloc(fx_ace* a, size_t bytes, void** out) {
  FX_TRY(ctx_alloc(a->ctx, bytes, out));
  a->owned.push_back({*out, bytes});
  return FX_OK;
}

fx_status ace_build_impl(fx_ctx* ctx, Workspace* ws, const fx_cell* cell, const fx_kernel* kern, const void* psi,
                         int n, int64_t ld, fx_dtype in_dtype, fx_prec vx_prec, fx_prec ace_prec, hipStream_t st,
                         fx_ace** out, double* ex_host, double* ex_dev_out) {
  FX_TRY(check_cell(cell));
  FX_TRY(check_kernel(kern));
  if (!out) FX_FAIL(FX_ERR_INVALID, "ace is NULL");
  *out = nullptr;
  if (!psi) FX_FAIL(FX_ERR_INVALID, "psi is NULL");
  const int64_t nr = (int64_t)cell->n[0] * cell->n[1] * cell->n[2];
  if (n <= 0) FX_FAIL(FX_ERR_INVALID, "n_psi = %d must be positive", n);
  if (n > 4096) FX_FAIL(FX_ERR_UNSUPPORTED, "n_psi = %d exceeds 4096", n);
  if (ld < nr) FX_FAIL(FX_ERR_INVALID, "ld_psi = %lld < N_r = %lld", (long long)ld, (long long)nr);
  if (in_dtype != FX_C128 && in_dtype != FX_C64) FX_FAIL(FX_ERR_UNSUPPORTED, "unknown in_dtype %d", in_dtype);
  if (vx_prec != FX_PREC_FP64 && vx_prec != FX_PREC_FP32 && vx_prec != FX_PREC_FP32_ACC64)
    FX_FAIL(FX_ERR_UNSUPPORTED, "vx_prec %d is not a V_X precision", vx_prec);
  if (ace_prec < FX_PREC_ACE_FP64 || ace_prec > FX_PREC_ACE_FP16)
    FX_FAIL(FX_ERR_UNSUPPORTED, "ace_prec %d is not an ACE precision", ace_prec);

  fx_ace* a = new fx_ace();
  a->ctx = ctx;
  a->n = n;
  a->nr = nr;
  a->cell = *cell;
  a->kern = *kern;
  a->prec = ace_prec;
  auto fail = [&](fx_status s) {
    ace_release(a);
    delete a;
    return s;
  };
  const size_t zsz = 16;
  void *W = nullptr, *psi64 = nullptr;
  fx_status s = FX_OK;
  // W = V_X Psi, FP64 output
  if ((s = ace_alloc(a, zsz * nr * n, &W)) != FX_OK) return fail(s);
  {
    VxArgs va;
    va.cell = cell;
    va.kern = kern;
    va.psi = psi;
    va.n_psi = n;
    va.ld_psi = ld;
    va.phi = psi;
    va.n_phi = n;
    va.ld_phi = ld;
    va.out = W;
    va.ld_out = nr;
    va.in_dtype = in_dtype;
    va.out_dtype = FX_C128;
    va.prec = vx_prec;
    if ((s = vx_apply(ctx, ws, va, st, nullptr)) != FX_OK) return fail(s);
  }
  int64_t ldp = ld;
  if (in_dtype == FX_C64) {
    if ((s = ws_get(ctx, ws, "ace_psi64", zsz * nr * n, &psi64)) != FX_OK) return fail(s);
    if ((s = convert_cols(psi, FX_C64, ld, psi64, FX_C128, nr, nr, n, st)) != FX_OK) return fail(s);
    ldp = nr;
  } else {
    psi64 = const_cast<void*>(psi);
  }
  // M = Psi^H W  (FP64), Hermitised into a->M; -M into the Cholesky buffer
  void *Mraw = nullptr, *Aneg = nullptr, *scal = nullptr;
  if ((s = ace_alloc(a, zsz * n * n, &a->M)) != FX_OK) return fail(s);
  if ((s = ace_alloc(a, zsz * n * n, &a->L)) != FX_OK) return fail(s);
  if ((s = ws_get(ctx, ws, "ace_Mraw", zsz * n * n, &Mraw)) != FX_OK) return fail(s);
  if ((s = ws_get(ctx, ws, "ace_scal", 64, &scal)) != FX_OK) return fail(s);
  if ((s = zgemm(ctx, ws, st, 1, 0, n, n, (int)nr, cpx<double>{1, 0}, psi64, ldp, W, nr, cpx<double>{0, 0}, Mraw, n,
                 1, 0, 0, 0, 0)) != FX_OK)
    return fail(s);
  Aneg = a->L;
  double* ex_dev = (double*)scal;
  int* info_dev = (int*)((char*)scal + 32);
  // the info flag must start at zero; a 4-byte fill kernel would do as well,
  // but this call is never captured (it waits on the host below)
  if (hipMemsetAsync(info_dev, 0, sizeof(int), st) != hipSuccess) return fail(FX_ERR_DEVICE);
  if ((s = zherm(st, n, Mraw, n, a->M, Aneg, ex_dev)) != FX_OK) return fail(s);
  if (ex_dev_out && hipMemcpyAsync(ex_dev_out, ex_dev, sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(FX_ERR_DEVICE);
  // -M = L L^H
  if ((s = zpotrf(ctx, ws, st, n, a->L, n, info_dev)) != FX_OK) return fail(s);
  double ex = 0.0;
  int info = 0;
  if (hipMemcpyAsync(&ex, ex_dev, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&info, info_dev, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    set_error("device error during the ACE build");
    return fail(FX_ERR_DEVICE);
  }
  a->ex = ex;
  if (ex_host) *ex_host = ex;
  if (info != 0) {
    set_error("-M is not positive definite (pivot %d of %d); ACE needs a negative definite Psi^H V_X Psi", info, n);
    return fail(FX_ERR_NOT_POSDEF);
  }
  // xi = W L^{-H}: Linv = L^{-1}, LinvH = Linv^H, xi = W LinvH
  void *Linv = nullptr, *LinvH = nullptr;
  if ((s = ws_get(ctx, ws, "ace_Linv", zsz * n * n, &Linv)) != FX_OK) return fail(s);
  if ((s = ws_get(ctx, ws, "ace_LinvH", zsz * n * n, &LinvH)) != FX_OK) return fail(s);
  if (hipMemcpyAsync(Linv, a->L, zsz * n * n, hipMemcpyDeviceToDevice, st) != hipSuccess) return fail(FX_ERR_DEVICE);
  if ((s = ztrinv(ctx, ws, st, n, Linv, n)) != FX_OK) return fail(s);
  if ((s = zconj_transpose(st, n, Linv, n, LinvH, n)) != FX_OK) return fail(s);
  if ((s = ace_alloc(a, zsz * nr * n, &a->xi)) != FX_OK) return fail(s);
  if ((s = zgemm(ctx, ws, st, 0, 0, (int)nr, n, n, cpx<double>{1, 0}, W, nr, LinvH, n, cpx<double>{0, 0}, a->xi, nr,
                 1, 0, 0, 0, 1)) != FX_OK)
    return fail(s);
  // W is no longer needed
  if (hipStreamSynchronize(st) != hipSuccess) return fail(FX_ERR_DEVICE);
  for (auto it = a->owned.begin(); it != a->owned.end(); ++it)
    if (it->first == W) {
      ctx_free(ctx, it->first, it->second);
      a->owned.erase(it);
      break;
    }
  // split forms for the requested precision
  if (ace_prec != FX_PREC_ACE_FP64) {
    if ((s = ace_prepare_split(a, ace_prec, st)) != FX_OK) return fail(s);
  }
  *out = a;
  return FX_OK;
}

fx_status ace_apply_impl(fx_ctx* ctx, Workspace* ws, const fx_ace* ac, const void* phi, int nphi, int64_t ld_phi,
                         void* out, int64_t ld_out, fx_dtype in_dtype, fx_dtype out_dtype, fx_prec prec,
                         hipStream_t st) {
  if (!ac) FX_FAIL(FX_ERR_INVALID, "ace is NULL");
  fx_ace* a = const_cast<fx_ace*>(ac);
  const int64_t nr = a->nr;
  const int n = a->n;
  if (!phi || !out) FX_FAIL(FX_ERR_INVALID, "phi and out must be non-NULL");
  if (nphi <= 0) FX_FAIL(FX_ERR_INVALID, "n_phi = %d must be positive", nphi);
  if (ld_phi < nr || ld_out < nr) FX_FAIL(FX_ERR_INVALID, "leading dimensions must be >= N_r = %lld", (long long)nr);
  if (in_dtype != FX_C128 && in_dtype != FX_C64) FX_FAIL(FX_ERR_UNSUPPORTED, "unknown in_dtype %d", in_dtype);
  if (out_dtype != FX_C128 && out_dtype != FX_C64) FX_FAIL(FX_ERR_UNSUPPORTED, "unknown out_dtype %d", out_dtype);
  if (prec < FX_PREC_ACE_FP64 || prec > FX_PREC_ACE_FP16)
    FX_FAIL(FX_ERR_UNSUPPORTED, "precision %d is not an ACE precision", prec);
  {
    const size_t isz = dtype_size(in_dtype), osz = dtype_size(out_dtype);
    const char* o0 = (const char*)out;
    const char* o1 = o0 + ((size_t)(nphi - 1) * ld_out + nr) * osz;
    const char* i0 = (const char*)phi;
    const char* i1 = i0 + ((size_t)(nphi - 1) * ld_phi + nr) * isz;
    if (o0 < i1 && i0 < o1) FX_FAIL(FX_ERR_INVALID, "out overlaps phi");
  }
  const size_t zsz = 16;
  if (prec == FX_PREC_ACE_FP64) {
    const void* p64 = phi;
    int64_t ldp = ld_phi;
    if (in_dtype == FX_C64) {
      void* t = nullptr;
      FX_TRY(ws_get(ctx, ws, "acea_phi64", zsz * nr * nphi, &t));
      FX_TRY(convert_cols(phi, FX_C64, ld_phi, t, FX_C128, nr, nr, nphi, st));
      p64 = t;
      ldp = nr;
    }
    void* C = nullptr;
    FX_TRY(ws_get(ctx, ws, "acea_C", zsz * n * nphi, &C));
    // split count fixed by N_r alone: results do not depend on n_phi
    const int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(64, nr / 8192));
    FX_TRY(zgemm(ctx, ws, st, 1, 0, n, nphi, (int)nr, cpx<double>{1, 0}, a->xi, nr, p64, ldp, cpx<double>{0, 0}, C, n,
                 1, 0, 0, 0, nsplit));
    void* y = out;
    int64_t ldy = ld_out;
    if (out_dtype == FX_C64) {
      FX_TRY(ws_get(ctx, ws, "acea_y64", zsz * nr * nphi, &y));
      ldy = nr;
    }
    FX_TRY(zgemm(ctx, ws, st, 0, 0, (int)nr, nphi, n, cpx<double>{-1, 0}, a->xi, nr, C, n, cpx<double>{0, 0}, y, ldy,
                 1, 0, 0, 0, 1));
    if (out_dtype == FX_C64) FX_TRY(convert_cols(y, FX_C128, nr, out, FX_C64, ld_out, nr, nphi, st));
    return FX_OK;
  }
  return ace_apply_mfma(ctx, ws, a, phi, nphi, ld_phi, out, ld_out, in_dtype, out_dtype, prec, st);
}

}  // namespace fx

extern "C" {

fx_status fx_build_ace(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel, const void* psi, int32_t n_psi,
                       int64_t ld_psi, fx_dtype in_dtype, fx_prec vx_prec, fx_prec ace_prec, void* stream,
                       fx_ace** ace, double* ex_energy_dev) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
  FX_TRY(note_capture(ctx, (hipStream_t)stream));
  if (ctx->capturing) FX_FAIL(FX_ERR_INVALID, "fx_build_ace waits on its stream and cannot be captured");
  FX_TRY(ace_build_impl(ctx, &ctx->ws, cell, kernel, psi, n_psi, ld_psi, in_dtype, vx_prec, ace_prec,
                        (hipStream_t)stream, ace, nullptr, ex_energy_dev));
  ctx->aces.insert(*ace);
  return FX_OK;
}

fx_status fx_apply_ace(fx_ctx* ctx, const fx_ace* ace, const void* phi, int32_t n_phi, int64_t ld_phi, void* out,
                       int64_t ld_out, fx_dtype in_dtype, fx_dtype out_dtype, fx_prec prec, void* stream) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  if (!ace) FX_FAIL(FX_ERR_INVALID, "ace is NULL");
  if (!ace->ctx) FX_FAIL(FX_ERR_INVALID, "the context of this ACE handle was finalized");
  if (ace->ctx != ctx) FX_FAIL(FX_ERR_INVALID, "ace was built on another context");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
  FX_TRY(note_capture(ctx, (hipStream_t)stream));
  auto body = [&](hipStream_t s) {
    return ace_apply_impl(ctx, &const_cast<fx_ace*>(ace)->ws, ace, phi, n_phi, ld_phi, out, ld_out, in_dtype,
                          out_dtype, prec, s);
  };
  if (ctx->graph_max <= 0) return body((hipStream_t)stream);
  KeyBytes k;
  k.add(1).add(ace).add(phi).add(n_phi).add(ld_phi).add(out).add(ld_out).add(in_dtype).add(out_dtype).add(prec);
  return graph_call(ctx, k.b, (hipStream_t)stream, body);
}

fx_status fx_ace_export(const fx_ace* ace, void* xi, void* L, void* M) {
  clear_error();
  if (!ace) FX_FAIL(FX_ERR_INVALID, "ace is NULL");
  if (!ace->ctx) FX_FAIL(FX_ERR_INVALID, "the context of this ACE handle was finalized");
  const size_t nn = (size_t)ace->n * ace->n * 16;
  FX_HIP(hipDeviceSynchronize());
  if (xi) FX_HIP(hipMemcpy(xi, ace->xi, (size_t)ace->nr * ace->n * 16, hipMemcpyDeviceToDevice));
  if (L) FX_HIP(hipMemcpy(L, ace->L, nn, hipMemcpyDeviceToDevice));
  if (M) FX_HIP(hipMemcpy(M, ace->M, nn, hipMemcpyDeviceToDevice));
  return FX_OK;
}

fx_status fx_ace_shape(const fx_ace* ace, int32_t* n, int64_t* n_r) {
  clear_error();
  if (!ace) FX_FAIL(FX_ERR_INVALID, "ace is NULL");
  if (n) *n = ace->n;
  if (n_r) *n_r = ace->nr;
  return FX_OK;
}

fx_status fx_ace_free(fx_ace* ace) {
  clear_error();
  if (!ace) FX_FAIL(FX_ERR_INVALID, "ace is NULL");
  // a handle whose context was finalized holds no device memory any more
  if (fx_ctx* ctx = ace->ctx) {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    FX_HIP(hipSetDevice(ctx->device));
    FX_HIP(hipDeviceSynchronize());
    ace_release(ace);
    ctx->aces.erase(ace);
  }
  delete ace;
  return FX_OK;
}

}  // extern "C"
