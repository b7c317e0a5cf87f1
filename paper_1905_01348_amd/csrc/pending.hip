// Entry points whose implementation is still being written: they report
// FX_ERR_UNSUPPORTED.
#include "common.hpp"

using namespace fx;

extern "C" {
fx_status fx_serve_create(fx_ctx*, const fx_serve_cfg*, fx_server**) { FX_FAIL(FX_ERR_UNSUPPORTED, "not available"); }
fx_status fx_serve_register(fx_server*, int32_t, const fx_cell*, const fx_kernel*, const void*, int32_t, int64_t,
                            fx_dtype, fx_prec, fx_prec) {
  FX_FAIL(FX_ERR_UNSUPPORTED, "not available");
}
fx_status fx_serve(fx_server*, const fx_request*, int32_t, fx_status*, double*, fx_serve_report*) {
  FX_FAIL(FX_ERR_UNSUPPORTED, "not available");
}
fx_status fx_serve_destroy(fx_server*) { FX_FAIL(FX_ERR_UNSUPPORTED, "not available"); }
}
