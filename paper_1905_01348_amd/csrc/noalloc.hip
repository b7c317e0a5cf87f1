// Allocation-free form of the V_X application (fx_apply_vx_noalloc), for
// callers that cannot allocate device memory: code under HIP graph capture,
// serving loops that must not call hipMalloc, harnesses that forbid it.
//
// Everything the call needs beyond its inputs and output lives in one
// file-scope device array, `scratch`, of kScratchBytes.  Each device the
// library runs on holds its own copy of the array (from the load of the code
// object until the process ends), at its own address: fx_init looks that
// address up once per device with hipGetSymbolAddress and host code uses
// only that address, never the array's name (which is a host-side stand-in
// in host code).  Inside one call the scratch region is carved, in order,
// into the grid tables (built on the device by k_build_tables), the pair
// work volume, the partial sums (only when `out` cannot hold them) and the
// energy partials.  Every buffer is fully written before it is read, so
// nothing has to start at zero.  All calls on one device share its copy:
// calls that overlap in time on one device (other streams, other host
// threads, other contexts) race on it.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "vx.hpp"

namespace fx {

constexpr size_t kScratchBytes = FX_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
constexpr int kMaxEdge = 96;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {nullptr};

fx_status scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) FX_FAIL(FX_ERR_UNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return FX_OK;
  int cur = -1;
  FX_HIP(hipGetDevice(&cur));
  if (cur != device) FX_FAIL(FX_ERR_INVALID, "scratch set-up for device %d while device %d is current", device, cur);
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    FX_FAIL(FX_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device, hipGetErrorString(e));
  g_scratch_ptr[device] = p;
  return FX_OK;
}

static void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

// Everything the table kernel needs, passed by value (about 1.3 KB).
struct TableArgs {
  int n[3];
  int h[3];  // n/2 + 1: the folded grid
  double len[3];
  int kind;
  double omega, scale, vol;
  int fold[3][kMaxEdge];  // folded frequency |m| held at each digit-reversed position
};

__device__ static double kernel_of(int kind, double omega, double g2) {
  const double pi = 3.14159265358979323846264338327950288;
  if (g2 == 0.0) return kind == FX_COULOMB ? 0.0 : pi / (omega * omega);
  double v = 4.0 * pi / g2;
  if (kind == FX_HSE) v *= -expm1(-g2 / (4.0 * omega * omega));
  return v;
}

// Twiddles w_n^t = exp(-2 pi i t/n) per axis, the fold maps, and
// K(G) * (-scale/Omega) on the folded grid, all computed in FP64 and stored
// in the table precision T.  The same quantities as the host-built tables of
// the other entry points (Sec. 2: the Coulomb or screened kernel on the
// reciprocal grid G = 2 pi m / L).
template <typename T>
__global__ void k_build_tables(TableArgs a, cpx<T>* tw0, cpx<T>* tw1, cpx<T>* tw2, int* f0, int* f1, int* f2,
                               T* kf) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  cpx<T>* tw[3] = {tw0, tw1, tw2};
  int* fo[3] = {f0, f1, f2};
  for (int ax = 0; ax < 3; ++ax)
    for (int i = tid; i < a.n[ax]; i += nth) {
      double s, c;
      sincospi(2.0 * (double)i / (double)a.n[ax], &s, &c);
      tw[ax][i] = cpx<T>{(T)c, (T)(-s)};
      fo[ax][i] = a.fold[ax][i];
    }
  const double pi = 3.14159265358979323846264338327950288;
  const int64_t total = (int64_t)a.h[0] * a.h[1] * a.h[2];
  for (int64_t e = tid; e < total; e += nth) {
    const int x = (int)(e % a.h[0]);
    const int y = (int)((e / a.h[0]) % a.h[1]);
    const int z = (int)(e / ((int64_t)a.h[0] * a.h[1]));
    const double gx = 2 * pi * x / a.len[0], gy = 2 * pi * y / a.len[1], gz = 2 * pi * z / a.len[2];
    const double g2 = gx * gx + gy * gy + gz * gz;
    kf[e] = (T)(-a.scale / a.vol * kernel_of(a.kind, a.omega, g2));
  }
}

fx_status scratch_tables(Workspace* ws, const fx_cell* cell, const fx_kernel* kern, int prec, const PlanSet* plans,
                         hipStream_t st, GridTables* out) {
  PlanSet ps;
  if (plans)
    ps = *plans;
  else
    default_plans(cell, &ps);
  TableArgs ta;
  for (int ax = 0; ax < 3; ++ax) {
    const int n = cell->n[ax];
    if (n > kMaxEdge) FX_FAIL(FX_ERR_UNSUPPORTED, "edge %d above %d", n, kMaxEdge);
    ta.n[ax] = n;
    ta.h[ax] = n / 2 + 1;
    ta.len[ax] = cell->len[ax];
    std::vector<int> fp;
    plan_positions(ps.ax[ax], &fp);
    for (int i = 0; i < kMaxEdge; ++i) ta.fold[ax][i] = i < n ? (fp[i] <= n - fp[i] ? fp[i] : n - fp[i]) : 0;
  }
  ta.kind = kern->kind;
  ta.omega = kern->omega;
  ta.scale = kern->scale;
  ta.vol = cell->len[0] * cell->len[1] * cell->len[2];
  const size_t tsz = prec == 0 ? 16 : 8, rsz = prec == 0 ? 8 : 4;
  GridTables t;
  static const char* twn[3] = {"nat_tw0", "nat_tw1", "nat_tw2"};
  static const char* fon[3] = {"nat_fold0", "nat_fold1", "nat_fold2"};
  for (int ax = 0; ax < 3; ++ax) {
    FX_TRY(ws_get(nullptr, ws, twn[ax], (size_t)ta.n[ax] * tsz, &t.tw[ax]));
    void* f = nullptr;
    FX_TRY(ws_get(nullptr, ws, fon[ax], (size_t)ta.n[ax] * sizeof(int), &f));
    t.fold[ax] = (int*)f;
  }
  FX_TRY(ws_get(nullptr, ws, "nat_kfold", (size_t)ta.h[0] * ta.h[1] * ta.h[2] * rsz, &t.kfold));
  const int64_t total = (int64_t)ta.h[0] * ta.h[1] * ta.h[2];
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 1024));
  if (prec == 0)
    hipLaunchKernelGGL(k_build_tables<double>, dim3(blocks), dim3(256), 0, st, ta, (cpx<double>*)t.tw[0],
                       (cpx<double>*)t.tw[1], (cpx<double>*)t.tw[2], t.fold[0], t.fold[1], t.fold[2],
                       (double*)t.kfold);
  else
    hipLaunchKernelGGL(k_build_tables<float>, dim3(blocks), dim3(256), 0, st, ta, (cpx<float>*)t.tw[0],
                       (cpx<float>*)t.tw[1], (cpx<float>*)t.tw[2], t.fold[0], t.fold[1], t.fold[2],
                       (float*)t.kfold);
  FX_LAUNCH_CHECK();
  *out = t;
  return FX_OK;
}

}  // namespace fx

using namespace fx;

extern "C" {

fx_status fx_apply_vx_noalloc(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel, const void* psi,
                              int32_t n_psi, int64_t ld_psi, const void* phi, int32_t n_phi, int64_t ld_phi, void* out,
                              int64_t ld_out, fx_dtype in_dtype, fx_dtype out_dtype, fx_prec prec, void* stream,
                              double* ex_energy_dev) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
  void* base = scratch_ptr(ctx->device);
  if (!base) FX_FAIL(FX_ERR_INVALID, "no scratch region set up for device %d", ctx->device);
  VxArgs a;
  a.cell = cell;
  a.kern = kernel;
  a.psi = psi;
  a.n_psi = n_psi;
  a.ld_psi = ld_psi;
  a.phi = phi;
  a.n_phi = n_phi;
  a.ld_phi = ld_phi;
  a.out = out;
  a.ld_out = ld_out;
  a.in_dtype = in_dtype;
  a.out_dtype = out_dtype;
  a.prec = prec;
  a.ex_dev = ex_energy_dev;
  a.no_alloc = true;
  hipStream_t st = (hipStream_t)stream;
  FX_TRY(note_capture(ctx, st));
  Workspace ws;
  ws.arena = (char*)base;
  ws.arena_bytes = kScratchBytes;
  return vx_apply(ctx, &ws, a, st, nullptr);
}

}  // extern "C"
