// fx_apply_vx: V_X applied to a block of targets by batched pair Poisson
// solves (Eq. applyVX; the Fock-application loop of Sec. 3.2 on one GPU's
// band-index share).  Pairs are processed in batches of nk targets x nj
// orbitals; every batch runs the three passes of vx_passes.hpp.
#include <algorithm>
#include <cstdlib>
#include <set>

#include "common.hpp"
#include "vx.hpp"
#include "vx_passes.hpp"

namespace fx {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_pass_a(const cpx<T>* __restrict__ psi, int64_t ld_psi,
                                                const cpx<T>* __restrict__ phi, int64_t ld_phi,
                                                cpx<T>* __restrict__ work, int j0, int nj, int k0, PassGeom g,
                                                const cpx<T>* __restrict__ twx_g, const cpx<T>* __restrict__ twy_g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* s = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twx = s + plane_lds_elems(g);
  cpx<T>* twy = twx + g.nx;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int i = tid; i < g.nx; i += nthr) twx[i] = twx_g[i];
  for (int i = tid; i < g.ny; i += nthr) twy[i] = twy_g[i];
  const int z = blockIdx.x % g.nz;
  const int p = blockIdx.x / g.nz;
  const int j = j0 + p % nj, k = k0 + p / nj;
  const size_t nxy = (size_t)g.nx * g.ny, nr = nxy * g.nz;
  pass_a_body<T>(psi + j * ld_psi + z * nxy, phi + k * ld_phi + z * nxy, work + p * nr + z * nxy, s, twx, twy, g,
                 tid, nthr, DeviceSync{});
}

template <typename T>
__global__ void __launch_bounds__(256) k_pass_b(cpx<T>* __restrict__ work, PassGeom g,
                                                const cpx<T>* __restrict__ twz_g, const T* __restrict__ kfold,
                                                const int* __restrict__ foldx_g, const int* __restrict__ foldy_g,
                                                const int* __restrict__ foldz_g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* s = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twz = s + xz_lds_elems(g);
  int* fxl = reinterpret_cast<int*>(twz + g.nz);
  int* fzl = fxl + g.nx;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int i = tid; i < g.nz; i += nthr) {
    twz[i] = twz_g[i];
    fzl[i] = foldz_g[i];
  }
  for (int i = tid; i < g.nx; i += nthr) fxl[i] = foldx_g[i];
  const int y = blockIdx.x % g.ny;
  const int p = blockIdx.x / g.ny;
  const size_t nr = (size_t)g.nx * g.ny * g.nz;
  pass_b_body<T>(work + p * nr, y, s, twz, kfold, fxl, fzl, foldy_g[y], g, tid, nthr, DeviceSync{});
}

// Pass C.  acc (ld_acc) holds the running sum over j of the targets in the
// accumulation precision A; when `last` is set the final sum goes to `out`
// in its own dtype instead (out may be the same memory as acc).
template <typename T, typename A, int EPT>
__global__ void __launch_bounds__(1024) k_pass_c(const cpx<T>* __restrict__ psi, int64_t ld_psi,
                                                 const cpx<T>* __restrict__ work, int j0, int nj, int k0,
                                                 cpx<A>* acc, int64_t ld_acc, int first, void* out, int64_t ld_out,
                                                 int out_c64, int last, PassGeom g,
                                                 const cpx<T>* __restrict__ twx_g, const cpx<T>* __restrict__ twy_g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* s = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twx = s + plane_lds_elems(g);
  cpx<T>* twy = twx + g.nx;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int i = tid; i < g.nx; i += nthr) twx[i] = twx_g[i];
  for (int i = tid; i < g.ny; i += nthr) twy[i] = twy_g[i];
  const int z = blockIdx.x % g.nz;
  const int kk = blockIdx.x / g.nz;
  const int k = k0 + kk;
  const int nxy = g.nx * g.ny;
  const size_t nr = (size_t)nxy * g.nz;
  cpx<A> a[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nthr;
    a[i] = cpx<A>{0, 0};
    if (!first && e < nxy) a[i] = acc[k * ld_acc + (size_t)z * nxy + e];
  }
  for (int jj = 0; jj < nj; ++jj) {
    const int j = j0 + jj;
    const size_t p = (size_t)kk * nj + jj;
    pass_c_fft<T>(work + p * nr + (size_t)z * nxy, s, twx, twy, g, tid, nthr, DeviceSync{});
    const cpx<T>* pj = psi + j * ld_psi + (size_t)z * nxy;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nthr;
      if (e < nxy) {
        const int y = e / g.nx, x = e - y * g.nx;
        const cpx<T> v = s[y * g.sx + x];
        const cpx<T> w = pj[e];
        a[i] = cadd(a[i], cmul(cpx<A>{(A)w.x, (A)w.y}, cpx<A>{(A)v.x, (A)v.y}));
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nthr;
    if (e >= nxy) continue;
    const size_t off = (size_t)z * nxy + e;
    if (last) {
      if (out_c64)
        reinterpret_cast<cpx<float>*>(out)[k * ld_out + off] = cpx<float>{(float)a[i].x, (float)a[i].y};
      else
        reinterpret_cast<cpx<double>*>(out)[k * ld_out + off] = cpx<double>{(double)a[i].x, (double)a[i].y};
    } else {
      acc[k * ld_acc + off] = a[i];
    }
  }
}

template <typename TI, typename TO>
__global__ void k_convert(const cpx<TI>* __restrict__ in, int64_t ld_in, cpx<TO>* __restrict__ out, int64_t ld_out,
                          int64_t nr, int ncols) {
  const int64_t total = nr * ncols;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = i / nr, r = i - c * nr;
    const cpx<TI> v = in[c * ld_in + r];
    out[c * ld_out + r] = cpx<TO>{(TO)v.x, (TO)v.y};
  }
}

// E_X: per-column Re <psi_k, w_k> in FP64 with a fixed reduction order.
template <typename TP, typename TW>
__global__ void __launch_bounds__(256) k_dot_cols(const cpx<TP>* __restrict__ psi, int64_t ldp,
                                                  const cpx<TW>* __restrict__ w, int64_t ldw, int64_t nr,
                                                  double* __restrict__ partial) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < nr; r += 256) {
    const cpx<TP> a = psi[k * ldp + r];
    const cpx<TW> b = w[k * ldw + r];
    acc += (double)a.x * (double)b.x + (double)a.y * (double)b.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[k] = red[0];
}

__global__ void k_half_sum(const double* __restrict__ partial, int n, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *out = 0.5 * s;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static AxisArg to_arg(const AxisPlan& p) {
  AxisArg a;
  a.n = p.n;
  a.nst = p.nst;
  for (int i = 0; i < 4; ++i) a.R[i] = p.R[i];
  return a;
}

PassGeom make_geom(const fx_cell* cell) {
  PassGeom g;
  g.nx = cell->n[0];
  g.ny = cell->n[1];
  g.nz = cell->n[2];
  // odd row stride (in elements) so consecutive rows start in different banks
  g.sx = g.nx % 2 ? g.nx : g.nx + 1;
  AxisPlan p;
  make_axis_plan(g.nx, &p);
  g.ax = to_arg(p);
  make_axis_plan(g.ny, &p);
  g.ay = to_arg(p);
  make_axis_plan(g.nz, &p);
  g.az = to_arg(p);
  g.hx = g.nx / 2 + 1;
  g.hy = g.ny / 2 + 1;
  return g;
}

static int round64(int v) { return (v + 63) / 64 * 64; }

template <typename K>
static fx_status allow_lds(K kernel, size_t bytes) {
  static std::set<const void*> done;
  const void* key = reinterpret_cast<const void*>(kernel);
  if (bytes > 65536 && !done.count(key)) {
    FX_HIP(hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    done.insert(key);
  }
  return FX_OK;
}

static size_t work_cap_bytes(fx_ctx* ctx) {
  size_t cap = (size_t)4096 << 20;
  if (const char* e = getenv("FX_WORK_MB")) cap = (size_t)atol(e) << 20;
  if (cap > ctx->budget / 4) cap = ctx->budget / 4;
  return cap;
}

// Pass C launch with the EPT (elements per thread) that fits the plane.
template <typename T, typename A>
static fx_status launch_pass_c(const PassGeom& g, int nthr_hint, dim3 grid, size_t lds, hipStream_t st,
                               const cpx<T>* psi, int64_t ld_psi, const cpx<T>* work, int j0, int nj, int k0,
                               cpx<A>* acc, int64_t ld_acc, int first, void* out, int64_t ld_out, int out_c64,
                               int last, const cpx<T>* twx, const cpx<T>* twy) {
  const int nxy = g.nx * g.ny;
  (void)nthr_hint;
  static const int epts[] = {4, 6, 9, 12, 16};
  int ept = 0, nthr = 0;
  for (int e : epts) {
    int t = round64((nxy + e - 1) / e);
    if (t <= 1024) {
      ept = e;
      nthr = t;
      break;
    }
  }
  if (!ept) FX_FAIL(FX_ERR_UNSUPPORTED, "plane of %d points is too large", nxy);
#define FX_PASSC(E)                                                                                       \
  case E:                                                                                                 \
    FX_TRY(allow_lds(k_pass_c<T, A, E>, lds));                                                            \
    hipLaunchKernelGGL((k_pass_c<T, A, E>), grid, dim3(nthr), lds, st, psi, ld_psi, work, j0, nj, k0, acc, \
                       ld_acc, first, out, ld_out, out_c64, last, g, twx, twy);                           \
    break;
  switch (ept) {
    FX_PASSC(4)
    FX_PASSC(6)
    FX_PASSC(9)
    FX_PASSC(12)
    FX_PASSC(16)
  }
#undef FX_PASSC
  FX_LAUNCH_CHECK();
  return FX_OK;
}

template <typename T, typename A>
static fx_status run_batches(fx_ctx* ctx, Workspace* ws, const VxArgs& a, const GridTables* tb,
                             const cpx<T>* psi, int64_t ld_psi, const cpx<T>* phi, int64_t ld_phi, hipStream_t st,
                             VxStats* stats) {
  const PassGeom g = make_geom(a.cell);
  const int64_t nr = (int64_t)g.nx * g.ny * g.nz;
  const size_t pair_bytes = (size_t)nr * sizeof(cpx<T>);
  size_t cap = a.work_cap ? a.work_cap : work_cap_bytes(ctx);
  const int64_t pairs_cap = (int64_t)std::max<size_t>(1, cap / pair_bytes);
  // Batch shape: up to 16 orbitals per batch first (the plane-inverse pass
  // reads and writes its partial sums once per batch), then as many targets
  // as fit, balanced over the target blocks, then any leftover capacity
  // back to orbitals.
  int nj = (int)std::min<int64_t>(a.n_psi, std::min<int64_t>(16, pairs_cap));
  if (a.force_nj > 0) nj = std::min(nj, a.force_nj);
  const int64_t nk_max = std::max<int64_t>(1, pairs_cap / nj);
  const int64_t kblocks = (a.n_phi + nk_max - 1) / nk_max;
  const int nk = (int)((a.n_phi + kblocks - 1) / kblocks);
  if (a.force_nj <= 0) nj = (int)std::min<int64_t>(a.n_psi, std::max<int64_t>(nj, pairs_cap / nk));
  void* work = nullptr;
  FX_TRY(ws_get(ctx, ws, "vx_work", (size_t)nk * nj * pair_bytes, &work));
  const bool out_c64 = a.out_dtype == FX_C64;
  const bool out_is_A = (sizeof(A) == 8) == !out_c64;
  const bool multi_j = nj < a.n_psi;
  cpx<A>* acc = nullptr;
  int64_t ld_acc = 0;
  if (multi_j) {
    if (out_is_A) {
      acc = reinterpret_cast<cpx<A>*>(a.out);
      ld_acc = a.ld_out;
    } else {
      void* p = nullptr;
      FX_TRY(ws_get(ctx, ws, "vx_acc", (size_t)a.n_phi * nr * sizeof(cpx<A>), &p));
      acc = reinterpret_cast<cpx<A>*>(p);
      ld_acc = nr;
    }
  }
  const cpx<T>* twx = reinterpret_cast<const cpx<T>*>(tb->tw[0]);
  const cpx<T>* twy = reinterpret_cast<const cpx<T>*>(tb->tw[1]);
  const cpx<T>* twz = reinterpret_cast<const cpx<T>*>(tb->tw[2]);
  const T* kf = reinterpret_cast<const T*>(tb->kfold);
  const size_t lds_plane = ((size_t)plane_lds_elems(g) + g.nx + g.ny) * sizeof(cpx<T>);
  const size_t lds_xz = ((size_t)xz_lds_elems(g) + g.nz) * sizeof(cpx<T>) + (size_t)(g.nx + g.nz) * sizeof(int);
  FX_TRY(allow_lds(k_pass_a<T>, lds_plane));
  FX_TRY(allow_lds(k_pass_b<T>, lds_xz));
  const int nthr_a = a.nthr_a > 0 ? a.nthr_a : 256;
  const int nthr_b = a.nthr_b > 0 ? a.nthr_b : 256;
  int64_t launches = 0;
  for (int k0 = 0; k0 < a.n_phi; k0 += nk) {
    const int kb = std::min(nk, a.n_phi - k0);
    for (int j0 = 0; j0 < a.n_psi; j0 += nj) {
      const int jb = std::min(nj, a.n_psi - j0);
      const int first = j0 == 0, last = j0 + jb >= a.n_psi;
      const int npairs = kb * jb;
      // algorithmic bytes of each pass (see the pass descriptions)
      const double vol = (double)npairs * nr * sizeof(cpx<T>);
      const double accb = (double)kb * nr *
                          ((first ? 0.0 : (double)sizeof(cpx<A>)) +
                           (last ? (out_c64 ? 8.0 : 16.0) : (double)sizeof(cpx<A>)));
      int slot;
      FX_TRY(prof_begin(ctx, st, FX_K_VX_PLANE_FWD, 3.0 * vol, &slot));
      hipLaunchKernelGGL((k_pass_a<T>), dim3((unsigned)(npairs * g.nz)), dim3(nthr_a), lds_plane, st, psi, ld_psi,
                         phi, ld_phi, reinterpret_cast<cpx<T>*>(work), j0, jb, k0, g, twx, twy);
      FX_LAUNCH_CHECK();
      FX_TRY(prof_end(ctx, st, slot));
      FX_TRY(prof_begin(ctx, st, FX_K_VX_PENCIL_Z, 2.0 * vol, &slot));
      hipLaunchKernelGGL((k_pass_b<T>), dim3((unsigned)(npairs * g.ny)), dim3(nthr_b), lds_xz, st,
                         reinterpret_cast<cpx<T>*>(work), g, twz, kf, tb->fold[0], tb->fold[1], tb->fold[2]);
      FX_LAUNCH_CHECK();
      FX_TRY(prof_end(ctx, st, slot));
      FX_TRY(prof_begin(ctx, st, FX_K_VX_PLANE_INV, 2.0 * vol + accb, &slot));
      FX_TRY((launch_pass_c<T, A>(g, 0, dim3((unsigned)(kb * g.nz)), lds_plane, st, psi, ld_psi,
                                  reinterpret_cast<const cpx<T>*>(work), j0, jb, k0, acc, ld_acc, first, a.out,
                                  a.ld_out, out_c64 ? 1 : 0, last, twx, twy)));
      FX_TRY(prof_end(ctx, st, slot));
      launches += 3;
    }
  }
  if (stats) {
    stats->nk = nk;
    stats->nj = nj;
    stats->launches = launches;
  }
  return FX_OK;
}

template <typename TI, typename TO>
fx_status convert(const void* in, int64_t ld_in, void* out, int64_t ld_out, int64_t nr, int ncols,
                         hipStream_t st) {
  const int64_t total = nr * ncols;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL((k_convert<TI, TO>), dim3(blocks), dim3(256), 0, st, reinterpret_cast<const cpx<TI>*>(in), ld_in,
                     reinterpret_cast<cpx<TO>*>(out), ld_out, nr, ncols);
  FX_LAUNCH_CHECK();
  return FX_OK;
}

fx_status convert_cols(const void* in, fx_dtype din, int64_t ld_in, void* out, fx_dtype dout, int64_t ld_out,
                       int64_t nr, int ncols, hipStream_t st) {
  if (din == FX_C128 && dout == FX_C128) return convert<double, double>(in, ld_in, out, ld_out, nr, ncols, st);
  if (din == FX_C128) return convert<double, float>(in, ld_in, out, ld_out, nr, ncols, st);
  if (dout == FX_C128) return convert<float, double>(in, ld_in, out, ld_out, nr, ncols, st);
  return convert<float, float>(in, ld_in, out, ld_out, nr, ncols, st);
}

fx_status check_vx_args(const VxArgs& a) {
  FX_TRY(check_cell(a.cell));
  FX_TRY(check_kernel(a.kern));
  const int64_t nr = (int64_t)a.cell->n[0] * a.cell->n[1] * a.cell->n[2];
  if (!a.psi || !a.phi || !a.out) FX_FAIL(FX_ERR_INVALID, "psi, phi and out must be non-NULL device pointers");
  if (a.n_psi <= 0 || a.n_phi <= 0) FX_FAIL(FX_ERR_INVALID, "n_psi = %d and n_phi = %d must be positive", a.n_psi, a.n_phi);
  if (a.ld_psi < nr || a.ld_phi < nr || a.ld_out < nr)
    FX_FAIL(FX_ERR_INVALID, "leading dimensions (%lld, %lld, %lld) must be >= N_r = %lld", (long long)a.ld_psi,
            (long long)a.ld_phi, (long long)a.ld_out, (long long)nr);
  if (a.in_dtype != FX_C128 && a.in_dtype != FX_C64) FX_FAIL(FX_ERR_UNSUPPORTED, "unknown in_dtype %d", a.in_dtype);
  if (a.out_dtype != FX_C128 && a.out_dtype != FX_C64) FX_FAIL(FX_ERR_UNSUPPORTED, "unknown out_dtype %d", a.out_dtype);
  if (a.prec != FX_PREC_FP64 && a.prec != FX_PREC_FP32 && a.prec != FX_PREC_FP32_ACC64)
    FX_FAIL(FX_ERR_UNSUPPORTED, "precision %d is not a V_X precision", a.prec);
  // aliasing of out with the inputs
  const size_t isz = dtype_size(a.in_dtype), osz = dtype_size(a.out_dtype);
  const char* o0 = (const char*)a.out;
  const char* o1 = o0 + ((size_t)(a.n_phi - 1) * a.ld_out + nr) * osz;
  const char* ins[2] = {(const char*)a.psi, (const char*)a.phi};
  const size_t ilen[2] = {((size_t)(a.n_psi - 1) * a.ld_psi + nr) * isz, ((size_t)(a.n_phi - 1) * a.ld_phi + nr) * isz};
  for (int i = 0; i < 2; ++i)
    if (o0 < ins[i] + ilen[i] && ins[i] < o1) FX_FAIL(FX_ERR_INVALID, "out overlaps an input array");
  if (a.ex_dev && !(a.phi == a.psi && a.ld_phi == a.ld_psi && a.n_phi <= a.n_psi))
    FX_FAIL(FX_ERR_INVALID, "ex_energy_dev requires phi == psi (same pointer and ld, n_phi <= n_psi)");
  return FX_OK;
}

fx_status vx_apply(fx_ctx* ctx, Workspace* ws, const VxArgs& a, hipStream_t st, VxStats* stats) {
  FX_TRY(check_vx_args(a));
  const int64_t nr = (int64_t)a.cell->n[0] * a.cell->n[1] * a.cell->n[2];
  const bool t64 = a.prec == FX_PREC_FP64;
  const GridTables* tb = nullptr;
  FX_TRY(grid_tables(ctx, a.cell, a.kern, t64 ? 0 : 1, &tb));
  const bool same = a.phi == a.psi && a.ld_phi == a.ld_psi;
  const bool need_conv = (a.in_dtype == FX_C128) != t64;
  const void* psi = a.psi;
  const void* phi = a.phi;
  int64_t ld_psi = a.ld_psi, ld_phi = a.ld_phi;
  if (need_conv) {
    const int ncp = same ? std::max(a.n_psi, a.n_phi) : a.n_psi;
    const size_t tsz = t64 ? 16 : 8;
    void* p = nullptr;
    FX_TRY(ws_get(ctx, ws, "vx_psiT", (size_t)ncp * nr * tsz, &p));
    if (t64)
      FX_TRY((convert<float, double>(a.psi, a.ld_psi, p, nr, nr, ncp, st)));
    else
      FX_TRY((convert<double, float>(a.psi, a.ld_psi, p, nr, nr, ncp, st)));
    psi = p;
    ld_psi = nr;
    if (same) {
      phi = p;
      ld_phi = nr;
    } else {
      void* q = nullptr;
      FX_TRY(ws_get(ctx, ws, "vx_phiT", (size_t)a.n_phi * nr * tsz, &q));
      if (t64)
        FX_TRY((convert<float, double>(a.phi, a.ld_phi, q, nr, nr, a.n_phi, st)));
      else
        FX_TRY((convert<double, float>(a.phi, a.ld_phi, q, nr, nr, a.n_phi, st)));
      phi = q;
      ld_phi = nr;
    }
  }
  if (a.prec == FX_PREC_FP64) {
    FX_TRY((run_batches<double, double>(ctx, ws, a, tb, (const cpx<double>*)psi, ld_psi, (const cpx<double>*)phi,
                                        ld_phi, st, stats)));
  } else if (a.prec == FX_PREC_FP32_ACC64) {
    FX_TRY((run_batches<float, double>(ctx, ws, a, tb, (const cpx<float>*)psi, ld_psi, (const cpx<float>*)phi, ld_phi,
                                       st, stats)));
  } else {
    FX_TRY((run_batches<float, float>(ctx, ws, a, tb, (const cpx<float>*)psi, ld_psi, (const cpx<float>*)phi, ld_phi,
                                      st, stats)));
  }
  if (a.ex_dev) {
    void* part = nullptr;
    FX_TRY(ws_get(ctx, ws, "vx_expart", (size_t)a.n_phi * sizeof(double), &part));
    const bool p64 = a.in_dtype == FX_C128, o64 = a.out_dtype == FX_C128;
    dim3 grid(a.n_phi), blk(256);
    if (p64 && o64)
      hipLaunchKernelGGL((k_dot_cols<double, double>), grid, blk, 0, st, (const cpx<double>*)a.psi, a.ld_psi,
                         (const cpx<double>*)a.out, a.ld_out, nr, (double*)part);
    else if (p64)
      hipLaunchKernelGGL((k_dot_cols<double, float>), grid, blk, 0, st, (const cpx<double>*)a.psi, a.ld_psi,
                         (const cpx<float>*)a.out, a.ld_out, nr, (double*)part);
    else if (o64)
      hipLaunchKernelGGL((k_dot_cols<float, double>), grid, blk, 0, st, (const cpx<float>*)a.psi, a.ld_psi,
                         (const cpx<double>*)a.out, a.ld_out, nr, (double*)part);
    else
      hipLaunchKernelGGL((k_dot_cols<float, float>), grid, blk, 0, st, (const cpx<float>*)a.psi, a.ld_psi,
                         (const cpx<float>*)a.out, a.ld_out, nr, (double*)part);
    FX_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_half_sum, dim3(1), dim3(64), 0, st, (const double*)part, a.n_phi, a.ex_dev);
    FX_LAUNCH_CHECK();
  }
  return FX_OK;
}

// Host run of the pass bodies for one pair: v = (-scale/Omega) *
// IFFT_u[K FFT_u(conj(psi_j) phi_k)], with the device code's plans, twiddles
// and folded kernel table, in FP64 (prec 0) or FP32 (prec 1).  Inputs and
// outputs are host arrays of N_r interleaved complex doubles.
template <typename T>
static void host_pair(const fx_cell* cell, const HostTables& h, const double* psi_j, const double* phi_k, double* v) {
  const PassGeom g = make_geom(cell);
  const size_t nxy = (size_t)g.nx * g.ny, nr = nxy * g.nz;
  std::vector<cpx<T>> a(nr), b(nr), vol(nr);
  for (size_t i = 0; i < nr; ++i) {
    a[i] = {(T)psi_j[2 * i], (T)psi_j[2 * i + 1]};
    b[i] = {(T)phi_k[2 * i], (T)phi_k[2 * i + 1]};
  }
  std::vector<cpx<T>> tw[3];
  for (int ax = 0; ax < 3; ++ax)
    for (auto& c : h.tw[ax]) tw[ax].push_back({(T)c.x, (T)c.y});
  std::vector<T> kf(h.kfold.begin(), h.kfold.end());
  std::vector<cpx<T>> s((size_t)std::max(plane_lds_elems(g), xz_lds_elems(g)));
  for (int z = 0; z < g.nz; ++z)
    pass_a_body<T>(a.data() + z * nxy, b.data() + z * nxy, vol.data() + z * nxy, s.data(), tw[0].data(), tw[1].data(),
                   g, 0, 1, HostSync{});
  for (int y = 0; y < g.ny; ++y)
    pass_b_body<T>(vol.data(), y, s.data(), tw[2].data(), kf.data(), h.fold[0].data(), h.fold[2].data(), h.fold[1][y], g,
                   0, 1, HostSync{});
  for (int z = 0; z < g.nz; ++z) {
    pass_c_fft<T>(vol.data() + z * nxy, s.data(), tw[0].data(), tw[1].data(), g, 0, 1, HostSync{});
    for (size_t e = 0; e < nxy; ++e) {
      const int y = (int)(e / g.nx), x = (int)(e - (size_t)y * g.nx);
      v[2 * (z * nxy + e)] = (double)s[(size_t)y * g.sx + x].x;
      v[2 * (z * nxy + e) + 1] = (double)s[(size_t)y * g.sx + x].y;
    }
  }
}

}  // namespace fx

using namespace fx;

extern "C" {

fx_status fx_apply_vx(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel, const void* psi, int32_t n_psi,
                      int64_t ld_psi, const void* phi, int32_t n_phi, int64_t ld_phi, void* out, int64_t ld_out,
                      fx_dtype in_dtype, fx_dtype out_dtype, fx_prec prec, void* stream, double* ex_energy_dev) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
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
  if (const char* e = getenv("FX_VX_NJ")) a.force_nj = atoi(e);
  if (const char* e = getenv("FX_VX_NTHR_A")) a.nthr_a = atoi(e);
  if (const char* e = getenv("FX_VX_NTHR_B")) a.nthr_b = atoi(e);
  hipStream_t st = (hipStream_t)stream;
  return vx_apply(ctx, &ctx->ws, a, st, nullptr);
}

fx_status fx_debug_host_pair(const fx_cell* cell, const fx_kernel* kernel, int prec, const double* psi_j,
                             const double* phi_k, double* v) {
  clear_error();
  FX_TRY(check_cell(cell));
  FX_TRY(check_kernel(kernel));
  if (!psi_j || !phi_k || !v) FX_FAIL(FX_ERR_INVALID, "NULL host pointer");
  HostTables h;
  host_tables(cell, kernel, &h);
  if (prec == 0)
    host_pair<double>(cell, h, psi_j, phi_k, v);
  else
    host_pair<float>(cell, h, psi_j, phi_k, v);
  return FX_OK;
}

}  // extern "C"
