// fx_apply_vx: V_X applied to a block of targets by batched pair Poisson
// solves (Eq. applyVX; the Fock-application loop of Sec. 3.2 on one GPU's
// band-index share).  Pairs are processed in batches of nk targets x nj
// orbitals; every batch runs the three passes of vx_passes.hpp.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <set>

#include "common.hpp"
#include "vx.hpp"
#include "vx_passes.hpp"

namespace fx {

// ---------------------------------------------------------------------------
// kernels
//
// The plane passes are persistent: each workgroup walks items (pair, z) or
// (target, z) with stride gridDim.x, and issues the global loads of the next
// plane into registers (EPT elements per thread) before running the FFT of
// the current one, so the loads are in flight while the LDS stages run.
// ---------------------------------------------------------------------------
constexpr int kPlaneThreads = 512;
// most threads of a generic z-pass workgroup (its launch bound)
constexpr int kPencilThreads = 256;

template <typename T, int EPT>
__global__ void __launch_bounds__(kPlaneThreads) k_pass_a(const cpx<T>* __restrict__ psi, int64_t ld_psi,
                                                 const cpx<T>* __restrict__ phi, int64_t ld_phi,
                                                 cpx<T>* __restrict__ work, int j0, int nj, int k0, int nitems,
                                                 PassGeom g, const cpx<T>* __restrict__ twx_g,
                                                 const cpx<T>* __restrict__ twy_g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* s = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twx = s + plane_lds_elems(g);
  cpx<T>* twy = twx + g.nx;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int i = tid; i < g.nx; i += nthr) twx[i] = twx_g[i];
  for (int i = tid; i < g.ny; i += nthr) twy[i] = twy_g[i];
  const int nxy = g.nx * g.ny;
  const size_t nr = (size_t)nxy * g.nz;
  cpx<T> va[EPT], vb[EPT];
  auto fetch = [&](int it) __attribute__((always_inline)) {
    if (it >= nitems) return;
    const int z = it % g.nz, p = it / g.nz;
    const cpx<T>* a = psi + (int64_t)(j0 + p % nj) * ld_psi + (size_t)z * nxy;
    const cpx<T>* b = phi + (int64_t)(k0 + p / nj) * ld_phi + (size_t)z * nxy;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nthr;
      if (e < nxy) {
        va[i] = a[e];
        vb[i] = b[e];
      }
    }
  };
  // FP32: the next plane loads while this one transforms; FP64 planes do
  // not leave room in registers for that, so they load just before use
  constexpr bool kPipe = sizeof(T) == 4;
  int item = blockIdx.x;
  if (kPipe) fetch(item);
  for (; item < nitems; item += gridDim.x) {
    if (!kPipe) fetch(item);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nthr;
      if (e < nxy) {
        const int y = e / g.nx, x = e - y * g.nx;
        s[y * g.sx + x] = cconjmul(va[i], vb[i]);
      }
    }
    __syncthreads();
    if (kPipe) fetch(item + gridDim.x);
    lds_fft<true, T>(s, g.ax, g.ny, 1, g.sx, twx, tid, nthr, DeviceSync{});
    lds_fft<true, T>(s, g.ay, g.nx, g.sx, 1, twy, tid, nthr, DeviceSync{});
    const int z = item % g.nz, p = item / g.nz;
    cpx<T>* o = work + p * nr + (size_t)z * nxy;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nthr;
      if (e < nxy) {
        const int y = e / g.nx, x = e - y * g.nx;
        o[e] = s[y * g.sx + x];
      }
    }
    __syncthreads();
  }
}

// Pass B: one (pair, y, x-tile) per workgroup; many small workgroups per CU.
template <typename T, int EPT>
__global__ void __launch_bounds__(kPencilThreads) k_pass_b(cpx<T>* __restrict__ work, int xt, int ntx, PassGeom g,
                                                const cpx<T>* __restrict__ twz_g, const T* __restrict__ kfold,
                                                const int* __restrict__ foldx_g, const int* __restrict__ foldy_g,
                                                const int* __restrict__ foldz_g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = g.nz * xt;
  cpx<T>* s = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twz = s + n;
  T* kl = reinterpret_cast<T*>(twz + g.nz);
  int* fxl = reinterpret_cast<int*>(kl + g.hz * g.hx);
  int* fzl = fxl + g.nx;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int tx = blockIdx.x % ntx;
  const int rest = blockIdx.x / ntx;
  const int y = rest % g.ny;
  const int p = rest / g.ny;
  const int x0 = tx * xt;
  cpx<T>* vol = work + (size_t)p * g.nx * g.ny * g.nz;
  cpx<T> v[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nthr;
    const int z = e / xt, x = x0 + (e - z * xt);
    v[i] = cpx<T>{0, 0};
    if (e < n && x < g.nx) v[i] = vol[((size_t)z * g.ny + y) * g.nx + x];
  }
  // tables while the loads are in flight
  const int fy = foldy_g[y];
  for (int i = tid; i < g.nz; i += nthr) {
    twz[i] = twz_g[i];
    fzl[i] = foldz_g[i];
  }
  for (int i = tid; i < g.nx; i += nthr) fxl[i] = foldx_g[i];
  for (int i = tid; i < g.hz * g.hx; i += nthr) {
    const int fz = i / g.hx, fx = i - fz * g.hx;
    kl[i] = kfold[((size_t)fz * g.hy + fy) * g.hx + fx];
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nthr;
    if (e < n) s[e] = v[i];
  }
  __syncthreads();
  const KSlice<T> kf{kl, fxl, fzl, x0, g.nx, g.hx};
  lds_conv<T>(s, g.az, xt, xt, 1, twz, kf, tid, nthr, DeviceSync{});
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nthr;
    const int z = e / xt, x = x0 + (e - z * xt);
    if (e < n && x < g.nx) vol[((size_t)z * g.ny + y) * g.nx + x] = s[e];
  }
}

// Pass C.  acc (ld_acc) holds the running sum over j of the targets in the
// accumulation precision A; when `last` is set the final sum goes to `out`
// in its own dtype instead (out may be the same memory as acc).  While the
// FFT of orbital j runs, psi_j and the work plane of orbital j+1 are loading.
template <typename T, typename A, int EPT, bool PIPE>
__global__ void __launch_bounds__(kPlaneThreads) k_pass_c(const cpx<T>* __restrict__ psi, int64_t ld_psi,
                                                 const cpx<T>* __restrict__ work, int j0, int nj, int k0, int nitems,
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
  const int nxy = g.nx * g.ny;
  const size_t nr = (size_t)nxy * g.nz;
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int z = item % g.nz;
    const int kk = item / g.nz;
    const int k = k0 + kk;
    cpx<A> a[EPT];
    cpx<T> vt[EPT], vp[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nthr;
      a[i] = cpx<A>{0, 0};
      if (!first && e < nxy) a[i] = acc[k * ld_acc + (size_t)z * nxy + e];
    }
    constexpr bool kPipe = PIPE;  // prefetch the next work plane during the FFT
    auto tload = [&](int jj) __attribute__((always_inline)) {
      const cpx<T>* tp = work + ((size_t)kk * nj + jj) * nr + (size_t)z * nxy;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * nthr;
        if (e < nxy) vt[i] = tp[e];
      }
    };
    if (kPipe) tload(0);
    for (int jj = 0; jj < nj; ++jj) {
      if (!kPipe) tload(jj);
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * nthr;
        if (e < nxy) {
          const int y = e / g.nx, x = e - y * g.nx;
          s[y * g.sx + x] = vt[i];
        }
      }
      __syncthreads();
      const cpx<T>* pj = psi + (int64_t)(j0 + jj) * ld_psi + (size_t)z * nxy;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * nthr;
        if (e < nxy) vp[i] = pj[e];
      }
      if (kPipe && jj + 1 < nj) tload(jj + 1);
      lds_fft<false, T>(s, g.ay, g.nx, g.sx, 1, twy, tid, nthr, DeviceSync{});
      lds_fft<false, T>(s, g.ax, g.ny, 1, g.sx, twx, tid, nthr, DeviceSync{});
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * nthr;
        if (e < nxy) {
          const int y = e / g.nx, x = e - y * g.nx;
          const cpx<T> v = s[y * g.sx + x];
          // FP32 transforms: four FMAs per term; FP64: product then sum (the
          // FMA chain costs the FP64 kernels registers they do not have)
          if constexpr (sizeof(T) == 4)
            a[i] = cfma(a[i], cpx<A>{(A)vp[i].x, (A)vp[i].y}, cpx<A>{(A)v.x, (A)v.y});
          else
            a[i] = cadd(a[i], cmul(cpx<A>{(A)vp[i].x, (A)vp[i].y}, cpx<A>{(A)v.x, (A)v.y}));
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

PassGeom make_geom(const fx_cell* cell, const PlanSet* plans = nullptr) {
  PassGeom g;
  g.nx = cell->n[0];
  g.ny = cell->n[1];
  g.nz = cell->n[2];
  // odd row stride (in elements) so consecutive rows start in different banks
  g.sx = g.nx % 2 ? g.nx : g.nx + 1;
  PlanSet ps;
  if (plans)
    ps = *plans;
  else
    default_plans(cell, &ps);
  g.ax = to_arg(ps.ax[0]);
  g.ay = to_arg(ps.ax[1]);
  g.az = to_arg(ps.ax[2]);
  g.hx = g.nx / 2 + 1;
  g.hy = g.ny / 2 + 1;
  g.hz = g.nz / 2 + 1;
  return g;
}

static int round64(int v) { return (v + 63) / 64 * 64; }

template <typename K>
static fx_status allow_lds(K kernel, size_t bytes) {
  return allow_dynamic_lds(reinterpret_cast<const void*>(kernel), bytes);
}

// Workgroups of a persistent kernel: resident workgroups per CU x CUs.
template <typename K>
static fx_status persistent_grid(fx_ctx* ctx, K kernel, int nthr, size_t lds, int items, int* grid) {
  int per_cu = 0;
  FX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), nthr, lds));
  if (per_cu < 1) per_cu = 1;
  *grid = std::max(1, std::min(items, per_cu * std::max(ctx->n_cu, 1)));
  return FX_OK;
}

static size_t work_cap_bytes(fx_ctx* ctx) {
  // pair work volume per batch: 8 GiB (a few percent of HBM) keeps launches
  // long and partial-sum traffic low; capped at a quarter of the budget
  size_t cap = (size_t)8192 << 20;
  if (const char* e = getenv("FX_WORK_MB")) cap = (size_t)atol(e) << 20;
  if (cap > ctx->budget / 4) cap = ctx->budget / 4;
  return cap;
}

// Elements per thread (a compile-time register count) and threads for
// `elems` elements and at most max_thr threads.
static const int kEpts[] = {1, 2, 3, 4, 6, 9, 18};
static bool pick_ept(int elems, int max_thr, int* ept, int* nthr) {
  for (int e : kEpts) {
    const int t = round64((elems + e - 1) / e);
    if (t <= max_thr) {
      *ept = e;
      *nthr = t;
      return true;
    }
  }
  return false;
}

#define FX_EPT_SWITCH(EPT_VAR, ...) \
  switch (EPT_VAR) {                 \
    case 1: { constexpr int E = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int E = 2; __VA_ARGS__; } break;   \
    case 3: { constexpr int E = 3; __VA_ARGS__; } break;   \
    case 4: { constexpr int E = 4; __VA_ARGS__; } break;   \
    case 6: { constexpr int E = 6; __VA_ARGS__; } break;   \
    case 9: { constexpr int E = 9; __VA_ARGS__; } break;   \
    case 18: { constexpr int E = 18; __VA_ARGS__; } break; \
    default: FX_FAIL(FX_ERR_UNSUPPORTED, "no kernel for %d elements per thread", EPT_VAR); \
  }

// z-pass form of the specialised kernels: the persistent kernel with whole x
// rows is the automatic choice at 96^3, where it measured faster (3.12 vs
// 3.38 ms per launch of 1170 pairs), whole x rows at 72^3 (15.6 vs 16.6 ms
// for 432 orbitals x 8 targets); elsewhere the autotuner decides.
static int ct_b_variant(const VxArgs& a) {
  if (a.b_var >= 1 && a.b_var <= 4) return a.b_var;
  return a.cell->n[0] == 96 ? 4 : (a.cell->n[0] == 72 ? 3 : 1);
}

// Plane-inverse threads of the specialised kernels: the larger count (fewer
// accumulators per thread, more waves per CU) is the automatic choice at
// 96^3, where it measured faster (3.34 vs 3.39 ms per launch of 1170 pairs),
// and at 72^3 (15.1 vs 15.6 ms for 432 orbitals x 8 targets, with whole-row
// z tiles), in its wave-level form (5): 2.75 vs 2.79 ms per launch at 96^3
// in FP32, 2.38 vs 2.50 in FP64.  Elsewhere the autotuner decides.
static int ct_c_variant(const VxArgs& a) {
  if (a.c_var >= 1 && a.c_var <= 5) return a.c_var;
  return a.cell->n[0] == 96 || a.cell->n[0] == 72 ? 5 : 1;
}

// How the XCDs share the items of the persistent plane passes (bit 0: the
// plane-forward pass, bit 1: the plane-inverse pass; set: each XCD takes a
// contiguous range of z planes of every unit, clear: a contiguous range of
// units at every z).  The plane-forward pass reads each orbital and target
// plane once per XCD with the z split instead of once per XCD per chunk of
// pairs (3.05 -> 2.82 ms per launch of 1170 pairs at 96^3); the plane-inverse
// pass measured slower with it (3.13 -> 3.30 ms), so it keeps the unit split.
// Sum groups of the specialised plane-inverse pass: the terms of orbital j
// go to partial sum j mod S of their target, each in ascending j, and the S
// partial sums are added in order of the group at the end.  With few targets
// the pass has few items (targets x planes); S times as many balance the
// CUs.  The grouping depends on the orbital index only, so a column's result
// is the same whatever the batch size and whichever targets share a launch.
// S = 1 (automatic) keeps one running sum per target; the allocation-free
// form always does.
static int ct_jsplit(const VxArgs& a) {
  if (a.no_alloc) return 1;
  return a.c_split == 2 || a.c_split == 4 || a.c_split == 8 ? a.c_split : 1;
}

// out[t] = sum over the groups g = 0, 1, ... of acc[g][t] (targets t0 ..
// t0 + nt - 1), converted to the output type.
template <typename A>
__global__ void k_combine_groups(const cpx<A>* __restrict__ acc, int64_t gstride, int64_t ld_acc, int jsplit, int t0,
                                 int nt, int64_t nr, void* __restrict__ out, int64_t ld_out, int out_c64) {
  const int64_t total = (int64_t)nt * nr;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = t0 + i / nr, e = i % nr;
    cpx<A> v = acc[t * ld_acc + e];
    for (int g = 1; g < jsplit; ++g) v = cadd(v, acc[g * gstride + t * ld_acc + e]);
    if (out_c64)
      reinterpret_cast<cpx<float>*>(out)[t * ld_out + e] = cpx<float>{(float)v.x, (float)v.y};
    else
      reinterpret_cast<cpx<double>*>(out)[t * ld_out + e] = cpx<double>{(double)v.x, (double)v.y};
  }
}

template <typename A>
static fx_status combine_groups(fx_ctx* ctx, hipStream_t st, const cpx<A>* acc, int64_t gstride, int64_t ld_acc,
                                int jsplit, int t0, int nt, int64_t nr, void* out, int64_t ld_out, int out_c64) {
  const int64_t total = (int64_t)nt * nr;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 8 * std::max(ctx->n_cu, 1)));
  hipLaunchKernelGGL((k_combine_groups<A>), dim3(blocks), dim3(256), 0, st, acc, gstride, ld_acc, jsplit, t0, nt, nr,
                     out, ld_out, out_c64);
  FX_LAUNCH_CHECK();
  return FX_OK;
}

// Work order of the specialised plane passes: bit 0 splits the plane-forward
// pass over the XCDs by z, bit 1 the plane-inverse pass (slower: 2.76 against
// 2.71 ms per launch at 96^3), bit 2 walks the plane-forward pass's pairs in
// blocks of 4 orbitals x 16 targets (unit_plane).  Only the order changes,
// never a result.
static int ct_zsplit() {
  const char* e = getenv("FX_VX_ZSPLIT");
  return e ? atoi(e) : 5;
}

// Halved apply for phi == psi (all N targets): each unordered pair {j, k} is
// solved once, as (min, max), since v_kj = conj(v_jk) for a real, even kernel.
// Orbitals are cut into blocks of B; block pairs (J <= K) run in ascending
// order of J, then K.  For each, pass C runs twice: role 0 adds the pairs to
// the targets of block K, role 1 (conjugated) to those of block J.  Every
// output column then receives its terms in ascending j, each term computed
// from the ordered pair (min(j,k), max(j,k)), so the result does not depend
// on B.  Diagonal block pairs hold only the B(B+1)/2 pairs j <= k.
template <typename T, typename A>
static fx_status run_halved(fx_ctx* ctx, Workspace* ws, const VxArgs& a, const GridTables* tb, const cpx<T>* psi,
                            int64_t ld_psi, int64_t pairs_cap, hipStream_t st, VxStats* stats) {
  const int n = a.cell->n[0];
  const int64_t nr = (int64_t)n * n * n;
  const size_t pair_bytes = (size_t)nr * sizeof(cpx<T>);
  const int N = a.n_psi;
  int B = (int)std::min<int64_t>(N, std::max<int64_t>(1, (int64_t)std::sqrt((double)pairs_cap)));
  if (a.force_nj > 0) B = std::min(B, a.force_nj);
  const int nblk = (N + B - 1) / B;
  B = (N + nblk - 1) / nblk;
  void* work = nullptr;
  FX_TRY(ws_get(ctx, ws, "vx_work", (size_t)B * B * pair_bytes, &work));
  const bool out_c64 = a.out_dtype == FX_C64;
  const bool out_is_A = (sizeof(A) == 8) == !out_c64;
  const int jsplit = ct_jsplit(a);
  // partial sums live between the two roles of every block pair
  cpx<A>* acc = nullptr;
  int64_t ld_acc = 0, gstride = 0;
  if (out_is_A && jsplit == 1) {
    acc = reinterpret_cast<cpx<A>*>(a.out);
    ld_acc = a.ld_out;
  } else {
    void* p = nullptr;
    FX_TRY(ws_get(ctx, ws, "vx_acc", (size_t)jsplit * N * nr * sizeof(cpx<A>), &p));
    acc = reinterpret_cast<cpx<A>*>(p);
    ld_acc = nr;
    gstride = (int64_t)N * nr;
  }
  const cpx<T>* tw = reinterpret_cast<const cpx<T>*>(tb->tw[0]);
  const T* kf = reinterpret_cast<const T*>(tb->kfold);
  const double sz = sizeof(cpx<T>), asz = sizeof(cpx<A>), osz = out_c64 ? 8.0 : 16.0;
  int64_t launches = 0, solves = 0;
  for (int J = 0; J < nblk; ++J) {
    const int j0 = J * B, jb = std::min(B, N - j0);
    for (int K = J; K < nblk; ++K) {
      const int k0 = K * B, kb = std::min(B, N - k0);
      const int tri = J == K;
      const int npairs = tri ? jb * (jb + 1) / 2 : jb * kb;
      CtBatch<T> cb{psi, ld_psi, psi, ld_psi, reinterpret_cast<cpx<T>*>(work), j0, jb, k0, kb, npairs, tw, kf,
                    tb->fold[0], tri, a.a_pipe > 0 ? 1 : 0, ct_b_variant(a), ct_c_variant(a), (a.a_var >= 1 && a.a_var <= 3) ? a.a_var : 0, a.nt_hint != 0 ? 1 : 0, ct_zsplit()};
      cb.jsplit = jsplit;
      const double vol = (double)npairs * nr * sz;
      int slot;
      FX_TRY(prof_begin(ctx, st, FX_K_VX_PLANE_FWD, 2.0 * vol, &slot));
      FX_TRY(ct_pass_a<T>(ctx, st, n, cb));
      FX_TRY(prof_end(ctx, st, slot));
      FX_TRY(prof_begin(ctx, st, FX_K_VX_PENCIL_Z, 2.0 * vol, &slot));
      FX_TRY(ct_pass_b<T>(ctx, st, n, cb));
      FX_TRY(prof_end(ctx, st, slot));
      // role 0: targets of block K; the first contribution to them is J = 0
      {
        const int first = J == 0;
        CtAcc<A> ca{acc, ld_acc, first, a.out, a.ld_out, out_c64 ? 1 : 0, 0, -1, gstride};
        const double accb = (double)kb * nr * ((first ? 0.0 : asz) + asz) * jsplit;
        FX_TRY(prof_begin(ctx, st, FX_K_VX_PLANE_INV, 2.0 * vol + accb, &slot));
        FX_TRY((ct_pass_c<T, A>(ctx, st, n, cb, ca, 0)));
        FX_TRY(prof_end(ctx, st, slot));
      }
      // role 1: targets of block J; their last contribution is K = nblk - 1
      {
        const int last = K == nblk - 1 && jsplit == 1;
        CtAcc<A> ca{acc, ld_acc, 0, a.out, a.ld_out, out_c64 ? 1 : 0, last, -1, gstride};
        const double planes = tri ? (double)(npairs - jb) : (double)npairs;
        const double accb = (double)jb * nr * (asz + (last ? osz : asz)) * jsplit;
        FX_TRY(prof_begin(ctx, st, FX_K_VX_PLANE_INV, 2.0 * planes * nr * sz + accb, &slot));
        FX_TRY((ct_pass_c<T, A>(ctx, st, n, cb, ca, 1)));
        FX_TRY(prof_end(ctx, st, slot));
      }
      launches += 4;
      solves += npairs;
    }
  }
  if (jsplit > 1) {
    int slot;
    FX_TRY(prof_begin(ctx, st, FX_K_REDUCE, (double)N * nr * (jsplit * asz + osz), &slot));
    FX_TRY(combine_groups<A>(ctx, st, acc, gstride, ld_acc, jsplit, 0, N, nr, a.out, a.ld_out, out_c64 ? 1 : 0));
    FX_TRY(prof_end(ctx, st, slot));
    ++launches;
  }
  if (stats) {
    stats->nk = B;
    stats->nj = B;
    stats->launches = launches;
    stats->solves = solves;
  }
  return FX_OK;
}

template <typename T, typename A>
static fx_status run_batches(fx_ctx* ctx, Workspace* ws, const VxArgs& a, const GridTables* tb,
                             const cpx<T>* psi, int64_t ld_psi, const cpx<T>* phi, int64_t ld_phi, hipStream_t st,
                             VxStats* stats) {
  const PassGeom g = make_geom(a.cell, a.plans_set ? &a.plans : nullptr);
  const int64_t nr = (int64_t)g.nx * g.ny * g.nz;
  const int nxy = g.nx * g.ny;
  const size_t pair_bytes = (size_t)nr * sizeof(cpx<T>);
  size_t cap = a.work_cap ? std::min(a.work_cap, ctx->budget / 4) : work_cap_bytes(ctx);
  const int64_t pairs_cap = (int64_t)std::max<size_t>(1, cap / pair_bytes);
  // cubic grids of the workload edges run the compile-time-specialised
  // kernels unless the generic family or another radix schedule is asked for
  bool use_ct = ct_supported(a.cell) && a.kernels != 2;
  if (use_ct && a.plans_set) {
    PlanSet d;
    default_plans(a.cell, &d);
    use_ct = same_plans(a.plans, d);
  }
  if (a.kernels == 1 && !use_ct)
    FX_FAIL(FX_ERR_UNSUPPORTED, "no specialised kernels for grid %dx%dx%d with this radix schedule", g.nx, g.ny,
            g.nz);
  if (a.segs.n > 0 && (!use_ct || psi == phi))
    FX_FAIL(FX_ERR_UNSUPPORTED, "multi-trajectory launches need the specialised kernels and phi != psi");
  if (use_ct && a.halve != 0 && psi == phi && ld_psi == ld_phi && a.n_psi == a.n_phi)
    return run_halved<T, A>(ctx, ws, a, tb, psi, ld_psi, pairs_cap, st, stats);
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
  const int jsplit = use_ct ? ct_jsplit(a) : 1;
  cpx<A>* acc = nullptr;
  int64_t ld_acc = 0, gstride = 0;
  if (jsplit > 1) {
    // the groups' partial sums, added into out after the last batch
    void* p = nullptr;
    FX_TRY(ws_get(ctx, ws, "vx_acc", (size_t)jsplit * a.n_phi * nr * sizeof(cpx<A>), &p));
    acc = reinterpret_cast<cpx<A>*>(p);
    ld_acc = nr;
    gstride = (int64_t)a.n_phi * nr;
  } else if (multi_j) {
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

  // launch shapes
  int ept_p = 0, nthr_p = 0;
  if (!pick_ept(nxy, kPlaneThreads, &ept_p, &nthr_p)) FX_FAIL(FX_ERR_UNSUPPORTED, "plane of %d points is too large", nxy);
  const bool pipe_c = a.pipe >= 0 ? a.pipe != 0 : ept_p < 18;
  int xt = g.nx < 32 ? g.nx : 32;
  if (a.xtile > 0) xt = std::min(g.nx, a.xtile);
  const int ntx = (g.nx + xt - 1) / xt;
  int ept_b = 0, nthr_b = 0;
  if (!pick_ept(g.nz * xt, a.nthr_b > 0 ? std::min(a.nthr_b, kPencilThreads) : kPencilThreads, &ept_b, &nthr_b))
    FX_FAIL(FX_ERR_UNSUPPORTED, "pencil tile of %d points is too large", g.nz * xt);
  const size_t lds_plane = ((size_t)plane_lds_elems(g) + g.nx + g.ny) * sizeof(cpx<T>);
  const size_t lds_b = ((size_t)g.nz * xt + g.nz) * sizeof(cpx<T>) + (size_t)g.hz * g.hx * sizeof(T) +
                       (size_t)(g.nx + g.nz) * sizeof(int);

  int64_t launches = 0;
  for (int k0 = 0; k0 < a.n_phi; k0 += nk) {
    const int kb = std::min(nk, a.n_phi - k0);
    for (int j0 = 0; j0 < a.n_psi; j0 += nj) {
      const int jb = std::min(nj, a.n_psi - j0);
      const int first = j0 == 0, last = j0 + jb >= a.n_psi;
      const int npairs = kb * jb;
      // algorithmic bytes of each pass, per pair and grid point: plane-forward
      // psi_j + T (phi_k is reused from cache across the batch's orbitals),
      // z-pass T read + write, plane-inverse T + psi_j, plus the partial sums
      // read and written once per batch and target
      const double vol = (double)npairs * nr * sizeof(cpx<T>);
      const double accb = (double)kb * nr *
                          ((first ? 0.0 : (double)sizeof(cpx<A>)) +
                           (last ? (out_c64 ? 8.0 : 16.0) : (double)sizeof(cpx<A>)));
      int slot;
      if (use_ct) {
        CtBatch<T> cb{psi, ld_psi, phi, ld_phi, reinterpret_cast<cpx<T>*>(work), j0, jb, k0, kb, npairs, twx, kf,
                      tb->fold[0], 0, a.a_pipe > 0 ? 1 : 0, ct_b_variant(a), ct_c_variant(a), (a.a_var >= 1 && a.a_var <= 3) ? a.a_var : 0, a.nt_hint != 0 ? 1 : 0, ct_zsplit(), a.segs, jsplit};
        CtAcc<A> ca{acc, ld_acc, first, a.out, a.ld_out, out_c64 ? 1 : 0, jsplit > 1 ? 0 : last, a.pipe, gstride};
        FX_TRY(prof_begin(ctx, st, FX_K_VX_PLANE_FWD, 2.0 * vol, &slot));
        FX_TRY(ct_pass_a<T>(ctx, st, g.nx, cb));
        FX_TRY(prof_end(ctx, st, slot));
        FX_TRY(prof_begin(ctx, st, FX_K_VX_PENCIL_Z, 2.0 * vol, &slot));
        FX_TRY(ct_pass_b<T>(ctx, st, g.nx, cb));
        FX_TRY(prof_end(ctx, st, slot));
        FX_TRY(prof_begin(ctx, st, FX_K_VX_PLANE_INV, 2.0 * vol + accb, &slot));
        FX_TRY((ct_pass_c<T, A>(ctx, st, g.nx, cb, ca, 0)));
        FX_TRY(prof_end(ctx, st, slot));
        launches += 3;
        if (jsplit > 1 && last) {
          const double osz = out_c64 ? 8.0 : 16.0;
          FX_TRY(prof_begin(ctx, st, FX_K_REDUCE, (double)kb * nr * (jsplit * sizeof(cpx<A>) + osz), &slot));
          FX_TRY(combine_groups<A>(ctx, st, acc, gstride, ld_acc, jsplit, k0, kb, nr, a.out, a.ld_out,
                                   out_c64 ? 1 : 0));
          FX_TRY(prof_end(ctx, st, slot));
          ++launches;
        }
        continue;
      }
      FX_TRY(prof_begin(ctx, st, FX_K_VX_PLANE_FWD, 2.0 * vol, &slot));
      FX_EPT_SWITCH(ept_p, {
        auto kern = k_pass_a<T, E>;
        FX_TRY(allow_lds(kern, lds_plane));
        int grid = 0;
        FX_TRY(persistent_grid(ctx, kern, nthr_p, lds_plane, npairs * g.nz, &grid));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(nthr_p), lds_plane, st, psi, ld_psi, phi, ld_phi,
                           reinterpret_cast<cpx<T>*>(work), j0, jb, k0, npairs * g.nz, g, twx, twy);
      });
      FX_LAUNCH_CHECK();
      FX_TRY(prof_end(ctx, st, slot));
      FX_TRY(prof_begin(ctx, st, FX_K_VX_PENCIL_Z, 2.0 * vol, &slot));
      FX_EPT_SWITCH(ept_b, {
        auto kern = k_pass_b<T, E>;
        FX_TRY(allow_lds(kern, lds_b));
        hipLaunchKernelGGL(kern, dim3((unsigned)((int64_t)npairs * g.ny * ntx)), dim3(nthr_b), lds_b, st,
                           reinterpret_cast<cpx<T>*>(work), xt, ntx, g, twz, kf, tb->fold[0], tb->fold[1],
                           tb->fold[2]);
      });
      FX_LAUNCH_CHECK();
      FX_TRY(prof_end(ctx, st, slot));
      FX_TRY(prof_begin(ctx, st, FX_K_VX_PLANE_INV, 2.0 * vol + accb, &slot));
      FX_EPT_SWITCH(ept_p, {
        // prefetching the next work plane needs registers the FP64 form and
        // the largest planes do not have
        auto kern = pipe_c ? k_pass_c<T, A, E, sizeof(T) == 4> : k_pass_c<T, A, E, false>;
        FX_TRY(allow_lds(kern, lds_plane));
        int grid = 0;
        FX_TRY(persistent_grid(ctx, kern, nthr_p, lds_plane, kb * g.nz, &grid));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(nthr_p), lds_plane, st, psi, ld_psi,
                           reinterpret_cast<const cpx<T>*>(work), j0, jb, k0, kb * g.nz, acc, ld_acc, first, a.out,
                           a.ld_out, out_c64 ? 1 : 0, last, g, twx, twy);
      });
      FX_LAUNCH_CHECK();
      FX_TRY(prof_end(ctx, st, slot));
      launches += 3;
    }
  }
  if (stats) {
    stats->nk = nk;
    stats->nj = nj;
    stats->launches = launches;
    stats->solves = (int64_t)a.n_psi * a.n_phi;
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
  FX_TRY(check_kernel(a.kern, a.internal_kernel));
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

bool plans_from_radix(const fx_cell* cell, const int32_t radix[3][4], PlanSet* ps, bool* any) {
  default_plans(cell, ps);
  *any = false;
  for (int x = 0; x < 3; ++x) {
    if (radix[x][0] == 0) continue;
    AxisPlan p;
    p.n = cell->n[x];
    p.nst = 0;
    for (int i = 0; i < 4; ++i) p.R[i] = 1;
    for (int i = 0; i < 4 && radix[x][i] != 0; ++i) p.R[p.nst++] = radix[x][i];
    for (int i = p.nst; i < 4; ++i)
      if (radix[x][i] != 0) return false;
    if (!valid_axis_plan(p)) return false;
    ps->ax[x] = p;
    *any = true;
  }
  return true;
}

std::array<int, 5> vx_tune_key(const fx_cell* cell, fx_prec prec, bool square) {
  return {cell->n[0], cell->n[1], cell->n[2], (int)prec, square ? 1 : 0};
}

void resolve_vx_config(fx_ctx* ctx, VxArgs* a) {
  // environment overrides, for experiments and comparisons
  if (const char* e = getenv("FX_VX_NJ")) a->force_nj = atoi(e);
  if (const char* e = getenv("FX_VX_XT")) a->xtile = atoi(e);
  if (const char* e = getenv("FX_VX_PIPE")) a->pipe = atoi(e);
  if (const char* e = getenv("FX_VX_NTHR_B")) a->nthr_b = atoi(e);
  if (const char* e = getenv("FX_VX_HALVE")) a->halve = atoi(e);
  if (const char* e = getenv("FX_VX_A_PIPE")) a->a_pipe = atoi(e);
  if (const char* e = getenv("FX_VX_B_VAR")) a->b_var = atoi(e);
  if (const char* e = getenv("FX_VX_C_VAR")) a->c_var = atoi(e);
  if (const char* e = getenv("FX_VX_A_VAR")) a->a_var = atoi(e);
  if (const char* e = getenv("FX_VX_NT")) a->nt_hint = atoi(e);
  if (const char* e = getenv("FX_VX_C_SPLIT")) a->c_split = atoi(e);
  if (getenv("FX_VX_GENERIC")) a->kernels = 2;
  if (const char* e = getenv("FX_WORK_MB")) a->work_cap = (size_t)atol(e) << 20;
  if (!ctx) return;
  auto it = ctx->vx_tuning.find(vx_tune_key(a->cell, a->prec, vx_square_form(*a)));
  if (it == ctx->vx_tuning.end()) return;
  const fx_vx_config& c = it->second;
  if (!a->kernels) a->kernels = c.kernels;
  if (!a->work_cap && c.work_mb > 0) a->work_cap = (size_t)c.work_mb << 20;
  if (a->a_pipe < 0 && c.a_prefetch >= 0) a->a_pipe = c.a_prefetch;
  if (!a->b_var) a->b_var = c.b_variant;
  if (!a->c_var) a->c_var = c.c_variant;
  if (!a->a_var) a->a_var = c.a_variant;
  if (a->nt_hint < 0 && c.nt_hint >= 0) a->nt_hint = c.nt_hint;
  if (!a->c_split) a->c_split = c.c_split;
  if (!a->xtile) a->xtile = c.b_xtile;
  if (!a->nthr_b) a->nthr_b = c.b_threads;
  if (!a->plans_set) {
    bool any = false;
    PlanSet ps;
    if (plans_from_radix(a->cell, c.radix, &ps, &any) && any) {
      a->plans = ps;
      a->plans_set = true;
    }
  }
}

fx_status vx_apply(fx_ctx* ctx, Workspace* ws, const VxArgs& a_in, hipStream_t st, VxStats* stats) {
  FX_TRY(check_vx_args(a_in));
  VxArgs a = a_in;
  resolve_vx_config(ctx, &a);
  const int64_t nr = (int64_t)a.cell->n[0] * a.cell->n[1] * a.cell->n[2];
  const bool t64 = a.prec == FX_PREC_FP64;
  const bool same = a.phi == a.psi && a.ld_phi == a.ld_psi;
  const bool need_conv = (a.in_dtype == FX_C128) != t64;
  const GridTables* tb = nullptr;
  GridTables tb_scratch;
  if (a.segs.n > 0 && need_conv)
    FX_FAIL(FX_ERR_UNSUPPORTED, "multi-trajectory launches take orbitals in the compute type");
  if (a.no_alloc) {
    if (!ws->arena) FX_FAIL(FX_ERR_INVALID, "allocation-free call without a scratch region");
    if (need_conv)
      FX_FAIL(FX_ERR_UNSUPPORTED, "the allocation-free form takes %s inputs for this precision (no conversion)",
              t64 ? "complex128" : "complex64");
    a.halve = 0;
    FX_TRY(scratch_tables(ws, a.cell, a.kern, t64 ? 0 : 1, a.plans_set ? &a.plans : nullptr, st, &tb_scratch));
    tb = &tb_scratch;
    // what the scratch region must still hold besides the pair volume: partial
    // sums when out cannot hold them, and the energy partials
    const size_t asz = a.prec == FX_PREC_FP32 ? 8 : 16;
    const size_t reserve = (dtype_size(a.out_dtype) != asz ? (size_t)a.n_phi * nr * asz : 0) +
                           (a.ex_dev ? (size_t)a.n_phi * sizeof(double) : 0) + 3 * 256;
    const size_t used = (ws->arena_used + 255) & ~(size_t)255;
    const size_t room = ws->arena_bytes > used + reserve ? ws->arena_bytes - used - reserve : 0;
    const size_t pair_bytes = (size_t)nr * (t64 ? 16 : 8);
    if (room < pair_bytes)
      FX_FAIL(FX_ERR_INVALID,
              "the %zu-byte scratch region cannot hold one pair volume (%zu bytes) besides %zu bytes of tables and "
              "%zu of partial sums; the call is too large for the allocation-free form",
              ws->arena_bytes, pair_bytes, used, reserve);
    a.work_cap = a.work_cap ? std::min(a.work_cap, room) : room;
  } else {
    FX_TRY(grid_tables(ctx, a.cell, a.kern, t64 ? 0 : 1, a.plans_set ? &a.plans : nullptr, &tb));
  }
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
// IFFT_u[K FFT_u(conj(psi_j) phi_k)], with the device code's plans, twiddles,
// folded kernel table and z-tiling, in FP64 (prec 0) or FP32 (prec 1).
// Inputs and outputs are host arrays of N_r interleaved complex doubles.
template <typename T>
static void host_pair(const fx_cell* cell, const HostTables& h, const double* psi_j, const double* phi_k, double* v,
                      int xtile, const PlanSet* plans) {
  const PassGeom g = make_geom(cell, plans);
  const size_t nxy = (size_t)g.nx * g.ny, nr = nxy * g.nz;
  std::vector<cpx<T>> a(nr), b(nr), vol(nr);
  for (size_t i = 0; i < nr; ++i) {
    a[i] = {(T)psi_j[2 * i], (T)psi_j[2 * i + 1]};
    b[i] = {(T)phi_k[2 * i], (T)phi_k[2 * i + 1]};
  }
  std::vector<cpx<T>> tw[3];
  for (int ax = 0; ax < 3; ++ax)
    for (auto& c : h.tw[ax]) tw[ax].push_back({(T)c.x, (T)c.y});
  const int xt = std::max(1, std::min(g.nx, xtile));
  std::vector<cpx<T>> s((size_t)std::max(plane_lds_elems(g), g.nz * xt));
  for (int z = 0; z < g.nz; ++z)
    pass_a_body<T>(a.data() + z * nxy, b.data() + z * nxy, vol.data() + z * nxy, s.data(), tw[0].data(), tw[1].data(),
                   g, 0, 1, HostSync{});
  std::vector<T> kl((size_t)g.hz * g.hx);
  for (int y = 0; y < g.ny; ++y) {
    const int fy = h.fold[1][y];
    for (int fz = 0; fz < g.hz; ++fz)
      for (int fx = 0; fx < g.hx; ++fx) kl[fz * g.hx + fx] = (T)h.kfold[((size_t)fz * g.hy + fy) * g.hx + fx];
    for (int x0 = 0; x0 < g.nx; x0 += xt) {
      const KSlice<T> kf{kl.data(), h.fold[0].data(), h.fold[2].data(), x0, g.nx, g.hx};
      pass_b_body<T>(vol.data(), y, x0, xt, s.data(), tw[2].data(), kf, g, 0, 1, HostSync{});
    }
  }
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
  hipStream_t st = (hipStream_t)stream;
  FX_TRY(note_capture(ctx, st));
  if (ctx->graph_max <= 0) return vx_apply(ctx, &ctx->ws, a, st, nullptr);
  if (!cell || !kernel) FX_FAIL(FX_ERR_INVALID, "cell and kernel must be non-NULL");
  KeyBytes k;
  k.add(0).add(cell->n[0]).add(cell->n[1]).add(cell->n[2]).add(cell->len[0]).add(cell->len[1]).add(cell->len[2]);
  k.add(kernel->kind).add(kernel->omega).add(kernel->scale).add(psi).add(n_psi).add(ld_psi).add(phi).add(n_phi);
  k.add(ld_phi).add(out).add(ld_out).add(in_dtype).add(out_dtype).add(prec).add(ex_energy_dev);
  return graph_call(ctx, k.b, st, [&](hipStream_t s) { return vx_apply(ctx, &ctx->ws, a, s, nullptr); });
}

fx_status fx_debug_host_pair_plan(const fx_cell* cell, const fx_kernel* kernel, int prec, const int32_t* radix,
                                  const double* psi_j, const double* phi_k, double* v) {
  int xtile = cell ? cell->n[0] : 1;
  if (const char* e = getenv("FX_VX_XT")) xtile = atoi(e);
  clear_error();
  FX_TRY(check_cell(cell));
  FX_TRY(check_kernel(kernel));
  if (!psi_j || !phi_k || !v) FX_FAIL(FX_ERR_INVALID, "NULL host pointer");
  PlanSet ps;
  bool any = false;
  if (radix && !plans_from_radix(cell, reinterpret_cast<const int32_t(*)[4]>(radix), &ps, &any))
    FX_FAIL(FX_ERR_INVALID, "invalid radix schedule");
  const PlanSet* pp = radix ? &ps : nullptr;
  HostTables h;
  host_tables(cell, kernel, &h, pp);
  if (prec == 0)
    host_pair<double>(cell, h, psi_j, phi_k, v, xtile, pp);
  else
    host_pair<float>(cell, h, psi_j, phi_k, v, xtile, pp);
  return FX_OK;
}

fx_status fx_debug_host_pair(const fx_cell* cell, const fx_kernel* kernel, int prec, const double* psi_j,
                             const double* phi_k, double* v) {
  return fx_debug_host_pair_plan(cell, kernel, prec, nullptr, psi_j, phi_k, v);
}

fx_status fx_debug_axis_plans(int32_t n, int32_t max_plans, int32_t* radix_out, int32_t* count) {
  clear_error();
  if (!radix_out || !count || max_plans <= 0) FX_FAIL(FX_ERR_INVALID, "bad output arguments");
  if (!supported_edge(n)) FX_FAIL(FX_ERR_UNSUPPORTED, "edge %d is not 2^a 3^b in [2, 96]", n);
  std::vector<AxisPlan> ps((size_t)max_plans);
  const int k = enumerate_axis_plans(n, ps.data(), max_plans);
  for (int i = 0; i < k; ++i)
    for (int r = 0; r < 4; ++r) radix_out[4 * i + r] = r < ps[i].nst ? ps[i].R[r] : 0;
  *count = k;
  return FX_OK;
}

}  // extern "C"
