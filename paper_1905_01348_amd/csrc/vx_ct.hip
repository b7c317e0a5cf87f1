// V_X pair passes specialised at compile time for the cubic grids of the
// workloads (edges 24, 48, 72, 96).  Same three passes and data layout as the
// generic kernels in vx.hip (see vx_passes.hpp); every shape is a constant.
#include <algorithm>
#include <cstdlib>

#include "fft_ct.hpp"
#include "pair_order.hpp"
#include "vx.hpp"
#include "vx_passes.hpp"

namespace fx {

template <int A, int B>
struct CeilDiv {
  static constexpr int value = (A + B - 1) / B;
};

// Work of a persistent plane kernel: `units` (pairs, or targets) x N planes.
// Workgroups are dispatched round-robin over the XCDs, so with a grid that is
// a multiple of the XCD count workgroup b runs on XCD b % kXcds.  Each XCD
// takes either a contiguous chunk of the units (zsplit 0) or a contiguous
// range of N / kXcds planes of every unit (zsplit 1), and walks its share
// z-major: the workgroups of one XCD work on the same z at the same time and
// find that plane's input data (orbital and target planes in pass A, orbital
// planes in pass C) in their shared L2 instead of reading it again from HBM.
// With the z split no two XCDs read the same input plane.
constexpr int kXcds = 8;

struct ItemMap {
  int u_lo, u_n, z_lo, first, step, total;
  FX_HD void at(int li, int* unit, int* z) const {
    const int zz = li / u_n;
    *z = z_lo + zz;
    *unit = u_lo + (li - zz * u_n);
  }
};

template <int N>
__device__ inline ItemMap item_map(int units, int zsplit) {
  ItemMap m;
  const int G = gridDim.x, b = blockIdx.x;
  m.u_lo = 0;
  m.u_n = units;
  m.z_lo = 0;
  m.first = b;
  m.step = G;
  m.total = units * N;
  if (G >= kXcds && G % kXcds == 0) {
    const int x = b % kXcds;
    m.first = b / kXcds;
    m.step = G / kXcds;
    if (zsplit && N % kXcds == 0) {
      m.z_lo = x * (N / kXcds);
      m.total = units * (N / kXcds);
    } else {
      m.u_lo = (int)((int64_t)units * x / kXcds);
      m.u_n = (int)((int64_t)units * (x + 1) / kXcds) - m.u_lo;
      m.total = m.u_n * N;
    }
  }
  return m;
}

// ---- pass A: pair product, forward FFT x and y (persistent, pipelined) ------
// PIPE: the next plane's loads are issued into registers before the current
// plane is transformed (one workgroup per CU at 96^2); without it the kernel
// is held to the registers that let two workgroups share a CU instead (128
// VGPRs at 512 threads, 80 at 768).
template <typename T, bool PIPE, int NT>
struct PassAWaves {
  static constexpr int value = (sizeof(T) == 4 && !PIPE) ? (NT > 512 ? 6 : 4) : 1;
};

// WX: the product formed in the registers of a wave-level forward x
// transform (RowStage::fwd_x_wave; at 72^2 and 96^2 with one row
// butterfly per thread), whose results go to LDS once for the y transform.
// VEC: FP32 inputs 16-byte aligned with even leading dimensions (checked on
// the host): each thread loads two consecutive plane values at a time.
template <typename T, int N, bool PIPE, int NT, bool NTS, bool WX = false, bool VEC = false>
__global__ void __launch_bounds__(NT, (PassAWaves<T, PIPE, NT>::value)) k_pass_a_ct(const cpx<T>* __restrict__ psi, int64_t ld_psi,
                                                                  const cpx<T>* __restrict__ phi, int64_t ld_phi,
                                                                  cpx<T>* __restrict__ work, int j0, int nj, int k0,
                                                                  int tri, int nitems, const cpx<T>* __restrict__ twg,
                                                                  int zsplit, TrajSegs segs) {
  constexpr int NXY = N * N, SX = N + 1, EPT = CeilDiv<NXY, NT>::value;
  constexpr size_t NR = (size_t)NXY * N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* s = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = s + N * SX;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  cpx<T> va[EPT], vb[EPT];
  const ItemMap im = item_map<N>(nitems / N, zsplit & 1);
  const bool kBlocked = (zsplit >> 2) & 1;
  // VEC with whole pairs of values per thread: each thread takes two
  // consecutive plane values per load (16-byte loads, half the load
  // instructions); value i of the thread is plane element elem(i)
  constexpr bool kVec = VEC && sizeof(T) == 4 && NXY % (2 * NT) == 0;
  auto elem = [&](int i) __attribute__((always_inline)) {
    return kVec ? 2 * (tid + (i >> 1) * NT) + (i & 1) : tid + i * NT;
  };
  auto fetch = [&](int li) __attribute__((always_inline)) {
    if (li >= im.total) return;
    int p, z;
    im.at(li, &p, &z);
    p = unit_plane(p, nitems / N, nj, tri, kBlocked);
    int jj, kk;
    pair_of(p, nj, tri, &jj, &kk);
    const cpx<T>* a = seg_psi<T>(segs, psi, k0 + kk) + (int64_t)(j0 + jj) * ld_psi + (size_t)z * NXY;
    const cpx<T>* b = phi + (int64_t)(k0 + kk) * ld_phi + (size_t)z * NXY;
    if constexpr (kVec) {
#pragma unroll
      for (int i = 0; i < EPT; i += 2) {
        const float4 u = *reinterpret_cast<const float4*>(a + elem(i));
        const float4 v = *reinterpret_cast<const float4*>(b + elem(i));
        va[i] = cpx<T>{(T)u.x, (T)u.y};
        va[i + 1] = cpx<T>{(T)u.z, (T)u.w};
        vb[i] = cpx<T>{(T)v.x, (T)v.y};
        vb[i + 1] = cpx<T>{(T)v.z, (T)v.w};
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = elem(i);
      if (NXY % NT == 0 || e < NXY) {
        va[i] = a[e];
        vb[i] = b[e];
      }
    }
  };
  constexpr bool kPipe = PIPE;
  int li = im.first;
  if constexpr (WX) {
    using RS = RowStage<T, N, NT>;
    static_assert(RS::kWave && !PIPE, "wave-level form: 72^2 or 96^2, one butterfly per thread");
    __syncthreads();  // twiddles
    for (; li < im.total; li += im.step) {
      int p, z;
      im.at(li, &p, &z);
      p = unit_plane(p, nitems / N, nj, tri, kBlocked);
      int jj, kk;
      pair_of(p, nj, tri, &jj, &kk);
      const cpx<T>* a = seg_psi<T>(segs, psi, k0 + kk) + (int64_t)(j0 + jj) * ld_psi + (size_t)z * NXY;
      const cpx<T>* b = phi + (int64_t)(k0 + kk) * ld_phi + (size_t)z * NXY;
      cpx<T> x[RS::R];
#pragma unroll
      for (int m = 0; m < RS::R; ++m) {
        const int e = RS::fwd_pos(tid, m);
        x[m] = cconjmul(a[e], b[e]);
      }
      RS::template fwd_x_wave<SX>(x, s, tw, tid);
      __syncthreads();
      constexpr int R0 = Plan2<N>::R0, R1 = Plan2<N>::R1;
      ct_stage<R0, true, T, N, N, N, SX, 1, NT>(s, tw, tid);
      __syncthreads();
      cpx<T>* o = work + p * NR + (size_t)z * NXY;
      if constexpr (sizeof(T) == 4 && PairIO<R1, N, N, NT>::kFits)
        ct_stage_io_pair<R1, true, T, N, N, SX, NT, false, true, N, NTS>(s, nullptr, o, tid);
      else
        ct_stage_io<R1, true, T, N, R1, N, SX, 1, NT, false, true, N, 1, NTS>(s, nullptr, o, tw, tid);
      __syncthreads();
    }
    return;
  }
  if (kPipe) fetch(li);
  for (; li < im.total; li += im.step) {
    if (!kPipe) fetch(li);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = elem(i);
      if (NXY % NT == 0 || e < NXY) s[(e / N) * SX + e % N] = cconjmul(va[i], vb[i]);
    }
    __syncthreads();
    if (kPipe) fetch(li + im.step);
    ct_fft<true, T, N, N, 1, SX, NT>(s, tw, tid);
    // y: first stage in LDS, last stage straight to the work plane
    constexpr int R0 = Plan2<N>::R0, R1 = Plan2<N>::R1;
    ct_stage<R0, true, T, N, N, N, SX, 1, NT>(s, tw, tid);
    __syncthreads();
    int p, z;
    im.at(li, &p, &z);
    p = unit_plane(p, nitems / N, nj, tri, kBlocked);
    cpx<T>* o = work + p * NR + (size_t)z * NXY;
    // FP32 with one pair of columns per thread: 16-byte stores
    if constexpr (sizeof(T) == 4 && PairIO<R1, N, N, NT>::kFits)
      ct_stage_io_pair<R1, true, T, N, N, SX, NT, false, true, N, NTS>(s, nullptr, o, tid);
    else
      ct_stage_io<R1, true, T, N, R1, N, SX, 1, NT, false, true, N, 1, NTS>(s, nullptr, o, tw, tid);
    __syncthreads();
  }
}

// ---- pass B: z convolution on an x tile ---------------------------------------
template <typename T, int N, int XT, int NT, bool NTS>
__global__ void __launch_bounds__(NT) k_pass_b_ct(cpx<T>* __restrict__ work, const cpx<T>* __restrict__ twg,
                                                  const T* __restrict__ kfold, const int* __restrict__ foldg) {
  constexpr int NTX = N / XT, NE = N * XT;
  constexpr int H = N / 2 + 1;
  static_assert(N % XT == 0, "x tile must divide the edge");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* s = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = s + NE;
  T* kl = reinterpret_cast<T*>(tw + N);
  int* fl = reinterpret_cast<int*>(kl + H * H);
  const int tid = threadIdx.x;
  const int tx = blockIdx.x % NTX;
  const int rest = blockIdx.x / NTX;
  const int y = rest % N;
  const int p = rest / N;
  const int x0 = tx * XT;
  cpx<T>* vol = work + (size_t)p * N * N * N;
  cpx<T>* g0 = vol + (size_t)y * N + x0;  // element (xi, z) at g0[xi + z*N*N]
  const int fy = foldg[y];
  for (int i = tid; i < N; i += NT) {
    tw[i] = twg[i];
    fl[i] = foldg[i];
  }
  for (int i = tid; i < H * H; i += NT) kl[i] = kfold[((size_t)(i / H) * H + fy) * H + i % H];
  constexpr int R0 = Plan2<N>::R0, R1 = Plan2<N>::R1;
  // first forward stage straight from the work volume (twiddles from the
  // cached global table: the LDS copy is not yet visible)
  ct_stage_io<R0, true, T, N, N, XT, XT, 1, NT, true, false, N * N, 1, NTS>(s, g0, nullptr, twg, tid);
  __syncthreads();
  // last forward stage x K x first inverse stage, in registers
  {
    constexpr int TOTAL = XT * (N / R1);
    constexpr int ITERS = (TOTAL + NT - 1) / NT;
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      const int b = tid + it * NT;
      if (TOTAL % NT == 0 || b < TOTAL) {
        const int f = b % XT;
        const int blk = b / XT;
        const int base = f + blk * R1 * XT;
        const int kx = fl[x0 + f];
        cpx<T> xv[R1];
#pragma unroll
        for (int m = 0; m < R1; ++m) xv[m] = s[base + m * XT];
        Dft<R1, -1, T>::run(xv);
#pragma unroll
        for (int k = 0; k < R1; ++k) xv[k] = cscale(xv[k], kl[fl[blk * R1 + k] * H + kx]);
        Dft<R1, 1, T>::run(xv);
#pragma unroll
        for (int m = 0; m < R1; ++m) s[base + m * XT] = xv[m];
      }
    }
  }
  __syncthreads();
  // last inverse stage straight back to the work volume
  ct_stage_io<R0, false, T, N, N, XT, XT, 1, NT, false, true, N * N, 1, NTS>(s, nullptr, g0, tw, tid);
}

// Asynchronous copy of one N x N plane from global memory into LDS, 16 bytes
// per lane (global_load_lds_dwordx4: lane i of a wave-instruction fills bytes
// [16 i, 16 i + 16) after the wave-uniform LDS address, so only full waves
// take part).  No registers hold the data in flight; the copy completes on
// the wave's vector-memory counter, so a reader waits for that counter to
// drain and then for a barrier.
template <typename T, int N, int NT, bool NTS>
__device__ inline void plane_to_lds(const cpx<T>* g, cpx<T>* lds, int tid) {
  static_assert((N * N * sizeof(cpx<T>)) % 16 == 0, "plane bytes must be a multiple of 16");
  constexpr int CH = (int)(N * N * sizeof(cpx<T>) / 16);  // 16-byte chunks
  // full waves share the wave-instructions (a last partial wave does none)
  constexpr int NW = NT / 64, WI = CeilDiv<CH, 64>::value;
  static_assert(NW >= 1, "at least one full wave");
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  if (NT % 64 != 0 && w >= NW) return;
  const char* gb = reinterpret_cast<const char*>(g);
  auto lb = (__attribute__((address_space(3))) char*)(reinterpret_cast<char*>(lds));
#pragma unroll
  for (int i = 0; i < CeilDiv<WI, NW>::value; ++i) {
    const int wi = i * NW + w;
    if (WI % NW == 0 || wi < WI) {
      const int c = wi * 64 + lane;
      if (CH % 64 == 0 || c < CH)
        __builtin_amdgcn_global_load_lds(gb + (size_t)c * 16, lb + wi * 1024, 16, 0, NTS ? 2 : 0);
    }
  }
}

// ---- pass B, persistent form -----------------------------------------------------
// The same tile transform as k_pass_b_ct, with a fixed y per workgroup (the K
// slice of that y is loaded into LDS once) and the tiles (pair, x tile) of
// that y walked in order by the grid / N workgroups of that y: the
// workgroups running at one time cover every y of the same few pair volumes.
// The first stage's loads of the next tile are issued before the current
// tile's middle and last stages, so HBM reads stay in flight while the
// workgroup computes.  The grid is a multiple of N.
template <typename T, int N, int XT, int NT, bool NTS>
__global__ void __launch_bounds__(NT) k_pass_b_pt(cpx<T>* __restrict__ work, const cpx<T>* __restrict__ twg,
                                                  const T* __restrict__ kfold, const int* __restrict__ foldg,
                                                  int ntiles) {
  constexpr int NTX = N / XT, NE = N * XT;
  constexpr int H = N / 2 + 1;
  static_assert(N % XT == 0, "x tile must divide the edge");
  constexpr int R0 = Plan2<N>::R0, R1 = Plan2<N>::R1;
  constexpr int IT0 = StageIters<R0, N, XT, NT>::value;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* s = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = s + NE;
  T* kl = reinterpret_cast<T*>(tw + N);
  int* fl = reinterpret_cast<int*>(kl + H * H);
  const int tid = threadIdx.x;
  const int y = blockIdx.x % N;
  const int step = gridDim.x / N;
  const int fy = foldg[y];
  for (int i = tid; i < N; i += NT) {
    tw[i] = twg[i];
    fl[i] = foldg[i];
  }
  for (int i = tid; i < H * H; i += NT) kl[i] = kfold[((size_t)(i / H) * H + fy) * H + i % H];
  // tile u = (pair u / NTX, x tile u % NTX); element (xi, z) at g[xi + z*N*N]
  auto tile = [&](int u) __attribute__((always_inline)) {
    return work + (size_t)(u / NTX) * N * N * N + (size_t)y * N + (u % NTX) * XT;
  };
  cpx<T> x0[IT0][R0];
  int u = blockIdx.x / N;
  if (u < ntiles) ct_bfly_load<R0, T, N, N, XT, NT, true, N * N, 1, XT, 1, NTS>(x0, tile(u), tid);
  __syncthreads();  // tables
  for (; u < ntiles; u += step) {
    const int x0t = (u % NTX) * XT;
    cpx<T>* g0 = tile(u);
    // first forward stage from the registers loaded ahead
    ct_bfly_run<R0, true, T, N, N, XT, NT>(x0, tw, tid);
    ct_bfly_store<R0, T, N, N, XT, NT, false, N * N, 1, XT, 1, false>(x0, s, tid);
    __syncthreads();
    // the next tile's first-stage loads, in flight during the rest of this one
    if (u + step < ntiles) ct_bfly_load<R0, T, N, N, XT, NT, true, N * N, 1, XT, 1, NTS>(x0, tile(u + step), tid);
    // last forward stage x K x first inverse stage, in registers
    {
      constexpr int TOTAL = XT * (N / R1);
      constexpr int ITERS = (TOTAL + NT - 1) / NT;
#pragma unroll
      for (int it = 0; it < ITERS; ++it) {
        const int b = tid + it * NT;
        if (TOTAL % NT == 0 || b < TOTAL) {
          const int f = b % XT;
          const int blk = b / XT;
          const int base = f + blk * R1 * XT;
          const int kx = fl[x0t + f];
          cpx<T> xv[R1];
#pragma unroll
          for (int m = 0; m < R1; ++m) xv[m] = s[base + m * XT];
          Dft<R1, -1, T>::run(xv);
#pragma unroll
          for (int k = 0; k < R1; ++k) xv[k] = cscale(xv[k], kl[fl[blk * R1 + k] * H + kx]);
          Dft<R1, 1, T>::run(xv);
#pragma unroll
          for (int m = 0; m < R1; ++m) s[base + m * XT] = xv[m];
        }
      }
    }
    __syncthreads();
    // last inverse stage straight back to the work volume
    ct_stage_io<R0, false, T, N, N, XT, XT, 1, NT, false, true, N * N, 1, NTS>(s, nullptr, g0, tw, tid);
    __syncthreads();  // before the next tile's first stage writes s
  }
}

// ---- pass C: inverse FFT y and x, times psi_j, j-sum in registers --------------
// One item = (target tt of the batch, plane z).  Role 0 (CONJ false): the
// targets are the batch's k (output column t0 + kk) and the sum runs over its
// j in ascending order, adding psi_{m0+jj} * v_{jk}.  Role 1 (CONJ true, the
// second half of a halved apply): the targets are the batch's j and the sum
// runs over its k in ascending order, adding psi_{m0+kk} * conj(v_{jk}),
// which is v_{kj} since the kernel is real and even.  On a diagonal batch
// (tri) role 0 takes jj <= kk and role 1 kk > jj.
// FORM 0: the plain form; 1 (STG): the next work plane (this item's next
// term, or the next item's first)
// is copied into a second LDS buffer while the current one is transformed, so
// the first inverse stage reads LDS instead of waiting on HBM with the whole
// workgroup (one workgroup per CU at 96^2, where the registers of the
// accumulators leave LDS to spare).  At 96^3 it measured slightly slower than
// the plain form (3.19 vs 3.13 ms per launch): a tuner candidate.  FORM 2
// (WX): the inverse x transform across the lanes of a wave (RowStage).
// FORM 2 at one butterfly per thread with two work planes in LDS: the terms
// alternate between them, so a term's first stage need not wait for the
// previous term's last reads (one barrier fewer per term).
// The FP32 plain form (FORM 0) does the same where two planes take at most
// 40 KB (edges 24 and 48), so that as many workgroups share a CU as with one
// (48^3 request: 0.333 -> 0.321 ms per launch).  In FP64 at 48^2 the larger
// planes cost workgroups per CU (halved 48^3 apply 822k -> 711k pairs/s).
template <typename T, int N, int NT, int FORM>
struct PassCDouble {
  static constexpr size_t kBytes = (2 * (size_t)N * (N + 1) + N) * sizeof(cpx<T>);
  static constexpr bool value = sizeof(T) == 4 && ((FORM == 2 && RowStage<T, N, NT>::kWave && kBytes <= 160 * 1024) ||
                                                   (FORM == 0 && kBytes <= 40 * 1024));
};

template <typename T, typename A, int N, bool CONJ, int NT, bool NTS, int FORM>
__global__ void __launch_bounds__(NT) k_pass_c_ct(const cpx<T>* __restrict__ mult, int64_t ld_mult,
                                                                  const cpx<T>* __restrict__ work, int nj, int nk,
                                                                  int tri, int m0, int t0, int nitems, cpx<A>* acc,
                                                                  int64_t ld_acc, int first, void* out, int64_t ld_out,
                                                                  int out_c64, int last, const cpx<T>* __restrict__ twg,
                                                                  int zsplit, TrajSegs segs, int jsplit, int64_t gstride) {
  constexpr int NXY = N * N, SX = N + 1, EPT = CeilDiv<NXY, NT>::value;
  constexpr size_t NR = (size_t)NXY * N;
  constexpr bool STG = FORM == 1, WX = FORM == 2;
  constexpr bool kDbl = PassCDouble<T, N, NT, FORM>::value;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* s = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = s + (kDbl ? 2 : 1) * N * SX;
  cpx<T>* stg = tw + N;  // STG only: N*N staged work plane, 16-byte aligned
  int par = 0;           // kDbl: the work plane of the current term
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  __syncthreads();
  // units: (target tt, sum group g) as tt * jsplit + g
  const ItemMap im = item_map<N>(nitems / N, zsplit);
  // terms l = lo, lo + jsplit, ... < hi of target tt in group g: the terms
  // whose orbital m0 + l is g modulo jsplit, in ascending order
  auto range = [&](int tt_, int g_, int* lo_, int* hi_) __attribute__((always_inline)) {
    int lo = CONJ ? (tri ? tt_ + 1 : 0) : 0;
    *hi_ = CONJ ? nk : (tri ? tt_ + 1 : nj);
    const int r = (m0 + lo) % jsplit;
    *lo_ = lo + (g_ >= r ? g_ - r : g_ - r + jsplit);
  };
  auto plane_ptr = [&](int tt_, int l_, int z_) __attribute__((always_inline)) {
    const int pl = CONJ ? plane_of(tt_, l_, nj, tri) : plane_of(l_, tt_, nj, tri);
    return work + (size_t)pl * NR + (size_t)z_ * NXY;
  };
  bool staged = false;  // STG: stg holds (or is receiving) this item's first term
  // FP64: the orbital plane is loaded only before the last x stage, so that
  // its registers are not live through the y stages beside the accumulators
  // (loaded early it spills at 96^2)
  constexpr bool kLateOrbital = sizeof(T) == 8;
  // of those, the values loaded before the last x stage: half, the other half
  // once the stage's registers are free (all of them beside the stage spilled
  // 164 bytes per lane at 96^2, half of them 132; 2.73 -> 2.51 ms per launch)
  constexpr int kEarly = (kLateOrbital && !STG) ? (EPT + 1) / 2 : EPT;
  // FP32 plain form with one last-stage butterfly per thread (96^2 at 768
  // threads, 72^2 at 576): the last inverse x stage accumulates from its
  // registers (RowStage), and the sums are held at the plane positions that
  // stage leaves in each thread.  At 96^3 this took the pass from 3.06 to
  // 2.79 ms per launch.  With more butterflies than threads, or idle threads,
  // the extra accumulators cost more registers than the saved LDS round trip
  // and barrier are worth.
  // WX: the whole inverse x transform in registers and across lanes
  // (RowStage::inv_x_wave): one LDS pass and one barrier fewer again.  In
  // FP64 this is the one register form (the orbital values loaded after the
  // transform): 2.50 -> 2.38 ms per launch at 96^3, 2.43 -> 2.23 at 72^3.
  using LX = RowStage<T, N, NT>;
  constexpr bool kRegX = (sizeof(T) == 4 || WX) && !STG && LX::TOTAL == NT;
  static_assert(!WX || (kRegX && LX::kWave), "wave-level form: 72^2 or 96^2, one butterfly per thread");
  // plane position of value m of butterfly it of this thread in the register form
  auto rpos = [&](int it, int m) __attribute__((always_inline)) {
    return WX ? LX::wave_pos(tid, m) : LX::pos(tid, it, m);
  };
  for (int li = im.first; li < im.total; li += im.step) {
    int u, z;
    im.at(li, &u, &z);
    const int tt = u / jsplit, g = u - tt * jsplit;
    const int t = t0 + tt;
    cpx<A>* accg = acc + g * gstride;  // this group's partial sums
    if constexpr (kRegX) {
      cpx<A> a[LX::IT][LX::R];
      cpx<T> vp[LX::IT][LX::R];
#pragma unroll
      for (int it = 0; it < LX::IT; ++it)
#pragma unroll
        for (int m = 0; m < LX::R; ++m) {
          a[it][m] = cpx<A>{0, 0};
          if (!first && LX::owns(tid, it)) a[it][m] = accg[t * ld_acc + (size_t)z * NXY + rpos(it, m)];
        }
      int lo, hi;
      range(tt, g, &lo, &hi);
      for (int l = lo; l < hi; l += jsplit) {
        const cpx<T>* pm = seg_psi<T>(segs, mult, t) + (int64_t)(m0 + l) * ld_mult + (size_t)z * NXY;
        constexpr int R0 = Plan2<N>::R0, R1 = Plan2<N>::R1;
        cpx<T>* sl = s + (kDbl ? par * N * SX : 0);
        // (16-byte paired loads here measured slower: 3.08 against 2.76 ms
        // per launch at 96^3, with a quarter of the threads idle in this stage)
        ct_stage_io<R1, false, T, N, R1, N, SX, 1, NT, true, false, N, 1, NTS>(sl, plane_ptr(tt, l, z), nullptr, tw,
                                                                              tid);
        __syncthreads();
        if constexpr (!kLateOrbital) {
#pragma unroll
          for (int it = 0; it < LX::IT; ++it)
#pragma unroll
            for (int m = 0; m < LX::R; ++m)
              if (LX::owns(tid, it)) vp[it][m] = pm[rpos(it, m)];
        }
        ct_stage<R0, false, T, N, N, N, SX, 1, NT>(sl, tw, tid);
        __syncthreads();
        cpx<T> x[LX::IT][LX::R];
        if constexpr (WX) {
          LX::template inv_x_wave<SX>(sl, tw, tid, x[0]);
        } else {
          ct_stage<R1, false, T, N, R1, N, 1, SX, NT>(sl, tw, tid);
          __syncthreads();
          LX::template inv_from_lds<SX>(sl, tw, tid, x);
        }
        // FP64 (wave-level form): the orbital values once the transform's
        // registers are free
        if constexpr (kLateOrbital) {
#pragma unroll
          for (int it = 0; it < LX::IT; ++it)
#pragma unroll
            for (int m = 0; m < LX::R; ++m)
              if (LX::owns(tid, it)) vp[it][m] = pm[rpos(it, m)];
        }
#pragma unroll
        for (int it = 0; it < LX::IT; ++it)
#pragma unroll
          for (int m = 0; m < LX::R; ++m)
            if (LX::owns(tid, it)) {
              const cpx<A> va{(A)x[it][m].x, CONJ ? -(A)x[it][m].y : (A)x[it][m].y};
              a[it][m] = cfma(a[it][m], cpx<A>{(A)vp[it][m].x, (A)vp[it][m].y}, va);
            }
        // the last stage's reads before the next term's writes of the plane:
        // with two planes, the next term writes the other one, and the term
        // after it waits at that term's barriers
        if constexpr (kDbl)
          par ^= 1;
        else
          __syncthreads();
      }
#pragma unroll
      for (int it = 0; it < LX::IT; ++it)
#pragma unroll
        for (int m = 0; m < LX::R; ++m) {
          if (!LX::owns(tid, it)) continue;
          const size_t off = (size_t)z * NXY + rpos(it, m);
          if (last) {
            if (out_c64)
              reinterpret_cast<cpx<float>*>(out)[t * ld_out + off] = cpx<float>{(float)a[it][m].x, (float)a[it][m].y};
            else
              reinterpret_cast<cpx<double>*>(out)[t * ld_out + off] = cpx<double>{(double)a[it][m].x, (double)a[it][m].y};
          } else {
            accg[t * ld_acc + off] = a[it][m];
          }
        }
      continue;
    }
    cpx<A> a[EPT];
    cpx<T> vp[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * NT;
      a[i] = cpx<A>{0, 0};
      if (!first && (NXY % NT == 0 || e < NXY)) a[i] = accg[t * ld_acc + (size_t)z * NXY + e];
    }
    constexpr int R0 = Plan2<N>::R0, R1 = Plan2<N>::R1;
    int lo, hi;
    range(tt, g, &lo, &hi);
    for (int l = lo; l < hi; l += jsplit) {
      // (multi-trajectory launches are never halved: role 0, target t's own orbitals)
      const cpx<T>* pm = seg_psi<T>(segs, mult, t) + (int64_t)(m0 + l) * ld_mult + (size_t)z * NXY;
      cpx<T>* sl = s + (kDbl ? par * N * SX : 0);
      if (STG) {
        if (!staged) plane_to_lds<T, N, NT, NTS>(plane_ptr(tt, l, z), stg, tid);
        __builtin_amdgcn_s_waitcnt(0);  // this wave's part of the copy has landed
        __syncthreads();                // ... and every other wave's
        // first inverse y stage from the staged plane
        ct_stage_io<R1, false, T, N, R1, N, SX, 1, NT, true, false, N, 1, false>(sl, stg, nullptr, tw, tid);
        __syncthreads();  // stg is free again
        // orbital plane first: waiting for it must not wait for the copy below
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
          const int e = tid + i * NT;
          if (NXY % NT == 0 || e < NXY) vp[i] = pm[e];
        }
        __builtin_amdgcn_sched_barrier(0);
        // start copying the next term: this item's, else the next item's first
        staged = false;
        if (l + jsplit < hi) {
          plane_to_lds<T, N, NT, NTS>(plane_ptr(tt, l + jsplit, z), stg, tid);
          staged = true;
        } else if (li + im.step < im.total) {
          int u2, z2, lo2, hi2;
          im.at(li + im.step, &u2, &z2);
          const int tt2 = u2 / jsplit;
          range(tt2, u2 - tt2 * jsplit, &lo2, &hi2);
          if (lo2 < hi2) {
            plane_to_lds<T, N, NT, NTS>(plane_ptr(tt2, lo2, z2), stg, tid);
            staged = true;
          }
        }
      } else {
        // first inverse y stage straight from the work plane
        ct_stage_io<R1, false, T, N, R1, N, SX, 1, NT, true, false, N, 1, NTS>(sl, plane_ptr(tt, l, z), nullptr, tw,
                                                                              tid);
        __syncthreads();
        if (!kLateOrbital) {
#pragma unroll
          for (int i = 0; i < EPT; ++i) {
            const int e = tid + i * NT;
            if (NXY % NT == 0 || e < NXY) vp[i] = pm[e];
          }
        }
      }
      ct_stage<R0, false, T, N, N, N, SX, 1, NT>(sl, tw, tid);
      __syncthreads();
      // inverse x: its two stages (ct_fft's), the orbital plane loaded between
      // them in FP64
      ct_stage<R1, false, T, N, R1, N, 1, SX, NT>(sl, tw, tid);
      __syncthreads();
      if (!STG && kLateOrbital) {
#pragma unroll
        for (int i = 0; i < kEarly; ++i) {
          const int e = tid + i * NT;
          if (NXY % NT == 0 || e < NXY) vp[i] = pm[e];
        }
      }
      ct_stage<R0, false, T, N, N, N, 1, SX, NT>(sl, tw, tid);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NT;
        // FP64: the second half of the orbital values, once the last stage's
        // registers are free
        if (!STG && kLateOrbital && i == kEarly) {
#pragma unroll
          for (int i2 = kEarly; i2 < EPT; ++i2) {
            const int e2 = tid + i2 * NT;
            if (NXY % NT == 0 || e2 < NXY) vp[i2] = pm[e2];
          }
        }
        if (NXY % NT == 0 || e < NXY) {
          const cpx<T> v = sl[(e / N) * SX + e % N];
          const cpx<A> va{(A)v.x, CONJ ? -(A)v.y : (A)v.y};
          // FP32 transforms: four FMAs per term; FP64: product then sum (the
          // FMA chain costs the FP64 kernel registers it does not have)
          if constexpr (sizeof(T) == 4)
            a[i] = cfma(a[i], cpx<A>{(A)vp[i].x, (A)vp[i].y}, va);
          else
            a[i] = cadd(a[i], cmul(cpx<A>{(A)vp[i].x, (A)vp[i].y}, va));
        }
      }
      // (STG: the barrier at the top of the next term orders these reads
      // before the next writes of s; kDbl: the next term writes the other
      // plane)
      if constexpr (kDbl)
        par ^= 1;
      else if (!STG)
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * NT;
      if (!(NXY % NT == 0 || e < NXY)) continue;
      const size_t off = (size_t)z * NXY + e;
      if (last) {
        if (out_c64)
          reinterpret_cast<cpx<float>*>(out)[t * ld_out + off] = cpx<float>{(float)a[i].x, (float)a[i].y};
        else
          reinterpret_cast<cpx<double>*>(out)[t * ld_out + off] = cpx<double>{(double)a[i].x, (double)a[i].y};
      } else {
        accg[t * ld_acc + off] = a[i];
      }
    }
  }
}

// ---- host side ------------------------------------------------------------------
bool ct_supported(const fx_cell* cell) {
  const int n = cell->n[0];
  if (cell->n[1] != n || cell->n[2] != n) return false;
  AxisPlan p;
  if (!make_axis_plan(n, &p) || p.nst != 2) return false;
  switch (n) {
    case 24: return p.R[0] == Plan2<24>::R0 && p.R[1] == Plan2<24>::R1;
    case 48: return p.R[0] == Plan2<48>::R0 && p.R[1] == Plan2<48>::R1;
    case 72: return p.R[0] == Plan2<72>::R0 && p.R[1] == Plan2<72>::R1;
    case 96: return p.R[0] == Plan2<96>::R0 && p.R[1] == Plan2<96>::R1;
    default: return false;
  }
}

template <typename K>
static fx_status ct_prepare(fx_ctx* ctx, K kernel, int nthr, size_t lds, int items, bool persistent, int* grid) {
  FX_TRY(allow_dynamic_lds(reinterpret_cast<const void*>(kernel), lds));
  if (!persistent) {
    *grid = items;
    return FX_OK;
  }
  int per_cu = 0;
  FX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), nthr, lds));
  int g = std::max(1, std::min(items, std::max(per_cu, 1) * std::max(ctx->n_cu, 1)));
  // a multiple of the XCD count, so that each XCD walks its own chunk (item_map)
  if (g >= kXcds) g -= g % kXcds;
  *grid = g;
  return FX_OK;
}

// Inputs that allow 16-byte loads of two plane values: FP32, every orbital
// and target base 16-byte aligned, even leading dimensions (plane offsets are
// even: N^2 is).
template <typename T>
static bool pass_a_vec_ok(const CtBatch<T>& b) {
  if (sizeof(T) != 4 || (b.ld_psi & 1) || (b.ld_phi & 1)) return false;
  uintptr_t bits = reinterpret_cast<uintptr_t>(b.psi) | reinterpret_cast<uintptr_t>(b.phi);
  for (int i = 0; i < b.segs.n; ++i) bits |= reinterpret_cast<uintptr_t>(b.segs.psi[i]);
  return (bits & 15) == 0;
}

template <typename T, int N, int NT, bool WX = false>
static fx_status pass_a_shape(fx_ctx* ctx, hipStream_t st, const CtBatch<T>& b) {
  const size_t lds = ((size_t)N * (N + 1) + N) * sizeof(cpx<T>);
  // the blocked pair order (bit 2 of zsplit) for the FP32 form with
  // coalesced loads only: the wave-level forms measured slower with it
  // (FP32 at 72^3: 0.705 -> 0.800 ms per launch; FP64 at 96^3: 2.53 -> 2.66)
  // the prefetching form exists for FP32 only (FP64 has no registers to spare)
  constexpr bool F32 = sizeof(T) == 4;
  const bool pipe = F32 && b.a_pipe && !WX;
  const bool vec = F32 && !WX && pass_a_vec_ok(b);
  auto kern = WX     ? (b.nts ? k_pass_a_ct<T, N, false, NT, true, WX> : k_pass_a_ct<T, N, false, NT, false, WX>)
              : pipe ? (vec ? (b.nts ? k_pass_a_ct<T, N, F32, NT, true, false, F32> : k_pass_a_ct<T, N, F32, NT, false, false, F32>)
                            : (b.nts ? k_pass_a_ct<T, N, F32, NT, true> : k_pass_a_ct<T, N, F32, NT, false>))
                     : (vec ? (b.nts ? k_pass_a_ct<T, N, false, NT, true, false, F32> : k_pass_a_ct<T, N, false, NT, false, false, F32>)
                            : (b.nts ? k_pass_a_ct<T, N, false, NT, true> : k_pass_a_ct<T, N, false, NT, false>));
  const int items = b.npairs * N;
  int grid = 0;
  FX_TRY(ct_prepare(ctx, kern, NT, lds, items, true, &grid));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, b.psi, b.ld_psi, b.phi, b.ld_phi, b.work, b.j0, b.nj, b.k0,
                     b.tri, items, b.tw, b.zsplit & (sizeof(T) == 4 && !WX ? 5 : 1), b.segs);
  FX_LAUNCH_CHECK();
  return FX_OK;
}

template <typename T, int N>
static fx_status pass_a_n(fx_ctx* ctx, hipStream_t st, const CtBatch<T>& b) {
  using S = CubeShape<N>;
  constexpr bool kWx = RowStage<T, N, S::NT_A2>::kWave;
  // automatic: the wave-level form in FP64 where it exists (one workgroup per
  // CU, whose barriers it halves: 3.21 -> 2.57-2.66 ms per launch of 585 pairs
  // at 96^3, 2.87 -> 2.75 at 72^3); FP32 keeps the default threads
  const int av = b.a_var ? b.a_var : (sizeof(T) == 8 && kWx ? 3 : 1);
  // the wave-level form: at 72 and 96, with the second thread count
  if constexpr (kWx)
    if (av == 3) return pass_a_shape<T, N, S::NT_A2, true>(ctx, st, b);
  if (av == 2 || av == 3) return pass_a_shape<T, N, S::NT_A2>(ctx, st, b);
  return pass_a_shape<T, N, S::NT_P>(ctx, st, b);
}

// LDS of one z-pass workgroup with an x tile of xt columns
template <typename T, int N>
constexpr size_t pass_b_lds(int xt) {
  return ((size_t)N * xt + N) * sizeof(cpx<T>) + (size_t)(N / 2 + 1) * (N / 2 + 1) * sizeof(T) + (size_t)N * sizeof(int);
}
constexpr size_t kLdsPerCu = 160 * 1024;

template <typename T, int N, int XT, int NT>
static fx_status pass_b_shape(fx_ctx* ctx, hipStream_t st, const CtBatch<T>& b) {
  static_assert(N % XT == 0, "x tile must divide the edge");
  const size_t lds = pass_b_lds<T, N>(XT);
  auto kern = b.nts ? k_pass_b_ct<T, N, XT, NT, true> : k_pass_b_ct<T, N, XT, NT, false>;
  const int items = b.npairs * N * (N / XT);
  int grid = 0;
  FX_TRY(ct_prepare(ctx, kern, NT, lds, items, false, &grid));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, b.work, b.tw, b.kfold, b.fold);
  FX_LAUNCH_CHECK();
  return FX_OK;
}

template <typename T, int N, int XT, int NT>
static fx_status pass_b_pt_shape(fx_ctx* ctx, hipStream_t st, const CtBatch<T>& b) {
  static_assert(N % XT == 0, "x tile must divide the edge");
  const size_t lds = pass_b_lds<T, N>(XT);
  auto kern = b.nts ? k_pass_b_pt<T, N, XT, NT, true> : k_pass_b_pt<T, N, XT, NT, false>;
  const int ntiles = b.npairs * (N / XT);
  FX_TRY(allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds));
  int per_cu = 0;
  FX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), NT, lds));
  // a whole number of workgroups per y that all run at once, no more than the
  // tiles of a y (at 96^3 with whole rows: 2 per y, 192 of the 256 CUs, which
  // measured faster than 256 workgroups over all CUs: the z pass runs at the
  // HBM limit and gains more from the locality of a fixed y than from CUs)
  int per_y = std::max(1, std::max(per_cu, 1) * std::max(ctx->n_cu, 1) / N);
  per_y = std::min(per_y, ntiles);
  hipLaunchKernelGGL(kern, dim3(per_y * N), dim3(NT), lds, st, b.work, b.tw, b.kfold, b.fold, ntiles);
  FX_LAUNCH_CHECK();
  return FX_OK;
}

template <typename T, int N>
static fx_status pass_b_n(fx_ctx* ctx, hipStream_t st, const CtBatch<T>& b) {
  using S = CubeShape<N>;
  // persistent form: whole x rows where they fit the LDS (not FP64 at 96), else the default tile
  if (b.b_var == 4) {
    if constexpr (pass_b_lds<T, N>(S::XT3) <= kLdsPerCu) return pass_b_pt_shape<T, N, S::XT3, S::NT_BP>(ctx, st, b);
    return pass_b_pt_shape<T, N, S::XT, S::NT_B>(ctx, st, b);
  }
  if (b.b_var == 2) return pass_b_shape<T, N, S::XT2, S::NT_B2>(ctx, st, b);
  // whole rows do not fit the LDS in FP64 at 96: the default tile instead
  if (b.b_var == 3 && pass_b_lds<T, N>(S::XT3) <= kLdsPerCu) return pass_b_shape<T, N, S::XT3, S::NT_B3>(ctx, st, b);
  return pass_b_shape<T, N, S::XT, S::NT_B>(ctx, st, b);
}

// LDS of one plane-inverse workgroup (STG: with the staged next plane)
template <typename T, int N>
constexpr size_t pass_c_lds(bool stg) {
  return ((size_t)N * (N + 1) + N + (stg ? (size_t)N * N : 0)) * sizeof(cpx<T>);
}

template <typename T, typename A, int N, int NT, int FORM>
static fx_status pass_c_shape(fx_ctx* ctx, hipStream_t st, const CtBatch<T>& b, const CtAcc<A>& c, int role) {
  const size_t lds = PassCDouble<T, N, NT, FORM>::value ? PassCDouble<T, N, NT, FORM>::kBytes
                                                         : pass_c_lds<T, N>(FORM == 1);
  const int items = (role ? b.nj : b.nk) * b.jsplit * N;
  auto kern = role ? (b.nts ? k_pass_c_ct<T, A, N, true, NT, true, FORM> : k_pass_c_ct<T, A, N, true, NT, false, FORM>)
                   : (b.nts ? k_pass_c_ct<T, A, N, false, NT, true, FORM> : k_pass_c_ct<T, A, N, false, NT, false, FORM>);
  int grid = 0;
  FX_TRY(ct_prepare(ctx, kern, NT, lds, items, true, &grid));
  if (role)
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, b.phi, b.ld_phi, (const cpx<T>*)b.work, b.nj, b.nk, b.tri,
                       b.k0, b.j0, items, c.acc, c.ld_acc, c.first, c.out, c.ld_out, c.out_c64, c.last, b.tw, (b.zsplit >> 1) & 1,
                       TrajSegs{}, b.jsplit, c.gstride);
  else
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, b.psi, b.ld_psi, (const cpx<T>*)b.work, b.nj, b.nk, b.tri,
                       b.j0, b.k0, items, c.acc, c.ld_acc, c.first, c.out, c.ld_out, c.out_c64, c.last, b.tw, (b.zsplit >> 1) & 1,
                       b.segs, b.jsplit, c.gstride);
  FX_LAUNCH_CHECK();
  return FX_OK;
}

template <typename T, typename A, int N>
static fx_status pass_c_n(fx_ctx* ctx, hipStream_t st, const CtBatch<T>& b, const CtAcc<A>& c, int role) {
  using S = CubeShape<N>;
  // the staged forms where the second plane fits the LDS (not FP64 at 72 and 96)
  constexpr bool kStg = pass_c_lds<T, N>(true) <= kLdsPerCu;
  // the wave-level form: at 72 and 96, with the larger thread count
  constexpr bool kWx = RowStage<T, N, S::NT_C2>::kWave;
  if constexpr (kWx)
    if (b.c_var == 5) return pass_c_shape<T, A, N, S::NT_C2, 2>(ctx, st, b, c, role);
  if (b.c_var == 3 && kStg) return pass_c_shape<T, A, N, S::NT_C2, kStg ? 1 : 0>(ctx, st, b, c, role);
  if (b.c_var == 4 && kStg) return pass_c_shape<T, A, N, S::NT_P, kStg ? 1 : 0>(ctx, st, b, c, role);
  if (b.c_var == 2 || b.c_var == 3 || b.c_var == 5) return pass_c_shape<T, A, N, S::NT_C2, 0>(ctx, st, b, c, role);
  return pass_c_shape<T, A, N, S::NT_P, 0>(ctx, st, b, c, role);
}

template <typename T>
fx_status ct_pass_a(fx_ctx* ctx, hipStream_t st, int n, const CtBatch<T>& b) {
  switch (n) {
    case 24: return pass_a_n<T, 24>(ctx, st, b);
    case 48: return pass_a_n<T, 48>(ctx, st, b);
    case 72: return pass_a_n<T, 72>(ctx, st, b);
    case 96: return pass_a_n<T, 96>(ctx, st, b);
    default: FX_FAIL(FX_ERR_UNSUPPORTED, "no specialised kernels for edge %d", n);
  }
}

template <typename T>
fx_status ct_pass_b(fx_ctx* ctx, hipStream_t st, int n, const CtBatch<T>& b) {
  switch (n) {
    case 24: return pass_b_n<T, 24>(ctx, st, b);
    case 48: return pass_b_n<T, 48>(ctx, st, b);
    case 72: return pass_b_n<T, 72>(ctx, st, b);
    case 96: return pass_b_n<T, 96>(ctx, st, b);
    default: FX_FAIL(FX_ERR_UNSUPPORTED, "no specialised kernels for edge %d", n);
  }
}

template <typename T, typename A>
fx_status ct_pass_c(fx_ctx* ctx, hipStream_t st, int n, const CtBatch<T>& b, const CtAcc<A>& c, int role) {
  switch (n) {
    case 24: return pass_c_n<T, A, 24>(ctx, st, b, c, role);
    case 48: return pass_c_n<T, A, 48>(ctx, st, b, c, role);
    case 72: return pass_c_n<T, A, 72>(ctx, st, b, c, role);
    case 96: return pass_c_n<T, A, 96>(ctx, st, b, c, role);
    default: FX_FAIL(FX_ERR_UNSUPPORTED, "no specialised kernels for edge %d", n);
  }
}

template fx_status ct_pass_a<float>(fx_ctx*, hipStream_t, int, const CtBatch<float>&);
template fx_status ct_pass_a<double>(fx_ctx*, hipStream_t, int, const CtBatch<double>&);
template fx_status ct_pass_b<float>(fx_ctx*, hipStream_t, int, const CtBatch<float>&);
template fx_status ct_pass_b<double>(fx_ctx*, hipStream_t, int, const CtBatch<double>&);
template fx_status ct_pass_c<float, double>(fx_ctx*, hipStream_t, int, const CtBatch<float>&, const CtAcc<double>&,
                                            int);
template fx_status ct_pass_c<float, float>(fx_ctx*, hipStream_t, int, const CtBatch<float>&, const CtAcc<float>&, int);
template fx_status ct_pass_c<double, double>(fx_ctx*, hipStream_t, int, const CtBatch<double>&, const CtAcc<double>&,
                                             int);

}  // namespace fx
