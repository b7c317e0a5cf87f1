// Compile-time-specialised FFT stages for cubic grids with a two-stage plan.
//
// Same algorithm as fft.hpp (in-place DIF forward stages, adjoint inverse
// stages, digit-reversed spectra), but the edge, the plan, the number of
// transforms, the LDS strides and the thread count are template constants:
// butterfly indices come from divisions by constants, LDS addresses fold
// into instruction offsets, each kernel carries only the two radices its
// edge needs, and the butterfly loop is fully unrolled.
#pragma once

#include "fft.hpp"

namespace fx {

// Two-stage plan of an edge; must equal make_axis_plan (checked on the host).
template <int N>
struct Plan2;
template <>
struct Plan2<24> {
  static constexpr int R0 = 6, R1 = 4;
};
template <>
struct Plan2<48> {
  static constexpr int R0 = 8, R1 = 6;
};
template <>
struct Plan2<72> {
  static constexpr int R0 = 9, R1 = 8;
};
template <>
struct Plan2<96> {
  static constexpr int R0 = 12, R1 = 8;
};

// One stage: transforms f < COUNT, element i of transform f at f*FS + i*ES;
// current sub-length L, radix R; NTHR threads deal the butterflies.
template <int R, bool FWD, typename T, int N, int L, int COUNT, int ES, int FS, int NTHR>
FX_HD void ct_stage(cpx<T>* s, const cpx<T>* tw, int tid) {
  constexpr int SPAN = L / R, TOTAL = COUNT * (N / R), TSTEP = N / L, STEP = SPAN * ES;
  constexpr int ITERS = (TOTAL + NTHR - 1) / NTHR;
#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const int b = tid + it * NTHR;
    if (TOTAL % NTHR == 0 || b < TOTAL) {
      const int f = b % COUNT;
      const int q = b / COUNT;
      const int blk = q / SPAN;
      const int i2 = q - blk * SPAN;
      const int base = f * FS + (blk * L + i2) * ES;
      cpx<T> x[R];
#pragma unroll
      for (int m = 0; m < R; ++m) x[m] = s[base + m * STEP];
      if (FWD) {
        Dft<R, -1, T>::run(x);
        if (SPAN > 1) {
#pragma unroll
          for (int k = 1; k < R; ++k) x[k] = cmul(x[k], tw[i2 * k * TSTEP]);
        }
      } else {
        if (SPAN > 1) {
#pragma unroll
          for (int k = 1; k < R; ++k) x[k] = cmulc(x[k], tw[i2 * k * TSTEP]);
        }
        Dft<R, 1, T>::run(x);
      }
#pragma unroll
      for (int m = 0; m < R; ++m) s[base + m * STEP] = x[m];
    }
  }
}

// Global accesses with a non-temporal hint: data read or written once (the
// pair volume) need not displace data that is reused from the caches (the
// orbital and target planes the workgroups of an XCD share).  At 96^3 the
// hint took the three passes from 10.5 to 9.5 ms per launch of 1170 pairs.
template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <bool NTS, typename T>
FX_HD cpx<T> g_load(const cpx<T>* p) {
  if (!NTS) return *p;
  const typename Vec2<T>::type v = __builtin_nontemporal_load(reinterpret_cast<const typename Vec2<T>::type*>(p));
  return cpx<T>{v.x, v.y};
}
template <bool NTS, typename T>
FX_HD void g_store(cpx<T>* p, cpx<T> a) {
  if (!NTS) {
    *p = a;
    return;
  }
  typename Vec2<T>::type v;
  v.x = a.x;
  v.y = a.y;
  __builtin_nontemporal_store(v, reinterpret_cast<typename Vec2<T>::type*>(p));
}

// A stage split into its three parts, so that a kernel can issue a stage's
// loads early (software pipelining): butterfly it of thread tid holds
// elements x[it][0..R) at positions pos0 + m*SPAN of transform f.  In global
// memory element i of transform f is g[f*GFS + i*GES]; in LDS it is
// s[f*FS + i*ES].
template <int R, int N, int COUNT, int NTHR>
struct StageIters {
  static constexpr int value = (COUNT * (N / R) + NTHR - 1) / NTHR;
};

template <int R, int N, int L, int COUNT, int NTHR>
struct Bfly {
  static constexpr int SPAN = L / R, TOTAL = COUNT * (N / R);
  int f, i2, pos0;
  bool ok;
  FX_HD Bfly(int tid, int it) {
    const int b = tid + it * NTHR;
    ok = TOTAL % NTHR == 0 || b < TOTAL;
    f = b % COUNT;
    const int q = b / COUNT;
    const int blk = q / SPAN;
    i2 = q - blk * SPAN;
    pos0 = blk * L + i2;
  }
};

template <int R, typename T, int N, int L, int COUNT, int NTHR, bool FROM_G, int GES, int GFS, int ES, int FS,
          bool NTS, int IT>
FX_HD void ct_bfly_load(cpx<T> (&x)[IT][R], const cpx<T>* src, int tid) {
  using B = Bfly<R, N, L, COUNT, NTHR>;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const B b(tid, it);
    if (b.ok) {
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const int pos = b.pos0 + m * B::SPAN;
        x[it][m] = FROM_G ? g_load<NTS>(src + b.f * GFS + pos * GES) : src[b.f * FS + pos * ES];
      }
    }
  }
}

template <int R, bool FWD, typename T, int N, int L, int COUNT, int NTHR, int IT>
FX_HD void ct_bfly_run(cpx<T> (&x)[IT][R], const cpx<T>* tw, int tid) {
  using B = Bfly<R, N, L, COUNT, NTHR>;
  constexpr int TSTEP = N / L;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const B b(tid, it);
    if (b.ok) {
      if (FWD) {
        Dft<R, -1, T>::run(x[it]);
        if (B::SPAN > 1) {
#pragma unroll
          for (int k = 1; k < R; ++k) x[it][k] = cmul(x[it][k], tw[b.i2 * k * TSTEP]);
        }
      } else {
        if (B::SPAN > 1) {
#pragma unroll
          for (int k = 1; k < R; ++k) x[it][k] = cmulc(x[it][k], tw[b.i2 * k * TSTEP]);
        }
        Dft<R, 1, T>::run(x[it]);
      }
    }
  }
}

template <int R, typename T, int N, int L, int COUNT, int NTHR, bool TO_G, int GES, int GFS, int ES, int FS, bool NTS,
          int IT>
FX_HD void ct_bfly_store(cpx<T> (&x)[IT][R], cpx<T>* dst, int tid) {
  using B = Bfly<R, N, L, COUNT, NTHR>;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const B b(tid, it);
    if (b.ok) {
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const int pos = b.pos0 + m * B::SPAN;
        if (TO_G)
          g_store<NTS>(dst + b.f * GFS + pos * GES, x[it][m]);
        else
          dst[b.f * FS + pos * ES] = x[it][m];
      }
    }
  }
}

// A stage that reads its inputs from global memory (FROM_G) and/or writes its
// outputs to global memory (TO_G) instead of LDS.  With consecutive threads on
// consecutive transforms f and GFS = 1, both global accesses are coalesced.
// Used for the first stage of a pass (data straight from HBM) and its last
// stage (results straight to HBM), saving an LDS round trip and a barrier at
// each end.  The loads of every butterfly of the thread are issued first, so
// they are all in flight together.
template <int R, bool FWD, typename T, int N, int L, int COUNT, int ES, int FS, int NTHR, bool FROM_G, bool TO_G,
          int GES, int GFS, bool NTS = false>
FX_HD void ct_stage_io(cpx<T>* s, const cpx<T>* gin, cpx<T>* gout, const cpx<T>* tw, int tid) {
  constexpr int IT = StageIters<R, N, COUNT, NTHR>::value;
  cpx<T> x[IT][R];
  ct_bfly_load<R, T, N, L, COUNT, NTHR, FROM_G, GES, GFS, ES, FS, NTS>(x, FROM_G ? gin : s, tid);
  ct_bfly_run<R, FWD, T, N, L, COUNT, NTHR>(x, tw, tid);
  ct_bfly_store<R, T, N, L, COUNT, NTHR, TO_G, GES, GFS, ES, FS, NTS>(x, TO_G ? gout : s, tid);
}

// ct_stage_io for a stage of span 1 (L = R) over COUNT transforms that are
// adjacent columns (transform f at offset f, GFS = FS = 1), FP32: a thread
// takes the butterflies of two adjacent transforms f, f + 1 and moves their
// global values in 16-byte accesses (the global rows must be 16-byte
// aligned, GES even).  The arithmetic is that of ct_stage_io.  kFits: one
// pair of butterflies per thread at most, so the stage is no longer than the
// unpaired one (which deals COUNT N / R butterflies over NTHR threads).
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <int R, int N, int COUNT, int NTHR>
struct PairIO {
  static constexpr int HALF = COUNT / 2, TOTAL = HALF * (N / R);
  static constexpr bool kFits = COUNT % 2 == 0 && TOTAL <= NTHR;
};
template <int R, bool FWD, typename T, int N, int COUNT, int ES, int NTHR, bool FROM_G, bool TO_G, int GES, bool NTS>
FX_HD void ct_stage_io_pair(cpx<T>* s, const cpx<T>* gin, cpx<T>* gout, int tid) {
  using P = PairIO<R, N, COUNT, NTHR>;
  static_assert(sizeof(T) == 4 && P::kFits && GES % 2 == 0, "paired stage: FP32, even count, one pair per thread");
  typedef typename Vec4<T>::type V;
  const int b = tid;
  if (P::TOTAL % NTHR != 0 && b >= P::TOTAL) return;
  const int f = 2 * (b % P::HALF), blk = b / P::HALF;
  cpx<T> x0[R], x1[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int pos = blk * R + m;
    if (FROM_G) {
      const V* p = reinterpret_cast<const V*>(gin + f + pos * GES);
      const V v = NTS ? __builtin_nontemporal_load(p) : *p;
      x0[m] = cpx<T>{v.x, v.y};
      x1[m] = cpx<T>{v.z, v.w};
    } else {
      x0[m] = s[f + pos * ES];
      x1[m] = s[f + 1 + pos * ES];
    }
  }
  Dft<R, FWD ? -1 : 1, T>::run(x0);
  Dft<R, FWD ? -1 : 1, T>::run(x1);
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int pos = blk * R + m;
    if (TO_G) {
      V v;
      v.x = x0[m].x;
      v.y = x0[m].y;
      v.z = x1[m].x;
      v.w = x1[m].y;
      V* p = reinterpret_cast<V*>(gout + f + pos * GES);
      if (NTS)
        __builtin_nontemporal_store(v, p);
      else
        *p = v;
    } else {
      s[f + pos * ES] = x0[m];
      s[f + 1 + pos * ES] = x1[m];
    }
  }
}

// Full forward or inverse transform along one axis (two stages + barriers).
template <bool FWD, typename T, int N, int COUNT, int ES, int FS, int NTHR>
__device__ inline void ct_fft(cpx<T>* s, const cpx<T>* tw, int tid) {
  constexpr int R0 = Plan2<N>::R0, R1 = Plan2<N>::R1;
  if (FWD) {
    ct_stage<R0, true, T, N, N, COUNT, ES, FS, NTHR>(s, tw, tid);
    __syncthreads();
    ct_stage<R1, true, T, N, R1, COUNT, ES, FS, NTHR>(s, tw, tid);
    __syncthreads();
  } else {
    ct_stage<R1, false, T, N, R1, COUNT, ES, FS, NTHR>(s, tw, tid);
    __syncthreads();
    ct_stage<R0, false, T, N, N, COUNT, ES, FS, NTHR>(s, tw, tid);
    __syncthreads();
  }
}

// Convolution along one axis: first forward stage, then the last forward
// stage + pointwise factor + first inverse stage in registers, then the last
// inverse stage.  kf(pos, f) as in lds_conv.
template <typename T, int N, int COUNT, int ES, int FS, int NTHR, class KF>
__device__ inline void ct_conv(cpx<T>* s, const cpx<T>* tw, KF kf, int tid) {
  constexpr int R0 = Plan2<N>::R0, R1 = Plan2<N>::R1;
  ct_stage<R0, true, T, N, N, COUNT, ES, FS, NTHR>(s, tw, tid);
  __syncthreads();
  constexpr int TOTAL = COUNT * (N / R1);
  constexpr int ITERS = (TOTAL + NTHR - 1) / NTHR;
#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const int b = tid + it * NTHR;
    if (TOTAL % NTHR == 0 || b < TOTAL) {
      const int f = b % COUNT;
      const int blk = b / COUNT;
      const int base = f * FS + blk * R1 * ES;
      cpx<T> x[R1];
#pragma unroll
      for (int m = 0; m < R1; ++m) x[m] = s[base + m * ES];
      Dft<R1, -1, T>::run(x);
#pragma unroll
      for (int k = 0; k < R1; ++k) x[k] = cscale(x[k], kf(blk * R1 + k, f));
      Dft<R1, 1, T>::run(x);
#pragma unroll
      for (int m = 0; m < R1; ++m) s[base + m * ES] = x[m];
    }
  }
  __syncthreads();
  ct_stage<R0, false, T, N, N, COUNT, ES, FS, NTHR>(s, tw, tid);
  __syncthreads();
}

// The stage over whole rows (radix R0, span N / R0) of a plane of N rows of
// N, with butterfly b on row row(b / SPAN) and offset i2 = b % SPAN: the SPAN
// lanes of a row hold the consecutive positions i2 + SPAN m of the row, so
// global data at those plane positions is read or written in runs of SPAN
// consecutive values.  inv_from_lds: the last inverse stage of the row
// transform leaves its outputs in registers, which saves an LDS round trip
// of the plane and a barrier; x[it][m] is value m of butterfly it, at plane
// position pos(tid, it, m).  inv_x_wave / fwd_x_wave: the whole row
// transform in registers and across the lanes of a wave (edges 72 and 96).
template <typename T, int N, int NT>
struct RowStage {
  static constexpr int R = Plan2<N>::R0, SPAN = N / R, TOTAL = N * SPAN;
  static constexpr int IT = (TOTAL + NT - 1) / NT;  // butterflies per thread
  // LDS rows are N + 1 values long, so row f starts at 8-byte slot f (edge
  // 96) or 9 f (edge 72) modulo the 32 slots a wave's 8-byte accesses spread
  // over.  The four rows of a 32-lane group are taken 8 apart: their starts
  // are then 8 slots apart (9 * 8 = 8 mod 32), and with the 8 offsets i2 of
  // each row the 32 lanes fall on 32 distinct slots.
  FX_HD static int row(int r) {
    if (SPAN == 8 && r < N / 32 * 32) return (r & ~31) + 8 * (r & 3) + ((r >> 2) & 7);
    return r;
  }
  FX_HD static bool owns(int tid, int it) { return TOTAL % NT == 0 || tid + it * NT < TOTAL; }
  FX_HD static int pos(int tid, int it, int m) {
    const int b = tid + it * NT;
    const int r = b / SPAN, i2 = b - r * SPAN;
    return row(r) * N + i2 + m * SPAN;
  }
  // ---- wave-level inverse row transform (both stages, edges 72 and 96) ----
  // With R1 = SPAN = 8, the 8 lanes holding one row's positions i2 + 8 m hold
  // value i2 of each radix-8 block m of the row's first inverse stage, so that
  // stage can run across those lanes instead of through LDS: each lane reads
  // its R values of the row transform's input, the radix-8 DFTs run as three
  // radix-2 steps between lanes whose DFT indices differ in one bit (the
  // partner's value arrives by a DPP move, both lanes of a pair compute their
  // own half of the butterfly), and the lane is then the butterfly i2 =
  // bitrev3(DFT index) of the radix-R stage, done in registers as in
  // inv_from_lds.  DFT index bits 0 and 1 sit on lane bits 0 and 1 and bit 2
  // on lane bit 3, so the partners are lane ^ 1 and lane ^ 2 (quad
  // permutations) and lane ^ 8 (rotation by 8 within a row of 16 lanes); lane
  // bits 2 and 4 and the wave index select the row, whose LDS reads stay on
  // distinct banks (four rows 8 apart per 32 lanes, as row() arranges).
  static constexpr bool kWave = Plan2<N>::R1 == 8 && SPAN == 8 && TOTAL == NT;
  // row and DFT index of thread tid
  FX_HD static void wave_lane(int tid, int* f, int* l) {
    *l = (tid & 3) | (((tid >> 3) & 1) << 2);
    *f = row((tid >> 5) * 4 + (((tid >> 2) & 1) | (((tid >> 4) & 1) << 1)));
  }
  FX_HD static int bitrev3(int l) { return ((l & 1) << 2) | (l & 2) | ((l >> 2) & 1); }
  // plane position of value m of thread tid after inv_x_wave
  FX_HD static int wave_pos(int tid, int m) {
    int f, l;
    wave_lane(tid, &f, &l);
    return f * N + bitrev3(l) + m * SPAN;
  }
  // the value of the lane whose DFT index is this lane's ^ H
  // (a 64-bit value moves as its two 32-bit halves)
  template <int H>
  __device__ static T partner(T v) {
    constexpr int ctrl = H == 1 ? 0xB1 : (H == 2 ? 0x4E : 0x128);  // quad_perm [1,0,3,2], [2,3,0,1]; row_ror:8
    if constexpr (sizeof(T) == 4) {
      return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, false));
    } else {
      const unsigned long long u = (unsigned long long)__double_as_longlong(v);
      const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, ctrl, 0xF, 0xF, false);
      const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), ctrl, 0xF, 0xF, false);
      return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }
  }
  // Radix-8 DFTs (sign S) across the 8 lanes of each row, one per value of
  // x, decimation in frequency: lane l holds input l of each DFT and ends with
  // output bitrev3(l).  At index distance H the lower lane of a pair keeps
  // a + b and the upper one (a - b) w^((l mod H) 4 / H), w = exp(S 2 pi i / 8).
  template <int S>
  __device__ static void lane_dft8(cpx<T> (&x)[R], int l) {
    const T c = (T)0.70710678118654752440084436210484903928;
    const bool h4 = l & 4, h2 = l & 2, h1 = l & 1;
    // twiddles of the first step: w^(l mod 4) on the upper lanes
    const int e = l & 3;
    const T wr = !h4 ? (T)1 : (e == 0 ? (T)1 : (e == 1 ? c : (e == 2 ? (T)0 : -c)));
    const T wi = !h4 ? (T)0 : (e == 0 ? (T)0 : (e == 2 ? (T)S : (T)S * c));
    const T s4 = h4 ? (T)-1 : (T)1, s2 = h2 ? (T)-1 : (T)1, s1 = h1 ? (T)-1 : (T)1;
    const bool rot = h2 && h1;  // second step: times w^2 = S i on the upper lanes of odd index
#pragma unroll
    for (int m = 0; m < R; ++m) {
      cpx<T> v = x[m];
      cpx<T> t{partner<4>(v.x) + s4 * v.x, partner<4>(v.y) + s4 * v.y};
      v = cpx<T>{t.x * wr - t.y * wi, t.x * wi + t.y * wr};
      t = cpx<T>{partner<2>(v.x) + s2 * v.x, partner<2>(v.y) + s2 * v.y};
      v = rot ? (S > 0 ? cpx<T>{-t.y, t.x} : cpx<T>{t.y, -t.x}) : t;
      x[m] = cpx<T>{partner<1>(v.x) + s1 * v.x, partner<1>(v.y) + s1 * v.y};
    }
  }
  // inverse row transform: LDS rows of stride SX -> x at wave_pos(tid, m)
  template <int SX>
  __device__ static void inv_x_wave(const cpx<T>* s, const cpx<T>* tw, int tid, cpx<T> (&x)[R]) {
    static_assert(kWave, "wave-level row transform needs R1 = N / R0 = 8 and one butterfly per thread");
    int f, l;
    wave_lane(tid, &f, &l);
#pragma unroll
    for (int m = 0; m < R; ++m) x[m] = s[f * SX + l + m * SPAN];
    lane_dft8<1>(x, l);
    const int i2 = bitrev3(l);
#pragma unroll
    for (int k = 1; k < R; ++k) x[k] = cmulc(x[k], tw[i2 * k]);
    Dft<R, 1, T>::run(x);
  }
  // forward row transform: x, the row's values at fwd_pos(tid, m), -> LDS rows
  // of stride SX (the same digit-reversed order as the two LDS stages)
  FX_HD static int fwd_pos(int tid, int m) {
    int f, l;
    wave_lane(tid, &f, &l);
    return f * N + l + m * SPAN;
  }
  template <int SX>
  __device__ static void fwd_x_wave(cpx<T> (&x)[R], cpx<T>* s, const cpx<T>* tw, int tid) {
    static_assert(kWave, "wave-level row transform needs R1 = N / R0 = 8 and one butterfly per thread");
    int f, l;
    wave_lane(tid, &f, &l);
    Dft<R, -1, T>::run(x);
#pragma unroll
    for (int k = 1; k < R; ++k) x[k] = cmul(x[k], tw[l * k]);
    lane_dft8<-1>(x, l);
    const int j = bitrev3(l);
#pragma unroll
    for (int m = 0; m < R; ++m) s[f * SX + 8 * m + j] = x[m];
  }
  // inverse stage (twiddles, then butterfly) from LDS rows of stride SX into x
  template <int SX>
  __device__ static void inv_from_lds(const cpx<T>* s, const cpx<T>* tw, int tid, cpx<T> (&x)[IT][R]) {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      if (!owns(tid, it)) continue;
      const int b = tid + it * NT;
      const int r = b / SPAN, i2 = b - r * SPAN, f = row(r);
#pragma unroll
      for (int m = 0; m < R; ++m) x[it][m] = s[f * SX + i2 + m * SPAN];
      if (SPAN > 1) {
#pragma unroll
        for (int k = 1; k < R; ++k) x[it][k] = cmulc(x[it][k], tw[i2 * k]);
      }
      Dft<R, 1, T>::run(x[it]);
    }
  }
};

// Launch shapes per edge: plane passes (threads), pencil pass (x tile,
// threads), second and third pencil-pass shapes (half the x tile; whole x
// rows, the longest contiguous runs in HBM), a second thread
// count for the plane-inverse pass (fewer accumulators per thread, more waves
// per CU) and one for the plane-forward pass (butterfly counts that divide
// evenly among the threads); threads of the persistent pencil pass with whole
// x rows.
template <int N>
struct CubeShape;
template <>
struct CubeShape<24> {
  static constexpr int NT_P = 192, XT = 24, NT_B = 192, XT2 = 12, NT_B2 = 96, NT_C2 = 288, NT_A2 = 288, XT3 = 24, NT_B3 = 192, NT_BP = 192;
};
template <>
struct CubeShape<48> {
  static constexpr int NT_P = 256, XT = 48, NT_B = 256, XT2 = 24, NT_B2 = 128, NT_C2 = 384, NT_A2 = 384, XT3 = 48, NT_B3 = 256, NT_BP = 384;
};
template <>
struct CubeShape<72> {
  static constexpr int NT_P = 512, XT = 24, NT_B = 256, XT2 = 12, NT_B2 = 128, NT_C2 = 576, NT_A2 = 576, XT3 = 72, NT_B3 = 512, NT_BP = 576;
};
template <>
struct CubeShape<96> {
  static constexpr int NT_P = 512, XT = 48, NT_B = 512, XT2 = 24, NT_B2 = 256, NT_C2 = 768, NT_A2 = 768, XT3 = 96, NT_B3 = 1024, NT_BP = 768;
};

}  // namespace fx
