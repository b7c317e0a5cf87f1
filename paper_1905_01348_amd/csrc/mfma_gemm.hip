// K_ACE phi = -xi (xi^H phi) on the matrix cores.
//
// Both projections are written as real GEMMs whose two operands are
// contiguous along the reduction dimension ("TN"), on the interleaved
// (re, im) real view of the complex arrays:
//
//   C = xi^H phi  : D (N x 2R) = A B^T, A row m = column m of xi (2 N_r reals),
//                   B row 2n = phi_n, B row 2n+1 = (-i phi_n) = (im, -re) pairs;
//                   Re C(m,n) = D(m, 2n), Im C(m,n) = D(m, 2n+1).  The reduction
//                   (2 N_r long) is split across workgroups; split partial sums
//                   are added in FP64 in a fixed order.
//   y = -xi C     : D (N_r x 2R) = A B^T, A row r = row r of xi (2 N reals),
//                   B row 2n = (Re C, -Im C) pairs, B row 2n+1 = (Im C, Re C);
//                   y(r,n) = -(D(r,2n), D(r,2n+1)).
//
// Precision forms: every operand X is split as X_p = round(X) and
// r_X = round(X - X_p) (FP32, BF16 or FP16), and with the residual step the
// GEMM computes A_p B_p (main accumulator) and A_p r_B + r_A B_p (correction
// accumulator), both in FP32 on the matrix cores, added in FP64 at the end.
// FP16 operands are scaled by powers of two first (xi by one factor, each
// right-hand side and each column of C by its own) so that the largest
// magnitude lands in [2^13, 2^14): the 11-bit significand then holds the
// values and their residuals without overflow or loss to subnormals, and the
// exact power-of-two factors are divided out in FP64 afterwards.
#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "fft.hpp"
#include "mfma_gemm.hpp"
#include "vx.hpp"

namespace fx {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

// ---- rounding ---------------------------------------------------------------
// float -> bfloat16, round to nearest even (NaN kept quiet)
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename S>
struct Prec;
template <>
struct Prec<float> {
  static constexpr int BK = 32;   // K elements per tile step (128 bytes per row)
  static constexpr int PAD = 4;   // LDS row padding (elements)
  __device__ static float round(double x) { return (float)x; }
  __device__ static double widen(float s) { return (double)s; }
  __device__ static float round_f(float x) { return x; }
  __device__ static float widen_f(float s) { return s; }
};
template <>
struct Prec<uint16_t> {
  static constexpr int BK = 64;
  static constexpr int PAD = 8;
  __device__ static uint16_t round(double x) { return f2bf((float)x); }
  __device__ static double widen(uint16_t s) { return (double)bf2f(s); }
  __device__ static uint16_t round_f(float x) { return f2bf(x); }
  __device__ static float widen_f(uint16_t s) { return bf2f(s); }
};

template <>
struct Prec<_Float16> {
  static constexpr int BK = 64;
  static constexpr int PAD = 8;
  __device__ static _Float16 round(double x) { return (_Float16)x; }
  __device__ static double widen(_Float16 s) { return (double)s; }
  __device__ static _Float16 round_f(float x) { return (_Float16)x; }
  __device__ static float widen_f(_Float16 s) { return (float)s; }
};

// Power-of-two factor that takes a largest magnitude m (as FP32 bits; m >= 0)
// into [2^13, 2^14); 1 for the FP32 and BF16 forms (no maxima) and for m = 0.
__device__ inline double scale_of(const unsigned* maxbits, int i) {
  if (!maxbits) return 1.0;
  const float m = __uint_as_float(maxbits[i]);
  if (!(m > 0.f) || !isfinite(m)) return 1.0;
  int e = 0;
  (void)frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
  return ldexp(1.0, 14 - e);
}

// Largest |x| of each column (per_col) or of all columns, as FP32 bits
// (monotone for non-negative floats, so an integer max merges blocks);
// `out` must hold zeros first.  x: real view, column c at x + c * ld.
template <typename T>
__global__ void k_absmax(const T* __restrict__ x, int64_t ld, int64_t len, int per_col, unsigned* __restrict__ out) {
  __shared__ float red[256];
  const int c = blockIdx.y;
  const T* col = x + (int64_t)c * ld;
  float m = 0.f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, (float)fabs((double)col[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out + (per_col ? c : 0), __float_as_uint(red[0]));
}

__global__ void k_zero_u32(unsigned* __restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

constexpr int KPAD = 64;  // reduction dims of split arrays are padded to this
static int64_t roundk(int64_t k) { return (k + KPAD - 1) / KPAD * KPAD; }

// (a, b) pairs -> (b, -a) on a 16-byte vector: multiplication by -i of the
// complex values it holds.
__device__ inline uint4 times_minus_i(uint4 v, int elem_bytes) {
  if (elem_bytes == 4) {
    return uint4{v.y, v.x ^ 0x80000000u, v.w, v.z ^ 0x80000000u};
  }
  // bf16: 4 pairs, each 32-bit word holds (lo = a, hi = b)
  uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t a = w[i] & 0xffffu, b = w[i] >> 16;
    w[i] = b | ((a ^ 0x8000u) << 16);
  }
  return uint4{w[0], w[1], w[2], w[3]};
}

// ---------------------------------------------------------------------------
// TN GEMM on matrix cores.  256 threads = 4 waves in a 2x2 arrangement, each
// wave a 64x64 block of D made of 2x2 MFMA 32x32 tiles.  Workgroup tile
// 128 x 128, K step BK.
//   A: rows m (M of them), A[m*lda + k];  B: rows n (N of them), B[n*ldb + k].
//   BDOUBLE: B holds N/2 source rows; LDS row 2c is source row c and row
//            2c+1 is source row c times -i (see header comment).
//   MODE 0: write FP64 partial sums, partial[(split*M + m)*N + n].
//   MODE 1: write y(r=m, n/2) component n&1 = -alpha * D to a complex output.
// ---------------------------------------------------------------------------
constexpr int TBM = 128, TBN = 128;

// Order of a wave's own LDS accesses across lanes: the wave's LDS
// instructions execute in issue order, so only the compiler has to be kept
// from moving accesses across this point.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Held to two waves per SIMD (accumulators in the unified register file), so
// that two workgroups share a CU and one's barriers and loads overlap the
// other's matrix work: at 96^3, N = R = 1024 this took the BF16+residual
// GEMMs from 20% to 37% of the BF16 peak and the FP32+residual ones from
// 67-68% to 73-82% of the FP32 peak (the output GEMM spills a few registers).
template <typename S>
struct MfmaWaves {
  static constexpr int value = 2;
};

// Epilogue of the TN GEMM kernels: D tile element e of MFMA tile (i, j) of a
// wave is row i*32 + 8*(e/4) + 4*(lane/32) + e%4, column j*32 + lane%32 of the
// wave's 64x64 block.  MODE 0 writes FP64 partial sums; MODE 1 turns each
// 32x32 tile around in the wave's own 32 x 33 doubles of `smem_raw` (the
// caller's LDS, idle by then) and writes y = -alpha * D along r.
template <bool REFINE, int MODE>
__device__ inline void tn_epilogue(floatx16 (&acc)[2][2], floatx16 (&cor)[2][2], unsigned char* smem_raw, int lane,
                                   int wave, int wm, int wn, int m0, int n0, int M, int N, int split,
                                   double* __restrict__ partial, void* __restrict__ out, int64_t ldo, int out_c64,
                                   double alpha, const double* __restrict__ colalpha) {
  if (MODE == 0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = n0 + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int m = m0 + wm * 64 + i * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
          if (m >= M || n >= N) continue;
          partial[((int64_t)split * M + m) * N + n] = (double)acc[i][j][e] + (REFINE ? (double)cor[i][j][e] : 0.0);
        }
      }
    return;
  }
  // MODE 1: the output runs along m (r) for each target, the tile along n:
  // each wave turns its 32x32 tiles around in its own slice of the (now idle)
  // LDS, then writes 32 consecutive r of one target per half-wave.
  constexpr int SL = 33;  // padded row of the staged tile (doubles)
  double* stg = reinterpret_cast<double*>(smem_raw) + wave * 32 * SL;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int ml = 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        stg[ml * SL + (lane & 31)] = (double)acc[i][j][e] + (REFINE ? (double)cor[i][j][e] : 0.0);
      }
      wave_lds_sync();
      const int ml = lane & 31;
      const int m = m0 + wm * 64 + i * 32 + ml;
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int tl = (lane >> 5) + 2 * it;  // target within the tile's 16
        const int n = n0 + wn * 64 + j * 32 + 2 * tl;
        const double re = stg[ml * SL + 2 * tl], im = stg[ml * SL + 2 * tl + 1];
        if (m < M && n < N) {
          const int64_t idx = (int64_t)(n >> 1) * ldo + m;
          const double al = colalpha ? colalpha[n >> 1] : alpha;
          if (out_c64)
            reinterpret_cast<float2*>(out)[idx] = make_float2((float)(-al * re), (float)(-al * im));
          else
            reinterpret_cast<double2*>(out)[idx] = make_double2(-al * re, -al * im);
        }
      }
      wave_lds_sync();
    }
}

template <typename S, bool REFINE, bool BDOUBLE, int MODE>
__global__ void __launch_bounds__(256, (MfmaWaves<S>::value)) k_tn_mfma(int M, int N, int K, int kchunk, const S* __restrict__ Ap,
                                                 const S* __restrict__ Ar, int64_t lda, const S* __restrict__ Bp,
                                                 const S* __restrict__ Br, int64_t ldb, double* __restrict__ partial,
                                                 void* __restrict__ out, int64_t ldo, int out_c64, double alpha,
                                                 const double* __restrict__ colalpha, int tiles_m, int tiles_n) {
  constexpr int BK = Prec<S>::BK;
  constexpr int LDK = BK + Prec<S>::PAD;
  constexpr int EPV = 16 / sizeof(S);  // elements per 16-byte vector
  constexpr int VPR = BK / EPV;        // vectors per tile row (8)
  constexpr int NT = REFINE ? 4 : 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  S* sm = reinterpret_cast<S*>(smem_raw);
  S* sAp = sm;
  S* sBp = sm + TBM * LDK;
  S* sAr = sm + 2 * TBM * LDK;
  S* sBr = sm + 3 * TBM * LDK;

  // block -> (tile_m, tile_n, split); consecutive blocks on one XCD share
  // the A row-tile: the hardware deals blocks to the 8 XCDs round-robin.
  const int nblk = gridDim.x;
  const int bid = blockIdx.x;
  const int per_xcd = (nblk + 7) / 8;
  int lid = (bid % 8) * per_xcd + bid / 8;
  if (nblk % 8 != 0) lid = bid;  // keep the mapping a bijection
  const int tn = lid % tiles_n;
  const int rest = lid / tiles_n;
  const int tm = rest % tiles_m;
  const int split = rest / tiles_m;
  const int m0 = tm * TBM, n0 = tn * TBN;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  floatx16 acc[2][2], cor[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        acc[i][j][e] = 0.f;
        cor[i][j][e] = 0.f;
      }
    }

  // register staging of one K step: 4 vectors per thread per A tile; B tile
  // rows: 128 (plain) or 64 source rows (BDOUBLE, 2 vectors per thread)
  constexpr int BV = BDOUBLE ? 2 : 4;
  uint4 ra[2][4], rb[2][BV];
  // rows past the edge load a clamped (valid) row and are zeroed by value,
  // so the loads need no branches
  auto zsel = [](uint4 v, bool keep) __attribute__((always_inline)) {
    return uint4{keep ? v.x : 0u, keep ? v.y : 0u, keep ? v.z : 0u, keep ? v.w : 0u};
  };
  auto gload = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int v = tid + 256 * u, row = v / VPR, c = v % VPR;
      const int m = m0 + row;
      const int mc = m < M ? m : M - 1;
      const int64_t off = (int64_t)mc * lda + k0 + c * EPV;
      ra[0][u] = zsel(*reinterpret_cast<const uint4*>(Ap + off), m < M);
      if (REFINE) ra[1][u] = zsel(*reinterpret_cast<const uint4*>(Ar + off), m < M);
    }
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      const int v = tid + 256 * u, row = v / VPR, c = v % VPR;
      const int n = BDOUBLE ? n0 / 2 + row : n0 + row;
      const int nlim = BDOUBLE ? N / 2 : N;
      const int nc = n < nlim ? n : nlim - 1;
      const int64_t off = (int64_t)nc * ldb + k0 + c * EPV;
      rb[0][u] = zsel(*reinterpret_cast<const uint4*>(Bp + off), n < nlim);
      if (REFINE) rb[1][u] = zsel(*reinterpret_cast<const uint4*>(Br + off), n < nlim);
    }
  };
  auto sstore = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int v = tid + 256 * u, row = v / VPR, c = v % VPR;
      *reinterpret_cast<uint4*>(sAp + row * LDK + c * EPV) = ra[0][u];
      if (REFINE) *reinterpret_cast<uint4*>(sAr + row * LDK + c * EPV) = ra[1][u];
    }
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      const int v = tid + 256 * u, row = v / VPR, c = v % VPR;
      if (BDOUBLE) {
        *reinterpret_cast<uint4*>(sBp + (2 * row) * LDK + c * EPV) = rb[0][u];
        *reinterpret_cast<uint4*>(sBp + (2 * row + 1) * LDK + c * EPV) = times_minus_i(rb[0][u], sizeof(S));
        if (REFINE) {
          *reinterpret_cast<uint4*>(sBr + (2 * row) * LDK + c * EPV) = rb[1][u];
          *reinterpret_cast<uint4*>(sBr + (2 * row + 1) * LDK + c * EPV) = times_minus_i(rb[1][u], sizeof(S));
        }
      } else {
        *reinterpret_cast<uint4*>(sBp + row * LDK + c * EPV) = rb[0][u];
        if (REFINE) *reinterpret_cast<uint4*>(sBr + row * LDK + c * EPV) = rb[1][u];
      }
    }
  };

  if (kbeg < kend) gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    sstore();
    __syncthreads();
    if (k0 + BK < kend) gload(k0 + BK);
    const int ar = wm * 64 + (lane & 31);
    const int br = wn * 64 + (lane & 31);
    if constexpr (sizeof(S) == 4) {
      // MFMA u of group q takes k = 4q + u (lanes 0-31) and BK/2 + 4q + u
      // (lanes 32-63): any order of the step's k terms gives the same sum up
      // to rounding, and this one lets each lane fetch the operands of four
      // MFMAs with one 16-byte LDS read (rows 36 floats apart fill the 32
      // banks in each group of 8 lanes; 4-byte reads of 32 rows did not)
#pragma unroll
      for (int q = 0; q < BK / 8; ++q) {
        const int kc = (lane >> 5) * (BK / 2) + 4 * q;
        float4 a[2], b[2], a2[2], b2[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          a[t] = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(sAp) + (ar + 32 * t) * LDK + kc);
          b[t] = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(sBp) + (br + 32 * t) * LDK + kc);
          if (REFINE) {
            a2[t] = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(sAr) + (ar + 32 * t) * LDK + kc);
            b2[t] = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(sBr) + (br + 32 * t) * LDK + kc);
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][u], b[j][u], acc[i][j], 0, 0, 0);
              if (REFINE) {
                cor[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][u], b2[j][u], cor[i][j], 0, 0, 0);
                cor[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a2[i][u], b[j][u], cor[i][j], 0, 0, 0);
              }
            }
      }
    } else if constexpr (std::is_same<S, _Float16>::value) {
#pragma unroll
      for (int kk = 0; kk < BK / 16; ++kk) {
        const int kc = kk * 16 + (lane >> 5) * 8;
        halfx8 a[2], b[2], a2[2], b2[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          a[t] = __builtin_bit_cast(halfx8, *reinterpret_cast<const uint4*>(sAp + (ar + 32 * t) * LDK + kc));
          b[t] = __builtin_bit_cast(halfx8, *reinterpret_cast<const uint4*>(sBp + (br + 32 * t) * LDK + kc));
          if (REFINE) {
            a2[t] = __builtin_bit_cast(halfx8, *reinterpret_cast<const uint4*>(sAr + (ar + 32 * t) * LDK + kc));
            b2[t] = __builtin_bit_cast(halfx8, *reinterpret_cast<const uint4*>(sBr + (br + 32 * t) * LDK + kc));
          }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[i], b[j], acc[i][j], 0, 0, 0);
            if (REFINE) {
              cor[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[i], b2[j], cor[i][j], 0, 0, 0);
              cor[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a2[i], b[j], cor[i][j], 0, 0, 0);
            }
          }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK / 16; ++kk) {
        const int kc = kk * 16 + (lane >> 5) * 8;
        bf16x8 a[2], b[2], a2[2], b2[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          a[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(sAp + (ar + 32 * t) * LDK + kc));
          b[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(sBp + (br + 32 * t) * LDK + kc));
          if (REFINE) {
            a2[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(sAr + (ar + 32 * t) * LDK + kc));
            b2[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(sBr + (br + 32 * t) * LDK + kc));
          }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            if (REFINE) {
              cor[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b2[j], cor[i][j], 0, 0, 0);
              cor[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2[i], b[j], cor[i][j], 0, 0, 0);
            }
          }
      }
    }
    __syncthreads();
  }

  tn_epilogue<REFINE, MODE>(acc, cor, smem_raw, lane, wave, wm, wn, m0, n0, M, N, split, partial, out, ldo, out_c64,
                            alpha, colalpha);
}

// ---------------------------------------------------------------------------
// The same TN GEMM for the 2-byte operand types (BF16, FP16) with the operand
// tiles loaded straight into LDS: 16-byte global_load_lds (no staging
// registers, no LDS store instructions), two LDS buffers so that the next K
// step's loads run while the current one is multiplied, one barrier per K
// step.  K steps of DL_BK = 32 elements: a tile row is 64 bytes (4 chunks of
// 8 elements), stored without padding; row r keeps global chunk g in slot
// g ^ ((r >> 2) & 3), so that the 16-byte operand reads of 16 consecutive
// rows (one pass of the LDS) fall on distinct banks.  With BDOUBLE only the
// N/2 source rows are stored; an odd B row is its source row times -i, made
// when the operand is read.  Same results as k_tn_mfma up to the order of
// the k terms within a step.
constexpr int DL_BK = 32;

__device__ inline int dl_swz(int row) { return (row >> 2) & 3; }

__device__ inline void dl_load16(const void* g, unsigned char* lds_wave_base) {
  __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds_wave_base, 16, 0, 0);
}

template <typename S, bool BDOUBLE>
struct DlShape {
  static constexpr int ROWB = DL_BK * (int)sizeof(S);  // 64 bytes
  static constexpr int AB = TBM * ROWB;                // one A operand tile
  static constexpr int BROWS = BDOUBLE ? TBN / 2 : TBN;
  static constexpr int BB = BROWS * ROWB;              // one B operand tile
};
template <typename S, bool REFINE, bool BDOUBLE>
constexpr size_t dl_stage_bytes() {
  return (size_t)(REFINE ? 2 : 1) * (DlShape<S, BDOUBLE>::AB + DlShape<S, BDOUBLE>::BB);
}

template <typename S, bool REFINE, bool BDOUBLE, int MODE>
__global__ void __launch_bounds__(256, 2) k_tn_mfma_dl(int M, int N, int K, int kchunk, const S* __restrict__ Ap,
                                                      const S* __restrict__ Ar, int64_t lda, const S* __restrict__ Bp,
                                                      const S* __restrict__ Br, int64_t ldb, double* __restrict__ partial,
                                                      void* __restrict__ out, int64_t ldo, int out_c64, double alpha,
                                                      const double* __restrict__ colalpha, int tiles_m, int tiles_n) {
  static_assert(sizeof(S) == 2, "2-byte operands");
  using D = DlShape<S, BDOUBLE>;
  constexpr int NOPS = REFINE ? 2 : 1;
  constexpr int STAGE = (int)dl_stage_bytes<S, REFINE, BDOUBLE>();
  extern __shared__ __align__(16) unsigned char smem_raw[];

  const int nblk = gridDim.x;
  const int bid = blockIdx.x;
  const int per_xcd = (nblk + 7) / 8;
  int lid = (bid % 8) * per_xcd + bid / 8;
  if (nblk % 8 != 0) lid = bid;
  const int tn = lid % tiles_n;
  const int rest = lid / tiles_n;
  const int tm = rest % tiles_m;
  const int split = rest / tiles_m;
  const int m0 = tm * TBM, n0 = tn * TBN;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  floatx16 acc[2][2], cor[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        acc[i][j][e] = 0.f;
        cor[i][j][e] = 0.f;
      }

  // loads of the K step at k0 into buffer b: each wave-instruction fills 1 KB
  // (16 rows); lane l lands in row l / 4, slot l % 4 of it.  Rows past the
  // edge load a clamped, valid row: they only reach outputs that are not
  // written.
  const int lrow = lane >> 2, lslot = lane & 3;
  auto issue = [&](int k0, int b) __attribute__((always_inline)) {
    unsigned char* base = smem_raw + b * STAGE;
#pragma unroll
    for (int q = 0; q < TBM / 64; ++q) {
      const int ch = wave + 4 * q, row = ch * 16 + lrow;
      const int m = min(m0 + row, M - 1);
      const int64_t off = (int64_t)m * lda + k0 + (lslot ^ dl_swz(row)) * 8;
      dl_load16(Ap + off, base + ch * 1024);
      if (REFINE) dl_load16(Ar + off, base + D::AB + ch * 1024);
    }
    const int nlim = BDOUBLE ? N / 2 : N;
    const int nb = BDOUBLE ? n0 / 2 : n0;
#pragma unroll
    for (int q = 0; q < D::BROWS / 64; ++q) {
      const int ch = wave + 4 * q, row = ch * 16 + lrow;
      const int nn = min(nb + row, nlim - 1);
      const int64_t off = (int64_t)nn * ldb + k0 + (lslot ^ dl_swz(row)) * 8;
      dl_load16(Bp + off, base + NOPS * D::AB + ch * 1024);
      if (REFINE) dl_load16(Br + off, base + NOPS * D::AB + D::BB + ch * 1024);
    }
  };
  auto frag = [&](const unsigned char* t, int row, int g) __attribute__((always_inline)) {
    return *reinterpret_cast<const uint4*>(t + row * D::ROWB + ((g ^ dl_swz(row)) << 4));
  };
  auto bfrag = [&](const unsigned char* t, int br, int g) __attribute__((always_inline)) {
    if (!BDOUBLE) return frag(t, br, g);
    const uint4 v = frag(t, br >> 1, g);
    const uint4 w = times_minus_i(v, 2);
    const bool odd = br & 1;
    return uint4{odd ? w.x : v.x, odd ? w.y : v.y, odd ? w.z : v.z, odd ? w.w : v.w};
  };

  const int nsteps = (kend - kbeg) / DL_BK;
  if (nsteps > 0) issue(kbeg, 0);
  for (int st = 0; st < nsteps; ++st) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of step st have landed
    __syncthreads();                // ... every wave's; and step st - 1's reads are done
    const unsigned char* base = smem_raw + (st & 1) * STAGE;
    const unsigned char* tAp = base;
    const unsigned char* tAr = base + D::AB;
    const unsigned char* tBp = base + NOPS * D::AB;
    const unsigned char* tBr = tBp + D::BB;
    // every operand of the step is read before the next step's loads are
    // issued: a read of LDS after those loads would wait for them
    uint4 a[2][2], b[2][2], a2[2][2], b2[2][2];  // [kk][t]
#pragma unroll
    for (int kk = 0; kk < DL_BK / 16; ++kk) {
      const int g = kk * 2 + (lane >> 5);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int ar = wm * 64 + (lane & 31) + 32 * t;
        const int br = wn * 64 + (lane & 31) + 32 * t;
        a[kk][t] = frag(tAp, ar, g);
        b[kk][t] = bfrag(tBp, br, g);
        if (REFINE) {
          a2[kk][t] = frag(tAr, ar, g);
          b2[kk][t] = bfrag(tBr, br, g);
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (st + 1 < nsteps) issue(kbeg + (st + 1) * DL_BK, (st + 1) & 1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < DL_BK / 16; ++kk)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if constexpr (std::is_same<S, _Float16>::value) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                __builtin_bit_cast(halfx8, a[kk][i]), __builtin_bit_cast(halfx8, b[kk][j]), acc[i][j], 0, 0, 0);
            if (REFINE) {
              cor[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                  __builtin_bit_cast(halfx8, a[kk][i]), __builtin_bit_cast(halfx8, b2[kk][j]), cor[i][j], 0, 0, 0);
              cor[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                  __builtin_bit_cast(halfx8, a2[kk][i]), __builtin_bit_cast(halfx8, b[kk][j]), cor[i][j], 0, 0, 0);
            }
          } else {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, a[kk][i]), __builtin_bit_cast(bf16x8, b[kk][j]), acc[i][j], 0, 0, 0);
            if (REFINE) {
              cor[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  __builtin_bit_cast(bf16x8, a[kk][i]), __builtin_bit_cast(bf16x8, b2[kk][j]), cor[i][j], 0, 0, 0);
              cor[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  __builtin_bit_cast(bf16x8, a2[kk][i]), __builtin_bit_cast(bf16x8, b[kk][j]), cor[i][j], 0, 0, 0);
            }
          }
        }
  }
  __syncthreads();  // the epilogue reuses the LDS
  tn_epilogue<REFINE, MODE>(acc, cor, smem_raw, lane, wave, wm, wn, m0, n0, M, N, split, partial, out, ldo, out_c64,
                            alpha, colalpha);
}

// ---- split kernels ----------------------------------------------------------
// xi (complex double, N_r x N, ld N_r) -> col form: row m = interleaved column m.
template <typename S>
__global__ void k_split_col(const double* __restrict__ xi, int64_t nr, int n, int64_t kc, S* __restrict__ p,
                            S* __restrict__ r, const unsigned* __restrict__ smax) {
  const int64_t total = (int64_t)n * kc;
  const double sc = scale_of(smax, 0);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = i / kc, k = i - m * kc;
    const double v = k < 2 * nr ? sc * xi[m * 2 * nr + k] : 0.0;
    const S hp = Prec<S>::round(v);
    p[i] = hp;
    r[i] = Prec<S>::round(v - Prec<S>::widen(hp));
  }
}

// xi -> row form: row r = interleaved row r of xi (N complex values), padded
// to kn.  64 grid points x 32 orbitals per block through LDS.
template <typename S>
__global__ void __launch_bounds__(256) k_split_row(const double* __restrict__ xi, int64_t nr, int n, int64_t kn,
                                                   S* __restrict__ p, S* __restrict__ r,
                                                   const unsigned* __restrict__ smax) {
  __shared__ double2 t[32][65];
  const double sc = scale_of(smax, 0);
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int m0 = blockIdx.y * 32;
  for (int e = threadIdx.x; e < 32 * 64; e += 256) {
    const int mi = e / 64, ri = e % 64;
    const int64_t rr = r0 + ri;
    const int m = m0 + mi;
    double2 v = {0.0, 0.0};
    if (m < n && rr < nr) v = reinterpret_cast<const double2*>(xi)[(int64_t)m * nr + rr];
    t[mi][ri] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int ri = e / 64, kk = e % 64;  // kk: position in the 64-wide k window
    const int64_t rr = r0 + ri;
    if (rr >= nr) continue;
    const double2 v = t[kk >> 1][ri];
    const double x = sc * ((kk & 1) ? v.y : v.x);
    const int64_t idx = rr * kn + 2 * (int64_t)m0 + kk;
    const S hp = Prec<S>::round(x);
    p[idx] = hp;
    r[idx] = Prec<S>::round(x - Prec<S>::widen(hp));
  }
}

// phi (complex, ld) -> B source rows: row n = interleaved phi_n, padded to kc.
template <typename S, typename TI>
__global__ void k_split_phi(const TI* __restrict__ phi, int64_t ld, int64_t nr, int R, int64_t kc,
                            S* __restrict__ p, S* __restrict__ r, const unsigned* __restrict__ smax) {
  const int64_t total = (int64_t)R * kc;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = i / kc, k = i - n * kc;
    const double sc = scale_of(smax, (int)n);
    if constexpr (std::is_same<TI, float>::value) {
      // FP32 input: the scaled value and its residual are exact in FP32
      // (a power-of-two factor that stays finite; X - round(X) of an FP32 X),
      // so the split is the same as in FP64, at FP32 speed
      if (sc < 0x1p100) {
        const float v = k < 2 * nr ? (float)sc * phi[n * 2 * ld + k] : 0.f;
        const S hp = Prec<S>::round_f(v);
        p[i] = hp;
        r[i] = Prec<S>::round_f(v - Prec<S>::widen_f(hp));
        continue;
      }
    }
    const double v = k < 2 * nr ? sc * (double)phi[n * 2 * ld + k] : 0.0;
    const S hp = Prec<S>::round(v);
    p[i] = hp;
    r[i] = Prec<S>::round(v - Prec<S>::widen(hp));
  }
}

// Fixed-order FP64 sum of the C = xi^H phi split partials, written as the B
// operand of y = -xi C: row 2n = (Re C(k,n), -Im C(k,n)) pairs, row 2n+1 =
// (Im C(k,n), Re C(k,n)) pairs, padded to kn; split p / r.
template <typename S>
__global__ void k_reduce_cn(const double* __restrict__ partial, int nsplit, int n, int R, int64_t kn,
                            S* __restrict__ p, S* __restrict__ r) {
  const int64_t M = n, NN = 2 * (int64_t)R;
  const int64_t total = (int64_t)R * (kn / 2);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    // neighbouring threads take neighbouring right-hand sides: their partial
    // sums are adjacent in memory (the reads are the bulk of the traffic)
    const int64_t k = i / R, nc = i - k * R;
    double cr = 0.0, ci = 0.0;
    if (k < n) {
      for (int s = 0; s < nsplit; ++s) {
        cr += partial[((int64_t)s * M + k) * NN + 2 * nc];
        ci += partial[((int64_t)s * M + k) * NN + 2 * nc + 1];
      }
    }
    const double v[4] = {cr, -ci, ci, cr};
    const int64_t base0 = (2 * nc) * kn + 2 * k, base1 = (2 * nc + 1) * kn + 2 * k;
    const int64_t idx[4] = {base0, base0 + 1, base1, base1 + 1};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const S hp = Prec<S>::round(v[q]);
      p[idx[q]] = hp;
      r[idx[q]] = Prec<S>::round(v[q] - Prec<S>::widen(hp));
    }
  }
}

// The same for scaled FP16 operands, in two passes.  First
// C(k, nc) = (fixed-order FP64 sum of the partials) / (s_xi s_nc), exact
// since the factors are powers of two, into an FP64 buffer, with each
// right-hand side's largest magnitude merged into cmax[nc] (zeroed first).
// Then the split of t_nc C with t_nc the power of two of cmax[nc], and
// colalpha[nc] = 1 / (s_xi t_nc) for the epilogue of y = -xi C.
__global__ void k_sum_cn_scaled(const double* __restrict__ partial, int nsplit, int n, int R,
                                const unsigned* __restrict__ xmax, const unsigned* __restrict__ pmax,
                                double2* __restrict__ c64, unsigned* __restrict__ cmax) {
  const int64_t M = n, NN = 2 * (int64_t)R;
  const double sx = scale_of(xmax, 0);
  const int64_t total = (int64_t)n * R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = i / R, nc = i - k * R;
    double cr = 0.0, ci = 0.0;
    for (int s = 0; s < nsplit; ++s) {
      cr += partial[((int64_t)s * M + k) * NN + 2 * nc];
      ci += partial[((int64_t)s * M + k) * NN + 2 * nc + 1];
    }
    const double f = 1.0 / (sx * scale_of(pmax, (int)nc));
    c64[i] = double2{cr * f, ci * f};
    atomicMax(cmax + nc, __float_as_uint((float)fmax(fabs(cr * f), fabs(ci * f))));
  }
}

template <typename S>
__global__ void k_split_cn_scaled(const double2* __restrict__ c64, int n, int R, int64_t kn,
                                  const unsigned* __restrict__ xmax, const unsigned* __restrict__ cmax,
                                  S* __restrict__ p, S* __restrict__ r, double* __restrict__ colalpha) {
  const double sx = scale_of(xmax, 0);
  const int64_t total = (int64_t)R * (kn / 2);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t nc = i / (kn / 2), k = i - nc * (kn / 2);
    const double t = scale_of(cmax, (int)nc);
    if (k == 0) colalpha[nc] = 1.0 / (sx * t);
    double cr = 0.0, ci = 0.0;
    if (k < n) {
      const double2 c = c64[k * R + nc];
      cr = c.x * t;
      ci = c.y * t;
    }
    const double v[4] = {cr, -ci, ci, cr};
    const int64_t base0 = (2 * nc) * kn + 2 * k, base1 = (2 * nc + 1) * kn + 2 * k;
    const int64_t idx[4] = {base0, base0 + 1, base1, base1 + 1};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const S hp = Prec<S>::round(v[q]);
      p[idx[q]] = hp;
      r[idx[q]] = Prec<S>::round(v[q] - Prec<S>::widen(hp));
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// FP16 operands are scaled by powers of two (see the header comment).
template <typename S>
constexpr bool kScaled = std::is_same<S, _Float16>::value;

// workspace names per element size: {phi p, phi r, B p, B r}
template <typename S>
static const char* split_name(int which) {
  static const char* n32[4] = {"mf_phi_p32", "mf_phi_r32", "mf_bnn_p32", "mf_bnn_r32"};
  static const char* n16[4] = {"mf_phi_p16", "mf_phi_r16", "mf_bnn_p16", "mf_bnn_r16"};
  return sizeof(S) == 4 ? n32[which] : n16[which];
}

template <typename K>
static fx_status allow_lds_mfma(K kernel, size_t bytes) {
  return allow_dynamic_lds(reinterpret_cast<const void*>(kernel), bytes);
}

template <typename S>
static fx_status prepare_split_t(fx_ace* a, AceSplit* sp, hipStream_t st) {
  if (sp->ready) return FX_OK;
  const int64_t nr = a->nr;
  const int n = a->n;
  sp->kc = roundk(2 * nr);
  sp->kn = roundk(2 * (int64_t)n);
  const size_t cb = sizeof(S) * (size_t)n * sp->kc, rb = sizeof(S) * (size_t)nr * sp->kn;
  FX_TRY(ace_alloc(a, cb, &sp->col_p));
  FX_TRY(ace_alloc(a, cb, &sp->col_r));
  FX_TRY(ace_alloc(a, rb, &sp->row_p));
  FX_TRY(ace_alloc(a, rb, &sp->row_r));
  const unsigned* smax = nullptr;
  if (kScaled<S>) {
    // one power-of-two factor for all of xi, from its largest magnitude
    FX_TRY(ace_alloc(a, 256, &sp->smax));
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, (unsigned*)sp->smax, 1);
    FX_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_absmax<double>), dim3(std::max(1, 4096 / std::max(n, 1)) , (unsigned)n), dim3(256), 0, st,
                       (const double*)a->xi, 2 * nr, 2 * nr, 0, (unsigned*)sp->smax);
    FX_LAUNCH_CHECK();
    smax = (const unsigned*)sp->smax;
  }
  const int64_t tc = (int64_t)n * sp->kc;
  hipLaunchKernelGGL((k_split_col<S>), dim3((unsigned)std::min<int64_t>((tc + 255) / 256, 16384)), dim3(256), 0, st,
                     (const double*)a->xi, nr, n, sp->kc, (S*)sp->col_p, (S*)sp->col_r, smax);
  FX_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_split_row<S>), dim3((unsigned)((nr + 63) / 64), (unsigned)(sp->kn / 64)), dim3(256), 0, st,
                     (const double*)a->xi, nr, n, sp->kn, (S*)sp->row_p, (S*)sp->row_r, smax);
  FX_LAUNCH_CHECK();
  sp->ready = true;
  return FX_OK;
}

fx_status ace_prepare_split(fx_ace* a, fx_prec prec, hipStream_t st) {
  if (prec == FX_PREC_ACE_FP32R || prec == FX_PREC_ACE_FP32) return prepare_split_t<float>(a, &a->f32, st);
  if (prec == FX_PREC_ACE_BF16R || prec == FX_PREC_ACE_BF16) return prepare_split_t<uint16_t>(a, &a->b16, st);
  if (prec == FX_PREC_ACE_FP16R || prec == FX_PREC_ACE_FP16) return prepare_split_t<_Float16>(a, &a->f16, st);
  return FX_OK;
}

// Which GEMMs of the 2-byte forms run the direct-to-LDS kernel: the output
// GEMM y = -xi C (measured faster: at 96^3, N = R = 1024, 34 -> 36% of the
// BF16 matrix peak with the residual step, 25 -> 29% without), not C =
// xi^H phi, whose -i rows made at read time cost more VALU work than the
// staged kernel's LDS stores (35 -> 26%).  FX_ACE_DL = 0 uses neither, 2
// both (for comparison).
static bool ace_direct_lds(int mode) {
  const char* e = getenv("FX_ACE_DL");
  const int v = e ? atoi(e) : 1;
  return v == 2 || (v == 1 && mode == 1);
}

template <typename S, bool REFINE>
static fx_status apply_t(fx_ctx* ctx, Workspace* ws, fx_ace* a, AceSplit* sp, const void* phi, int R, int64_t ld_phi,
                         void* out, int64_t ld_out, fx_dtype in_dtype, fx_dtype out_dtype, hipStream_t st) {
  constexpr int BK = Prec<S>::BK;
  constexpr int LDK = BK + Prec<S>::PAD;
  const int64_t nr = a->nr;
  const int n = a->n;
  FX_TRY(prepare_split_t<S>(a, sp, st));
  // phi split (FP16: each right-hand side scaled by its own power of two)
  void *php = nullptr, *phr = nullptr;
  const size_t pb = sizeof(S) * (size_t)R * sp->kc;
  FX_TRY(ws_get(ctx, ws, split_name<S>(0), pb, &php));
  FX_TRY(ws_get(ctx, ws, split_name<S>(1), pb, &phr));
  unsigned* pmax = nullptr;
  double* colalpha = nullptr;
  if (kScaled<S>) {
    void* t = nullptr;
    FX_TRY(ws_get(ctx, ws, "mf_phimax", sizeof(unsigned) * (size_t)R, &t));
    pmax = (unsigned*)t;
    FX_TRY(ws_get(ctx, ws, "mf_colalpha", sizeof(double) * (size_t)R, &t));
    colalpha = (double*)t;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::min(64, (R + 255) / 256)), dim3(256), 0, st, pmax, R);
    FX_LAUNCH_CHECK();
    const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (2 * nr + 65535) / 65536)), (unsigned)R);
    if (in_dtype == FX_C128)
      hipLaunchKernelGGL((k_absmax<double>), g, dim3(256), 0, st, (const double*)phi, 2 * ld_phi, 2 * nr, 1, pmax);
    else
      hipLaunchKernelGGL((k_absmax<float>), g, dim3(256), 0, st, (const float*)phi, 2 * ld_phi, 2 * nr, 1, pmax);
    FX_LAUNCH_CHECK();
  }
  const int64_t tp = (int64_t)R * sp->kc;
  int slot;
  FX_TRY(prof_begin(ctx, st, FX_K_SPLIT, (double)R * nr * (in_dtype == FX_C128 ? 16 : 8) + 2.0 * pb, &slot));
  if (in_dtype == FX_C128)
    hipLaunchKernelGGL((k_split_phi<S, double>), dim3((unsigned)std::min<int64_t>((tp + 255) / 256, 16384)),
                       dim3(256), 0, st, (const double*)phi, ld_phi, nr, R, sp->kc, (S*)php, (S*)phr, pmax);
  else
    hipLaunchKernelGGL((k_split_phi<S, float>), dim3((unsigned)std::min<int64_t>((tp + 255) / 256, 16384)),
                       dim3(256), 0, st, (const float*)phi, ld_phi, nr, R, sp->kc, (S*)php, (S*)phr, pmax);
  FX_LAUNCH_CHECK();
  FX_TRY(prof_end(ctx, st, slot));

  const size_t lds = (size_t)(REFINE ? 4 : 2) * TBM * LDK * sizeof(S);
  // C = xi^H phi: M = n, N = 2R, K = kc, split over K
  {
    const int tiles_m = (n + TBM - 1) / TBM, tiles_n = (2 * R + TBN - 1) / TBN;
    const int tiles = tiles_m * tiles_n;
    const int64_t ksteps = sp->kc / BK;
    // the split depends on the reduction length only, so a column's result
    // does not depend on how many right-hand sides share the launch
    (void)tiles;
    // (up to 128 chunks of at least 16 steps: enough workgroups for a few
    // right-hand sides, where the output has only a handful of tiles)
    int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(128, ksteps / 16));
    if (const char* e = getenv("FX_ACE_NSPLIT")) nsplit = std::max(1, atoi(e));
    int64_t kchunk = (ksteps + nsplit - 1) / nsplit * BK;
    nsplit = (int)((sp->kc + kchunk - 1) / kchunk);
    void* part = nullptr;
    FX_TRY(ws_get(ctx, ws, "mf_partial", sizeof(double) * (size_t)nsplit * n * 2 * R, &part));
    auto kern = k_tn_mfma<S, REFINE, true, 0>;
    size_t lds_cn = lds;
    if constexpr (sizeof(S) == 2) {
      if (ace_direct_lds(0)) {
        kern = k_tn_mfma_dl<S, REFINE, true, 0>;
        lds_cn = 2 * dl_stage_bytes<S, REFINE, true>();
      }
    }
    FX_TRY(allow_lds_mfma(kern, lds_cn));
    FX_TRY(prof_begin(ctx, st, FX_K_GEMM_CN, (REFINE ? 3.0 : 1.0) * 2.0 * n * 2.0 * R * (double)sp->kc, &slot));
    hipLaunchKernelGGL(kern, dim3((unsigned)(tiles * nsplit)), dim3(256), lds_cn, st, n, 2 * R, (int)sp->kc,
                       (int)kchunk, (const S*)sp->col_p, (const S*)sp->col_r, sp->kc, (const S*)php, (const S*)phr,
                       sp->kc, (double*)part, (void*)nullptr, (int64_t)0, 0, 0.0, (const double*)nullptr, tiles_m,
                       tiles_n);
    FX_LAUNCH_CHECK();
    FX_TRY(prof_end(ctx, st, slot));
    // reduce -> B operand of the second product
    void *bp = nullptr, *br = nullptr;
    const size_t bb = sizeof(S) * (size_t)2 * R * sp->kn;
    FX_TRY(ws_get(ctx, ws, split_name<S>(2), bb, &bp));
    FX_TRY(ws_get(ctx, ws, split_name<S>(3), bb, &br));
    const int64_t tr = (int64_t)R * (sp->kn / 2);
    FX_TRY(prof_begin(ctx, st, FX_K_REDUCE, 8.0 * nsplit * n * 2.0 * R + 2.0 * bb, &slot));
    if (kScaled<S>) {
      void *c64 = nullptr, *cmax = nullptr;
      FX_TRY(ws_get(ctx, ws, "mf_c64", 16 * (size_t)n * R, &c64));
      FX_TRY(ws_get(ctx, ws, "mf_cmax", sizeof(unsigned) * (size_t)R, &cmax));
      hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::min(64, (R + 255) / 256)), dim3(256), 0, st,
                         (unsigned*)cmax, R);
      FX_LAUNCH_CHECK();
      const int64_t tc = (int64_t)n * R;
      hipLaunchKernelGGL(k_sum_cn_scaled, dim3((unsigned)std::min<int64_t>((tc + 255) / 256, 16384)), dim3(256), 0,
                         st, (const double*)part, nsplit, n, R, (const unsigned*)sp->smax, (const unsigned*)pmax,
                         (double2*)c64, (unsigned*)cmax);
      FX_LAUNCH_CHECK();
      hipLaunchKernelGGL((k_split_cn_scaled<S>), dim3((unsigned)std::min<int64_t>((tr + 255) / 256, 16384)),
                         dim3(256), 0, st, (const double2*)c64, n, R, sp->kn, (const unsigned*)sp->smax,
                         (const unsigned*)cmax, (S*)bp, (S*)br, colalpha);
    } else {
      hipLaunchKernelGGL((k_reduce_cn<S>), dim3((unsigned)std::min<int64_t>((tr + 255) / 256, 16384)), dim3(256), 0,
                         st, (const double*)part, nsplit, n, R, sp->kn, (S*)bp, (S*)br);
    }
    FX_LAUNCH_CHECK();
    FX_TRY(prof_end(ctx, st, slot));
    // y = -xi C: M = nr, N = 2R, K = kn
    const int tm2 = (int)((nr + TBM - 1) / TBM), tn2 = (2 * R + TBN - 1) / TBN;
    auto kern2 = k_tn_mfma<S, REFINE, false, 1>;
    // the epilogue turns each wave's 32x32 tiles around in 32 x 33 doubles of LDS
    size_t lds2 = std::max(lds, (size_t)4 * 32 * 33 * sizeof(double));
    if constexpr (sizeof(S) == 2) {
      if (ace_direct_lds(1)) {
        kern2 = k_tn_mfma_dl<S, REFINE, false, 1>;
        lds2 = std::max(2 * dl_stage_bytes<S, REFINE, false>(), (size_t)4 * 32 * 33 * sizeof(double));
      }
    }
    FX_TRY(allow_lds_mfma(kern2, lds2));
    FX_TRY(prof_begin(ctx, st, FX_K_GEMM_NN, (REFINE ? 3.0 : 1.0) * 2.0 * (double)nr * 2.0 * R * (double)sp->kn, &slot));
    hipLaunchKernelGGL(kern2, dim3((unsigned)(tm2 * tn2)), dim3(256), lds2, st, (int)nr, 2 * R, (int)sp->kn,
                       (int)sp->kn, (const S*)sp->row_p, (const S*)sp->row_r, sp->kn, (const S*)bp, (const S*)br,
                       sp->kn, (double*)nullptr, out, ld_out, out_dtype == FX_C64 ? 1 : 0, 1.0,
                       (const double*)colalpha, tm2, tn2);
    FX_LAUNCH_CHECK();
    FX_TRY(prof_end(ctx, st, slot));
  }
  return FX_OK;
}

fx_status ace_apply_mfma(fx_ctx* ctx, Workspace* ws, fx_ace* a, const void* phi, int nphi, int64_t ld_phi, void* out,
                         int64_t ld_out, fx_dtype in_dtype, fx_dtype out_dtype, fx_prec prec, hipStream_t st) {
  switch (prec) {
    case FX_PREC_ACE_FP32R:
      return apply_t<float, true>(ctx, ws, a, &a->f32, phi, nphi, ld_phi, out, ld_out, in_dtype, out_dtype, st);
    case FX_PREC_ACE_FP32:
      return apply_t<float, false>(ctx, ws, a, &a->f32, phi, nphi, ld_phi, out, ld_out, in_dtype, out_dtype, st);
    case FX_PREC_ACE_BF16R:
      return apply_t<uint16_t, true>(ctx, ws, a, &a->b16, phi, nphi, ld_phi, out, ld_out, in_dtype, out_dtype, st);
    case FX_PREC_ACE_BF16:
      return apply_t<uint16_t, false>(ctx, ws, a, &a->b16, phi, nphi, ld_phi, out, ld_out, in_dtype, out_dtype, st);
    case FX_PREC_ACE_FP16R:
      return apply_t<_Float16, true>(ctx, ws, a, &a->f16, phi, nphi, ld_phi, out, ld_out, in_dtype, out_dtype, st);
    case FX_PREC_ACE_FP16:
      return apply_t<_Float16, false>(ctx, ws, a, &a->f16, phi, nphi, ld_phi, out, ld_out, in_dtype, out_dtype, st);
    default:
      FX_FAIL(FX_ERR_UNSUPPORTED, "precision %d is not a matrix-core ACE precision", prec);
  }
}

}  // namespace fx
