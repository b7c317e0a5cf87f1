// Register and LDS building blocks of libfock's batched 3D FFTs (gfx950).
//
// A length-n transform (n = 2^a 3^b <= 96) is a sequence of in-place
// Cooley-Tukey stages over data resident in LDS.  Forward transforms use
// decimation in frequency: natural-order input, output in mixed-radix
// digit-reversed order.  Inverse transforms apply the adjoint stages in reverse
// order, so they take exactly that permuted order and return natural order.
// The spectrum is therefore never un-permuted: the pointwise kernel multiply
// between the forward and inverse transforms reads K at the permuted
// positions.  Inside a stage each thread runs whole radix-R butterflies in
// registers (R in {2,3,4,6,8,9,12}); composite radices are evaluated in
// registers by a nested four-step with compile-time twiddles.
//
// Everything here is __host__ __device__ so the same stage code can be run on
// the host to check plans against a direct DFT.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

// Everything is force-inlined: a call inside a kernel would cost a stack
// frame in scratch memory and block register allocation across the stages.
#define FX_HD __host__ __device__ inline __attribute__((always_inline))

namespace fx {

// ---- complex arithmetic -----------------------------------------------------
template <typename T>
FX_HD cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
FX_HD cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
FX_HD cpx<T> cmul(cpx<T> a, cpx<T> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
FX_HD float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
FX_HD double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
// acc + a*b as four fused multiply-adds (written as cadd(acc, cmul(a, b)) the
// compiler emits a multiply, a fused multiply-add and an add per component)
template <typename T>
FX_HD cpx<T> cfma(cpx<T> acc, cpx<T> a, cpx<T> b) {
  acc.x = fmadd(a.x, b.x, acc.x);
  acc.x = fmadd(-a.y, b.y, acc.x);
  acc.y = fmadd(a.x, b.y, acc.y);
  acc.y = fmadd(a.y, b.x, acc.y);
  return acc;
}
// a * conj(b)
template <typename T>
FX_HD cpx<T> cmulc(cpx<T> a, cpx<T> b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }
// conj(a) * b
template <typename T>
FX_HD cpx<T> cconjmul(cpx<T> a, cpx<T> b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }
template <typename T>
FX_HD cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by +i (s > 0) or -i (s < 0)
template <int S, typename T>
FX_HD cpx<T> mul_i(cpx<T> a) { return S > 0 ? cpx<T>{-a.y, a.x} : cpx<T>{a.y, -a.x}; }

// ---- compile-time sin/cos of 2 pi p / q ------------------------------------
// The angle is written as m*(pi/2) +- z with z in [0, pi/4] using integer
// arithmetic on p/q, then sin z and cos z come from their Taylor series,
// which converge to double precision there in a handful of terms.
namespace ct {
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double sin_series(double z) {
  double term = z, sum = z, z2 = z * z;
  for (int k = 1; k < 14; ++k) {
    term *= -z2 / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cos_series(double z) {
  double term = 1.0, sum = 1.0, z2 = z * z;
  for (int k = 1; k < 14; ++k) {
    term *= -z2 / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// returns {cos, sin} of 2 pi p/q
struct cs {
  double c, s;
};
constexpr cs turn(long p, long q) {
  long pp = ((p % q) + q) % q;             // [0, q)
  long o = (8 * pp) / q;                   // octant 0..7
  long r = 8 * pp - o * q;                 // remainder in [0, q)
  double z = 0.0;
  long m = 0;
  int sgn = 1;
  if (o % 2 == 0) {
    m = o / 2;
    z = (double)r / (double)q * (kPi / 4.0);
    sgn = 1;
  } else {
    m = (o + 1) / 2;
    z = (double)(q - r) / (double)q * (kPi / 4.0);
    sgn = -1;
  }
  double sz = sgn * sin_series(z), cz = cos_series(z);
  // angle = m*pi/2 + sz-angle
  switch (m % 4) {
    case 0: return {cz, sz};
    case 1: return {-sz, cz};
    case 2: return {-cz, -sz};
    default: return {sz, -cz};
  }
}
}  // namespace ct

// Multiply by exp(2 pi i e / R) for a compile-time-resolvable e (loops below
// are fully unrolled, so e is a constant and the branches fold away).
template <int R, typename T>
FX_HD cpx<T> twc(cpx<T> a, int e) {
  e = ((e % R) + R) % R;
  if (e == 0) return a;
  if (2 * e == R) return {-a.x, -a.y};
  if (4 * e == R) return mul_i<1>(a);
  if (4 * e == 3 * R) return mul_i<-1>(a);
  const ct::cs w = ct::turn(e, R);
  return cmul(a, cpx<T>{(T)w.c, (T)w.s});
}

// ---- in-register DFTs: x[k] <- sum_m x[m] exp(S 2 pi i m k / R) -------------
template <int R>
struct first_factor {
  static constexpr int value = (R % 4 == 0 && R != 4) ? 4 : (R % 2 == 0 && R != 2) ? 2 : (R % 3 == 0 && R != 3) ? 3 : R;
};

template <int R, int S, typename T>
struct Dft;

template <int S, typename T>
struct Dft<1, S, T> {
  FX_HD static void run(cpx<T>*) {}
};

template <int S, typename T>
struct Dft<2, S, T> {
  FX_HD static void run(cpx<T>* x) {
    cpx<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int S, typename T>
struct Dft<3, S, T> {
  FX_HD static void run(cpx<T>* x) {
    const T h = (T)0.5;
    const T r3 = (T)0.86602540378443864676372317075293618;  // sqrt(3)/2
    cpx<T> s = cadd(x[1], x[2]);
    cpx<T> d = csub(x[1], x[2]);
    cpx<T> t = {x[0].x - h * s.x, x[0].y - h * s.y};
    cpx<T> u = mul_i<S>(cpx<T>{r3 * d.x, r3 * d.y});
    x[0] = cadd(x[0], s);
    x[1] = cadd(t, u);
    x[2] = csub(t, u);
  }
};

template <int S, typename T>
struct Dft<4, S, T> {
  FX_HD static void run(cpx<T>* x) {
    cpx<T> a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    cpx<T> c = cadd(x[1], x[3]), d = mul_i<S>(csub(x[1], x[3]));
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cadd(b, d);
    x[3] = csub(b, d);
  }
};

// Composite R = A*B: input index m = B*m1 + m2, output index k = k1 + A*k2.
template <int R, int S, typename T>
struct Dft {
  static constexpr int A = first_factor<R>::value;
  static constexpr int B = R / A;
  FX_HD static void run(cpx<T>* x) {
    cpx<T> t[B][A];
#pragma unroll
    for (int m2 = 0; m2 < B; ++m2) {
#pragma unroll
      for (int m1 = 0; m1 < A; ++m1) t[m2][m1] = x[B * m1 + m2];
      Dft<A, S, T>::run(t[m2]);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) t[m2][k1] = twc<R, T>(t[m2][k1], S * m2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cpx<T> b[B];
#pragma unroll
      for (int m2 = 0; m2 < B; ++m2) b[m2] = t[m2][k1];
      Dft<B, S, T>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) x[k1 + A * k2] = b[k2];
    }
  }
};

// ---- one radix-R stage over `count` transforms held in LDS -----------------
// Element i of transform f is s[f*fs + i*es].  L is the current sub-transform
// length and span = L/R.  tw[t] = exp(-2 pi i t/n), t < n.
// FWD: gather R points at stride span, DFT (sign -), multiply output k by
//      w_L^{i2 k}, scatter back.  INV: the adjoint (conjugate twiddles first,
//      DFT with sign +).
// Butterflies are dealt to threads with consecutive threads on consecutive
// transforms f.
template <int R, bool FWD, typename T>
FX_HD void stage_bfly(cpx<T>* s, int n, int L, int count, int es, int fs, const cpx<T>* tw, int b) {
  const int span = L / R;
  const int f = b % count;
  const int q = b / count;
  const int blk = q / span;
  const int i2 = q - blk * span;
  const int tstep = n / L;
  const int base = f * fs + (blk * L + i2) * es;
  const int step = span * es;
  cpx<T> x[R];
#pragma unroll
  for (int m = 0; m < R; ++m) x[m] = s[base + m * step];
  // the last forward stage (first inverse stage) has span 1: i2 = 0 and
  // every twiddle is 1
  if (FWD) {
    Dft<R, -1, T>::run(x);
    if (span > 1) {
#pragma unroll
      for (int k = 1; k < R; ++k) x[k] = cmul(x[k], tw[i2 * k * tstep]);
    }
  } else {
    if (span > 1) {
#pragma unroll
      for (int k = 1; k < R; ++k) x[k] = cmulc(x[k], tw[i2 * k * tstep]);
    }
    Dft<R, 1, T>::run(x);
  }
#pragma unroll
  for (int m = 0; m < R; ++m) s[base + m * step] = x[m];
}

// All butterflies of one stage, dealt round-robin to threads tid, tid+nthr, ...
template <int R, bool FWD, typename T>
FX_HD void stage_loop(cpx<T>* s, int n, int L, int count, int es, int fs, const cpx<T>* tw, int tid, int nthr) {
  const int total = count * (n / R);
  for (int b = tid; b < total; b += nthr) stage_bfly<R, FWD, T>(s, n, L, count, es, fs, tw, b);
}

template <bool FWD, typename T>
FX_HD void stage_dispatch(int R, cpx<T>* s, int n, int L, int count, int es, int fs, const cpx<T>* tw, int tid,
                          int nthr) {
  switch (R) {
    case 2: stage_loop<2, FWD, T>(s, n, L, count, es, fs, tw, tid, nthr); break;
    case 3: stage_loop<3, FWD, T>(s, n, L, count, es, fs, tw, tid, nthr); break;
    case 4: stage_loop<4, FWD, T>(s, n, L, count, es, fs, tw, tid, nthr); break;
    case 6: stage_loop<6, FWD, T>(s, n, L, count, es, fs, tw, tid, nthr); break;
    case 8: stage_loop<8, FWD, T>(s, n, L, count, es, fs, tw, tid, nthr); break;
    case 9: stage_loop<9, FWD, T>(s, n, L, count, es, fs, tw, tid, nthr); break;
    case 12: stage_loop<12, FWD, T>(s, n, L, count, es, fs, tw, tid, nthr); break;
    default: break;
  }
}

// Plan in kernel-argument form.
struct AxisArg {
  int n, nst;
  int R[4];
};

// Barrier policies: the device one is the workgroup barrier; the host one is
// empty, used when a single host "thread" (tid 0, nthr 1) runs every
// butterfly of a stage before the next stage starts.
struct DeviceSync {
  __device__ void operator()() const { __syncthreads(); }
};
struct HostSync {
  __host__ void operator()() const {}
};

// Forward or inverse transform along one axis of an LDS-resident block,
// executed by threads tid < nthr of the workgroup with a barrier after every
// stage.  Every thread of the workgroup must call it.
template <bool FWD, typename T, class Sync>
FX_HD void lds_fft(cpx<T>* s, const AxisArg& a, int count, int es, int fs, const cpx<T>* tw, int tid, int nthr,
                   Sync sync) {
  if (FWD) {
    int L = a.n;
    for (int st = 0; st < a.nst; ++st) {
      stage_dispatch<true, T>(a.R[st], s, a.n, L, count, es, fs, tw, tid, nthr);
      sync();
      L /= a.R[st];
    }
  } else {
    // stage st of the forward run had L_st = n / (R_0 ... R_{st-1})
    for (int st = a.nst - 1; st >= 0; --st) {
      int L = a.n;
      for (int u = 0; u < st; ++u) L /= a.R[u];
      stage_dispatch<false, T>(a.R[st], s, a.n, L, count, es, fs, tw, tid, nthr);
      sync();
    }
  }
}

// ---- convolution along one axis: forward FFT, pointwise factor, inverse ----
// The last forward stage has span 1, so each of its butterflies owns R
// consecutive positions — exactly the points the first inverse stage
// combines.  That stage, the pointwise factor and the first inverse stage
// therefore run in registers as one pass.  kf(pos, f) is the real factor at
// digit-reversed position pos of transform f.
template <int R, typename T, class KF>
FX_HD void mid_bfly(cpx<T>* s, int count, int es, int fs, int b, KF kf) {
  const int f = b % count;
  const int blk = b / count;
  const int base = f * fs + blk * R * es;
  cpx<T> x[R];
#pragma unroll
  for (int m = 0; m < R; ++m) x[m] = s[base + m * es];
  Dft<R, -1, T>::run(x);
#pragma unroll
  for (int k = 0; k < R; ++k) x[k] = cscale(x[k], kf(blk * R + k, f));
  Dft<R, 1, T>::run(x);
#pragma unroll
  for (int m = 0; m < R; ++m) s[base + m * es] = x[m];
}

template <int R, typename T, class KF>
FX_HD void mid_loop(cpx<T>* s, int n, int count, int es, int fs, KF kf, int tid, int nthr) {
  const int total = count * (n / R);
  for (int b = tid; b < total; b += nthr) mid_bfly<R, T>(s, count, es, fs, b, kf);
}

template <typename T, class KF>
FX_HD void mid_dispatch(int R, cpx<T>* s, int n, int count, int es, int fs, KF kf, int tid, int nthr) {
  switch (R) {
    case 2: mid_loop<2, T>(s, n, count, es, fs, kf, tid, nthr); break;
    case 3: mid_loop<3, T>(s, n, count, es, fs, kf, tid, nthr); break;
    case 4: mid_loop<4, T>(s, n, count, es, fs, kf, tid, nthr); break;
    case 6: mid_loop<6, T>(s, n, count, es, fs, kf, tid, nthr); break;
    case 8: mid_loop<8, T>(s, n, count, es, fs, kf, tid, nthr); break;
    case 9: mid_loop<9, T>(s, n, count, es, fs, kf, tid, nthr); break;
    case 12: mid_loop<12, T>(s, n, count, es, fs, kf, tid, nthr); break;
    default: break;
  }
}

template <typename T, class KF, class Sync>
FX_HD void lds_conv(cpx<T>* s, const AxisArg& a, int count, int es, int fs, const cpx<T>* tw, KF kf, int tid,
                    int nthr, Sync sync) {
  int L = a.n;
  for (int st = 0; st + 1 < a.nst; ++st) {
    stage_dispatch<true, T>(a.R[st], s, a.n, L, count, es, fs, tw, tid, nthr);
    sync();
    L /= a.R[st];
  }
  mid_dispatch<T>(a.R[a.nst - 1], s, a.n, count, es, fs, kf, tid, nthr);
  sync();
  for (int st = a.nst - 2; st >= 0; --st) {
    int Ls = a.n;
    for (int u = 0; u < st; ++u) Ls /= a.R[u];
    stage_dispatch<false, T>(a.R[st], s, a.n, Ls, count, es, fs, tw, tid, nthr);
    sync();
  }
}

}  // namespace fx
