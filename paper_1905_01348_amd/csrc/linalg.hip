// FP64 complex dense linear algebra for the ACE operator (hand-written HIP):
//   zgemm   C = alpha op(A) op(B) + beta C, op in {N, C}, batched, split over K
//           with a fixed-order FP64 reduction of the split partial sums;
//   potrf   blocked Cholesky of a Hermitian positive definite matrix (lower);
//   trinv   inverse of a lower triangular matrix (recursive 2x2 blocking);
//   herm    Hermitised copy, its negation and half its trace.
// All matrices are column-major complex double: element (i, j) at P[i + j*ld].
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <vector>

#include "common.hpp"
#include "fft.hpp"
#include "linalg.hpp"

namespace fx {

using z = cpx<double>;

FX_HD z zconj(z a) { return {a.x, -a.y}; }
// acc + a*b as four fused multiply-adds (written as `acc += a.x*b.x - a.y*b.y`
// the compiler emits a multiply, a fused multiply-add and an add per
// component: six FP64 instructions instead of four)
FX_HD z zfma(z acc, z a, z b) {
  acc.x = __builtin_fma(a.x, b.x, acc.x);
  acc.x = __builtin_fma(-a.y, b.y, acc.x);
  acc.y = __builtin_fma(a.x, b.y, acc.y);
  acc.y = __builtin_fma(a.y, b.x, acc.y);
  return acc;
}

// ---------------------------------------------------------------------------
// zgemm: 128x64 output tile per 256-thread workgroup, K steps of 8; each
// thread owns an 8x4 block of outputs (rows tx + 16 i, cols ty + 16 j), so
// one LDS read feeds 2.7 complex multiply-adds.  The next K step's tiles are
// loaded into registers while the current one is multiplied out of the other
// half of a double-buffered LDS, one barrier per step.
// Split over K: blockIdx.z = batch * nsplit + split; split s covers
// K range [s*kchunk, min(K, (s+1)*kchunk)).  With a partial buffer the raw
// sum of split s goes to partial[(batch*nsplit + s) * M*N] (ld M); without
// one (nsplit == 1) the result C = alpha*sum + beta*C is written directly.
// ---------------------------------------------------------------------------
constexpr int ZBM = 128, ZBN = 64, ZK = 8;

template <int OPA, int OPB>
__global__ void __launch_bounds__(256, 2) k_zgemm(int M, int N, int K, const z* __restrict__ A, int64_t lda,
                                               int64_t sA, const z* __restrict__ B, int64_t ldb, int64_t sB,
                                               z* C, int64_t ldc, int64_t sC, z alpha, z beta, int nsplit,
                                               int kchunk, z* __restrict__ partial) {
  __shared__ z As[2][ZK][ZBM + 1];
  __shared__ z Bs[2][ZK][ZBN + 1];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int m0 = blockIdx.x * ZBM, n0 = blockIdx.y * ZBN;
  const int bz = blockIdx.z, batch = bz / nsplit, split = bz % nsplit;
  A += batch * sA;
  B += batch * sB;
  const int kbeg = split * kchunk, kend = min(K, kbeg + kchunk);
  // staged loads: the A tile (128 x 8) is 4 elements per thread, the B tile
  // (8 x 64) 2; op C reads along k (column of the stored matrix).  Element
  // u of this thread sits at (row a_m(u), step a_k(u)) of the A tile and at
  // (step b_k(u), column b_n(u)) of the B tile.
  const auto a_m = [tid](int u) { return OPA == 0 ? (tid + 256 * u) % ZBM : (tid + 256 * u) / ZK; };
  const auto a_k = [tid](int u) { return OPA == 0 ? (tid + 256 * u) / ZBM : (tid + 256 * u) % ZK; };
  const auto b_n = [tid](int u) { return OPB == 0 ? (tid + 256 * u) / ZK : (tid + 256 * u) % ZBN; };
  const auto b_k = [tid](int u) { return OPB == 0 ? (tid + 256 * u) % ZK : (tid + 256 * u) / ZBN; };
  z ra0, ra1, ra2, ra3, rb0, rb1;
#define FX_ZG_LOAD_A(u, dst)                                                                     \
  {                                                                                              \
    const int m = m0 + a_m(u), k = k0n + a_k(u);                                                \
    dst = z{0.0, 0.0};                                                                           \
    if (m < M && k < kend) dst = OPA == 0 ? A[m + (int64_t)k * lda] : zconj(A[k + (int64_t)m * lda]); \
  }
#define FX_ZG_LOAD_B(u, dst)                                                                     \
  {                                                                                              \
    const int n = n0 + b_n(u), k = k0n + b_k(u);                                                \
    dst = z{0.0, 0.0};                                                                           \
    if (n < N && k < kend) dst = OPB == 0 ? B[k + (int64_t)n * ldb] : zconj(B[n + (int64_t)k * ldb]); \
  }
#define FX_ZG_GLOAD()      \
  FX_ZG_LOAD_A(0, ra0);    \
  FX_ZG_LOAD_A(1, ra1);    \
  FX_ZG_LOAD_A(2, ra2);    \
  FX_ZG_LOAD_A(3, ra3);    \
  FX_ZG_LOAD_B(0, rb0);    \
  FX_ZG_LOAD_B(1, rb1);
#define FX_ZG_SSTORE(bf)                  \
  As[bf][a_k(0)][a_m(0)] = ra0;           \
  As[bf][a_k(1)][a_m(1)] = ra1;           \
  As[bf][a_k(2)][a_m(2)] = ra2;           \
  As[bf][a_k(3)][a_m(3)] = ra3;           \
  Bs[bf][b_k(0)][b_n(0)] = rb0;           \
  Bs[bf][b_k(1)][b_n(1)] = rb1;
  z acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = z{0.0, 0.0};
  if (kbeg < kend) {
    const int k0n = kbeg;
    FX_ZG_GLOAD();
    FX_ZG_SSTORE(0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += ZK) {
    const bool more = k0 + ZK < kend;
    if (more) {
      const int k0n = k0 + ZK;
      FX_ZG_GLOAD();
    }
#pragma unroll 2
    for (int kk = 0; kk < ZK; ++kk) {
      // the step's operands are read before its multiply-adds, so that the
      // LDS reads overlap
      z b[4], a[8];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[buf][kk][ty + 16 * j];
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = As[buf][kk][tx + 16 * i];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = zfma(acc[i][j], a[i], b[j]);
    }
    if (more) {
      FX_ZG_SSTORE(buf ^ 1);
    }
    __syncthreads();
    buf ^= 1;
  }
#undef FX_ZG_SSTORE
#undef FX_ZG_GLOAD
#undef FX_ZG_LOAD_B
#undef FX_ZG_LOAD_A
  if (partial) {
    z* P = partial + (int64_t)bz * M * N;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + tx + 16 * i, n = n0 + ty + 16 * j;
        if (m < M && n < N) P[m + (int64_t)n * M] = acc[i][j];
      }
  } else {
    z* Cb = C + batch * sC;
    const bool bz0 = beta.x == 0.0 && beta.y == 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + tx + 16 * i, n = n0 + ty + 16 * j;
        if (m < M && n < N) {
          z r = cmul(alpha, acc[i][j]);
          if (!bz0) r = cadd(r, cmul(beta, Cb[m + (int64_t)n * ldc]));
          Cb[m + (int64_t)n * ldc] = r;
        }
      }
  }
}

// C = alpha * sum_s partial_s + beta * C, summing splits in ascending order.
__global__ void k_split_reduce(int M, int N, int nsplit, int nbatch, const z* __restrict__ partial, z* C,
                               int64_t ldc, int64_t sC, z alpha, z beta) {
  const int64_t MN = (int64_t)M * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < MN * nbatch;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / MN, e = i - b * MN;
    const int64_t m = e % M, n = e / M;
    z s = {0.0, 0.0};
    for (int q = 0; q < nsplit; ++q) s = cadd(s, partial[(b * nsplit + q) * MN + e]);
    z r = cmul(alpha, s);
    z* c = C + b * sC + m + n * ldc;
    if (!(beta.x == 0.0 && beta.y == 0.0)) r = cadd(r, cmul(beta, *c));
    *c = r;
  }
}

fx_status zgemm(fx_ctx* ctx, Workspace* ws, hipStream_t st, int opa, int opb, int M, int N, int K, z alpha,
                const void* A, int64_t lda, const void* B, int64_t ldb, z beta, void* C, int64_t ldc, int batch,
                int64_t sA, int64_t sB, int64_t sC, int nsplit_hint) {
  if (M <= 0 || N <= 0) return FX_OK;
  if (K <= 0) {
    // empty sum: C = beta C (no splits to add)
    hipLaunchKernelGGL(k_split_reduce, dim3(std::min<int64_t>(((int64_t)M * N * batch + 255) / 256, 4096)),
                       dim3(256), 0, st, M, N, 0, batch, (const z*)nullptr, (z*)C, ldc, sC, alpha, beta);
    FX_LAUNCH_CHECK();
    return FX_OK;
  }
  const int tiles = ((M + ZBM - 1) / ZBM) * ((N + ZBN - 1) / ZBN) * batch;
  int nsplit = nsplit_hint;
  if (nsplit <= 0) {
    // enough workgroups to fill the chip (per_cu per CU: 16 measured 2-4%
    // faster than 4 for the 1024 x 1024 overlaps at 96^3), each with at least
    // 512 K-steps
    int per_cu = 16;
    if (const char* e = getenv("FX_ZGEMM_PER_CU")) per_cu = std::max(1, std::min(64, atoi(e)));
    const int want = std::max(1, (per_cu * std::max(ctx->n_cu, 1)) / std::max(tiles, 1));
    nsplit = std::max(1, std::min(want, K / 4096));
  }
  int kchunk = (K + nsplit - 1) / nsplit;
  kchunk = (kchunk + ZK - 1) / ZK * ZK;
  nsplit = (K + kchunk - 1) / kchunk;
  z* part = nullptr;
  if (nsplit > 1) {
    void* p = nullptr;
    FX_TRY(ws_get(ctx, ws, "zgemm_part", sizeof(z) * (size_t)M * N * nsplit * batch, &p));
    part = (z*)p;
  }
  dim3 grid((M + ZBM - 1) / ZBM, (N + ZBN - 1) / ZBN, nsplit * batch);
  int slot;
  FX_TRY(prof_begin(ctx, st, opa ? FX_K_GEMM_CN : FX_K_GEMM_NN, 8.0 * M * N * (double)K * batch, &slot));
#define FX_ZG(a, b)                                                                                                 \
  hipLaunchKernelGGL((k_zgemm<a, b>), grid, dim3(256), 0, st, M, N, K, (const z*)A, lda, sA, (const z*)B, ldb, sB, \
                     (z*)C, ldc, sC, alpha, beta, nsplit, kchunk, part)
  if (opa == 0 && opb == 0)
    FX_ZG(0, 0);
  else if (opa == 0)
    FX_ZG(0, 1);
  else if (opb == 0)
    FX_ZG(1, 0);
  else
    FX_ZG(1, 1);
#undef FX_ZG
  FX_LAUNCH_CHECK();
  FX_TRY(prof_end(ctx, st, slot));
  if (nsplit > 1) {
    FX_TRY(prof_begin(ctx, st, FX_K_REDUCE, 16.0 * M * N * batch * (nsplit + 2.0), &slot));
    hipLaunchKernelGGL(k_split_reduce, dim3(std::min<int64_t>(((int64_t)M * N * batch + 255) / 256, 4096)),
                       dim3(256), 0, st, M, N, nsplit, batch, (const z*)part, (z*)C, ldc, sC, alpha, beta);
    FX_LAUNCH_CHECK();
    FX_TRY(prof_end(ctx, st, slot));
  }
  return FX_OK;
}

// ---------------------------------------------------------------------------
// Hermitisation: H = (M + M^H)/2, Aneg = -H, ex = 1/2 Re tr H.
// ---------------------------------------------------------------------------
__global__ void k_herm(int n, const z* __restrict__ M, int64_t ldm, z* __restrict__ H, z* __restrict__ Aneg) {
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const z a = M[i + (int64_t)j * ldm], b = M[j + (int64_t)i * ldm];
    z h = {0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
    if (i == j) h.y = 0.0;
    H[e] = h;
    Aneg[e] = z{-h.x, -h.y};
  }
}

__global__ void k_half_trace(int n, const z* __restrict__ H, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += H[i + (int64_t)i * n].x;
    *out = 0.5 * s;
  }
}

// ---------------------------------------------------------------------------
// Blocked Cholesky, lower: A = L L^H, block size CB.
// ---------------------------------------------------------------------------
constexpr int CB = 32;

// Unblocked factorisation of the nb x nb diagonal block at (k, k), in LDS.
// A non-positive or non-finite pivot records column+1 in *info (first one
// wins) and is replaced by 1 so the rest stays finite.
__global__ void __launch_bounds__(256) k_potrf_diag(int n, z* A, int64_t lda, int k, int* info) {
  __shared__ z S[CB][CB + 1];
  __shared__ double piv;
  const int nb = min(CB, n - k);
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e % nb, j = e / nb;
    S[i][j] = A[(k + i) + (int64_t)(k + j) * lda];
  }
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    if (tid == 0) {
      double d = S[c][c].x;
      if (!(d > 0.0) || !isfinite(d)) {
        if (*info == 0) *info = k + c + 1;
        d = 1.0;
      }
      piv = sqrt(d);
      S[c][c] = z{piv, 0.0};
    }
    __syncthreads();
    const double inv = 1.0 / piv;
    for (int r = c + 1 + tid; r < nb; r += 256) S[r][c] = z{S[r][c].x * inv, S[r][c].y * inv};
    __syncthreads();
    const int rem = nb - c - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      const int r = c + 1 + e % rem, s = c + 1 + e / rem;
      if (s <= r) {
        const z a = S[r][c], b = S[s][c];
        S[r][s] = z{S[r][s].x - (a.x * b.x + a.y * b.y), S[r][s].y - (a.y * b.x - a.x * b.y)};
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e % nb, j = e / nb;
    A[(k + i) + (int64_t)(k + j) * lda] = i >= j ? S[i][j] : z{0.0, 0.0};
  }
}

// Rows below the diagonal block: L[r, k:k+nb] = A[r, k:k+nb] L_kk^{-H}.
// One thread per row; x L_kk^H = a solved by forward substitution.
__global__ void __launch_bounds__(256) k_potrf_panel(int n, z* A, int64_t lda, int k) {
  __shared__ z Lk[CB][CB + 1];
  const int nb = min(CB, n - k);
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e % nb, j = e / nb;
    Lk[i][j] = A[(k + i) + (int64_t)(k + j) * lda];
  }
  __syncthreads();
  const int r = k + nb + blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  z x[CB];
  for (int c = 0; c < nb; ++c) {
    z a = A[r + (int64_t)(k + c) * lda];
    for (int s = 0; s < c; ++s) {
      // a -= x_s * conj(L[c][s])
      const z l = Lk[c][s];
      a.x -= x[s].x * l.x + x[s].y * l.y;
      a.y -= x[s].y * l.x - x[s].x * l.y;
    }
    const double d = Lk[c][c].x;
    x[c] = z{a.x / d, a.y / d};
  }
  for (int c = 0; c < nb; ++c) A[r + (int64_t)(k + c) * lda] = x[c];
}

__global__ void k_zero_upper(int n, z* A, int64_t lda) {
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i < j) A[i + (int64_t)j * lda] = z{0.0, 0.0};
  }
}

fx_status zpotrf(fx_ctx* ctx, Workspace* ws, hipStream_t st, int n, void* A, int64_t lda, int* info_dev) {
  z* a = (z*)A;
  for (int k = 0; k < n; k += CB) {
    const int nb = std::min(CB, n - k);
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, n, a, lda, k, info_dev);
    FX_LAUNCH_CHECK();
    const int rest = n - k - nb;
    if (rest <= 0) break;
    hipLaunchKernelGGL(k_potrf_panel, dim3((rest + 255) / 256), dim3(256), 0, st, n, a, lda, k);
    FX_LAUNCH_CHECK();
    // trailing update A22 -= L21 L21^H
    z* L21 = a + (k + nb) + (int64_t)k * lda;
    z* A22 = a + (k + nb) + (int64_t)(k + nb) * lda;
    FX_TRY(zgemm(ctx, ws, st, 0, 1, rest, rest, nb, z{-1.0, 0.0}, L21, lda, L21, lda, z{1.0, 0.0}, A22, lda, 1, 0,
                 0, 0, 1));
  }
  hipLaunchKernelGGL(k_zero_upper, dim3(std::min(((int64_t)n * n + 255) / 256, (int64_t)4096)), dim3(256), 0, st, n,
                     a, lda);
  FX_LAUNCH_CHECK();
  return FX_OK;
}

// ---------------------------------------------------------------------------
// Inverse of a lower triangular matrix, in place.
// ---------------------------------------------------------------------------
// Diagonal block (nb <= CB) at (k, k) inverted by forward substitution, one
// thread per column.
__global__ void __launch_bounds__(64) k_trinv_diag(z* A, int64_t lda, int k, int nb) {
  __shared__ z S[CB][CB + 1];
  __shared__ z X[CB][CB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 64) {
    const int i = e % nb, j = e / nb;
    S[i][j] = A[(k + i) + (int64_t)(k + j) * lda];
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < nb) {
    for (int r = 0; r < nb; ++r) X[r][c] = z{0.0, 0.0};
    const z d = S[c][c];
    const double dd = d.x * d.x + d.y * d.y;
    X[c][c] = z{d.x / dd, -d.y / dd};
    for (int r = c + 1; r < nb; ++r) {
      z s = {0.0, 0.0};
      for (int q = c; q < r; ++q) s = zfma(s, S[r][q], X[q][c]);
      const z l = S[r][r];
      const double ll = l.x * l.x + l.y * l.y;
      // X[r][c] = -s / l
      X[r][c] = z{-(s.x * l.x + s.y * l.y) / ll, -(s.y * l.x - s.x * l.y) / ll};
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nb * nb; e += 64) {
    const int i = e % nb, j = e / nb;
    A[(k + i) + (int64_t)(k + j) * lda] = X[i][j];
  }
}

// inv([[P, 0], [Q, R]]) = [[inv P, 0], [-inv R Q inv P, inv R]] on rows/cols
// [k, k+n), split at n1.
static fx_status trinv_rec(fx_ctx* ctx, Workspace* ws, hipStream_t st, z* A, int64_t lda, int k, int n, z* T) {
  if (n <= CB) {
    hipLaunchKernelGGL(k_trinv_diag, dim3(1), dim3(64), 0, st, A, lda, k, n);
    FX_LAUNCH_CHECK();
    return FX_OK;
  }
  int n1 = (n / 2 + CB - 1) / CB * CB;
  if (n1 >= n) n1 = n - CB;
  const int n2 = n - n1;
  FX_TRY(trinv_rec(ctx, ws, st, A, lda, k, n1, T));
  FX_TRY(trinv_rec(ctx, ws, st, A, lda, k + n1, n2, T));
  z* P = A + k + (int64_t)k * lda;
  z* Q = A + (k + n1) + (int64_t)k * lda;
  z* R = A + (k + n1) + (int64_t)(k + n1) * lda;
  // T = Q inv(P)   (n2 x n1), then Q = -inv(R) T
  FX_TRY(zgemm(ctx, ws, st, 0, 0, n2, n1, n1, z{1.0, 0.0}, Q, lda, P, lda, z{0.0, 0.0}, T, n2, 1, 0, 0, 0, 1));
  FX_TRY(zgemm(ctx, ws, st, 0, 0, n2, n1, n2, z{-1.0, 0.0}, R, lda, T, n2, z{0.0, 0.0}, Q, lda, 1, 0, 0, 0, 1));
  return FX_OK;
}

fx_status ztrinv(fx_ctx* ctx, Workspace* ws, hipStream_t st, int n, void* A, int64_t lda) {
  void* T = nullptr;
  FX_TRY(ws_get(ctx, ws, "trinv_T", sizeof(z) * (size_t)n * n, &T));
  return trinv_rec(ctx, ws, st, (z*)A, lda, 0, n, (z*)T);
}

fx_status zherm(hipStream_t st, int n, const void* M, int64_t ldm, void* H, void* Aneg, double* ex_dev) {
  hipLaunchKernelGGL(k_herm, dim3(std::min(((int64_t)n * n + 255) / 256, (int64_t)4096)), dim3(256), 0, st, n,
                     (const z*)M, ldm, (z*)H, (z*)Aneg);
  FX_LAUNCH_CHECK();
  if (ex_dev) {
    hipLaunchKernelGGL(k_half_trace, dim3(1), dim3(64), 0, st, n, (const z*)H, ex_dev);
    FX_LAUNCH_CHECK();
  }
  return FX_OK;
}

// conj-transpose copy: B (n x n) = A^H
__global__ void k_conj_transpose(int n, const z* __restrict__ A, int64_t lda, z* __restrict__ B, int64_t ldb) {
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    B[i + (int64_t)j * ldb] = zconj(A[j + (int64_t)i * lda]);
  }
}

fx_status zconj_transpose(hipStream_t st, int n, const void* A, int64_t lda, void* B, int64_t ldb) {
  hipLaunchKernelGGL(k_conj_transpose, dim3(std::min(((int64_t)n * n + 255) / 256, (int64_t)4096)), dim3(256), 0, st,
                     n, (const z*)A, lda, (z*)B, ldb);
  FX_LAUNCH_CHECK();
  return FX_OK;
}

}  // namespace fx
