// Pair enumeration of the specialised plane passes: which work plane of a
// batch holds the pair (jj, kk), and the order in which the plane-forward
// pass walks the planes.  Integer logic only, for host and device (FX_HD must
// be defined before inclusion), so that it can be checked on the CPU.
#pragma once
#include <cmath>

namespace fx {

// Pair (jj, kk) of work plane p of a batch.  A rectangular batch stores its
// pairs target-major (p = kk*nj + jj); a diagonal batch of a halved apply
// (tri != 0, the same orbitals on both sides) stores only jj <= kk, packed
// as p = kk*(kk+1)/2 + jj.
FX_HD void pair_of(int p, int nj, int tri, int* jj, int* kk) {
  if (!tri) {
    *kk = p / nj;
    *jj = p - *kk * nj;
    return;
  }
  int k = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
  while (k > 0 && k * (k + 1) / 2 > p) --k;
  while ((k + 1) * (k + 2) / 2 <= p) ++k;
  *kk = k;
  *jj = p - k * (k + 1) / 2;
}

FX_HD int plane_of(int jj, int kk, int nj, int tri) { return tri ? kk * (kk + 1) / 2 + jj : kk * nj + jj; }

// Work plane of traversal unit u (0 <= u < units) of the plane-forward pass.
// In the plain order u is the plane itself.  In the blocked order
// (rectangular batches, units = nj * nk) the units walk blocks of up to 4
// orbitals x 16 targets, the blocks of each row of 4 orbitals one target
// block after the other, so that the 64 workgroups an XCD runs at once, which
// take consecutive units at the same z, share 20 input planes instead of all
// the batch's orbital planes.  (Blocks of 4 x 32 measured the same at 96^3,
// 8 x 8 and 8 x 32 2.6-3% slower, 2 x 16, 2 x 32 and 16 x 4 6-7%, 1 x 32
// 27%.)  A bijection of [0, units) either way.
FX_HD int unit_plane(int u, int units, int nj, int tri, bool blocked) {
  if (tri || !blocked) return u;
  constexpr int BJ = 4, BK = 16;
  const int nk = units / nj;
  const int jb = u / (BJ * nk), r = u - jb * BJ * nk;
  const int bj = nj - jb * BJ < BJ ? nj - jb * BJ : BJ;
  const int kb = r / (BK * bj), w = r - kb * BK * bj;
  const int jj = jb * BJ + w % bj, kk = kb * BK + w / bj;
  return kk * nj + jj;
}

}  // namespace fx
