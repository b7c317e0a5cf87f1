// The three passes of one batch of pair Poisson solves (Eq. applyVX):
//
//   A  plane pass, one (pair, z) at a time: rho = conj(psi_j) phi_k on the xy
//      plane, forward FFT along x then y, written to the pair's work volume.
//   B  pencil pass, one (pair, y, x-tile): forward FFT along z, times K at the
//      digit-reversed positions (the table carries -scale/Omega), inverse FFT
//      along z, written back in place.
//   C  plane pass, one (target k, z), looping over the batch's orbitals j in
//      ascending order: inverse FFT along y then x, times psi_j, added to the
//      k-th output plane held in registers.
//
// The bodies here are __host__ __device__ templates over a barrier policy;
// the host runs them one thread at a time to check plans and tables, and the
// device kernels (vx.hip) use the same FFT cores with pipelined loads.
#pragma once

#include "fft.hpp"

namespace fx {

struct PassGeom {
  int nx, ny, nz;
  int sx;  // LDS row stride (elements) of an xy plane: nx, or nx + 1 when nx is even
  AxisArg ax, ay, az;
  int hx, hy, hz;  // folded kernel table dims n/2 + 1
};

// LDS elements an xy plane needs (twiddles come after).
FX_HD int plane_lds_elems(const PassGeom& g) { return g.ny * g.sx; }

// Pass A body.  psi_j / phi_k / out point at plane z (contiguous nx*ny).
template <typename T, class Sync>
FX_HD void pass_a_body(const cpx<T>* psi_j, const cpx<T>* phi_k, cpx<T>* out, cpx<T>* s, const cpx<T>* twx,
                       const cpx<T>* twy, const PassGeom& g, int tid, int nthr, Sync sync) {
  const int nxy = g.nx * g.ny;
  for (int e = tid; e < nxy; e += nthr) {
    const int y = e / g.nx, x = e - y * g.nx;
    s[y * g.sx + x] = cconjmul(psi_j[e], phi_k[e]);
  }
  sync();
  lds_fft<true, T>(s, g.ax, g.ny, 1, g.sx, twx, tid, nthr, sync);
  lds_fft<true, T>(s, g.ay, g.nx, g.sx, 1, twy, tid, nthr, sync);
  for (int e = tid; e < nxy; e += nthr) {
    const int y = e / g.nx, x = e - y * g.nx;
    out[e] = s[y * g.sx + x];
  }
}

// Factor of the z-convolution: K at (digit-reversed) z position pos and x
// column x0 + f of the tile, from the K slice of this y held in LDS.
template <typename T>
struct KSlice {
  const T* kl;       // hz x hx values at the tile's folded y
  const int* foldx;  // folded frequency of each x position
  const int* foldz;
  int x0, nx, hx;
  FX_HD T operator()(int pos, int f) const {
    int x = x0 + f;
    x = x < nx ? x : nx - 1;  // columns past the edge are discarded later
    return kl[foldz[pos] * hx + foldx[x]];
  }
};

// Pass B body for the x-tile [x0, x0 + xt) of the xz plane at (digit-reversed)
// y of one pair volume; s holds nz * xt values.
template <typename T, class Sync>
FX_HD void pass_b_body(cpx<T>* vol, int y, int x0, int xt, cpx<T>* s, const cpx<T>* twz, KSlice<T> kf,
                       const PassGeom& g, int tid, int nthr, Sync sync) {
  const int n = g.nz * xt;
  for (int e = tid; e < n; e += nthr) {
    const int z = e / xt, x = x0 + (e - z * xt);
    s[e] = x < g.nx ? vol[((size_t)z * g.ny + y) * g.nx + x] : cpx<T>{0, 0};
  }
  sync();
  lds_conv<T>(s, g.az, xt, xt, 1, twz, kf, tid, nthr, sync);
  for (int e = tid; e < n; e += nthr) {
    const int z = e / xt, x = x0 + (e - z * xt);
    if (x < g.nx) vol[((size_t)z * g.ny + y) * g.nx + x] = s[e];
  }
}

// Pass C transform part: plane (digit-reversed spectrum in y and x) -> real
// space, left in s with row stride sx.
template <typename T, class Sync>
FX_HD void pass_c_fft(const cpx<T>* plane, cpx<T>* s, const cpx<T>* twx, const cpx<T>* twy, const PassGeom& g, int tid,
                      int nthr, Sync sync) {
  const int nxy = g.nx * g.ny;
  for (int e = tid; e < nxy; e += nthr) {
    const int y = e / g.nx, x = e - y * g.nx;
    s[y * g.sx + x] = plane[e];
  }
  sync();
  lds_fft<false, T>(s, g.ay, g.nx, g.sx, 1, twy, tid, nthr, sync);
  lds_fft<false, T>(s, g.ax, g.ny, 1, g.sx, twx, tid, nthr, sync);
}

}  // namespace fx
