// The three passes of one batch of pair Poisson solves (Eq. applyVX):
//
//   A  plane pass, one (pair, z) per workgroup: rho = conj(psi_j) phi_k on the
//      xy plane, forward FFT along x then y, written to the pair's work volume.
//   B  pencil pass, one (pair, y) per workgroup: the xz plane, forward FFT
//      along z, times K at the digit-reversed positions (the table already
//      carries -scale/Omega), inverse FFT along z, written back in place.
//   C  plane pass, one (target k, z) per workgroup, looping over the batch's
//      orbitals j in ascending order: inverse FFT along y then x, times psi_j,
//      added to the k-th output plane held in registers.
//
// Pass bodies are __host__ __device__ templates over a barrier policy, so the
// host can run them one thread at a time to check the plan and table logic.
#pragma once

#include "fft.hpp"

namespace fx {

struct PassGeom {
  int nx, ny, nz;
  int sx;  // LDS row stride (elements) of an xy plane; nx + pad
  AxisArg ax, ay, az;
  int hx, hy;  // folded kernel table dims nx/2+1, ny/2+1
};

// LDS elements a plane pass needs for its data (twiddles come after).
FX_HD int plane_lds_elems(const PassGeom& g) { return g.ny * g.sx; }
FX_HD int xz_lds_elems(const PassGeom& g) { return g.nz * g.nx; }

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

// Pass B body for the xz plane at (digit-reversed) y of one pair volume.
template <typename T, class Sync>
FX_HD void pass_b_body(cpx<T>* vol, int y, cpx<T>* s, const cpx<T>* twz, const T* kfold, const int* foldx,
                       const int* foldz, int fy, const PassGeom& g, int tid, int nthr, Sync sync) {
  const int nxz = g.nx * g.nz;
  for (int e = tid; e < nxz; e += nthr) {
    const int z = e / g.nx, x = e - z * g.nx;
    s[e] = vol[((size_t)z * g.ny + y) * g.nx + x];
  }
  sync();
  lds_fft<true, T>(s, g.az, g.nx, g.nx, 1, twz, tid, nthr, sync);
  for (int e = tid; e < nxz; e += nthr) {
    const int z = e / g.nx, x = e - z * g.nx;
    const T kv = kfold[((size_t)foldz[z] * g.hy + fy) * g.hx + foldx[x]];
    s[e] = cscale(s[e], kv);
  }
  sync();
  lds_fft<false, T>(s, g.az, g.nx, g.nx, 1, twz, tid, nthr, sync);
  for (int e = tid; e < nxz; e += nthr) {
    const int z = e / g.nx, x = e - z * g.nx;
    vol[((size_t)z * g.ny + y) * g.nx + x] = s[e];
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
