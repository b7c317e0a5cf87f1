// The pair enumeration of the specialised plane passes on the CPU: pair_of
// inverts plane_of for rectangular and diagonal (packed triangle) batches,
// and unit_plane is a bijection of [0, units) in the plain and the blocked
// order, the blocked order keeping each aligned run of 64 units within 4
// orbitals and 16 targets where the batch is whole blocks.  Prints
// "ok <cases>" on success.
#include <cstdio>
#include <vector>
#define FX_HD inline
#include "pair_order.hpp"

static int fails = 0;
#define CHECK(c, ...)                   \
  do {                                  \
    if (!(c)) {                         \
      if (fails < 20) {                 \
        std::printf("FAIL: " __VA_ARGS__); \
        std::printf("\n");              \
      }                                 \
      ++fails;                          \
    }                                   \
  } while (0)

int main() {
  long cases = 0;
  // rectangular batches
  for (int nj = 1; nj <= 80; ++nj)
    for (int nk = 1; nk <= 80; ++nk) {
      const int units = nj * nk;
      for (int kk = 0; kk < nk; ++kk)
        for (int jj = 0; jj < nj; ++jj) {
          int j2, k2;
          fx::pair_of(fx::plane_of(jj, kk, nj, 0), nj, 0, &j2, &k2);
          CHECK(j2 == jj && k2 == kk, "rect nj %d pair (%d, %d)", nj, jj, kk);
        }
      for (int blocked = 0; blocked < 2; ++blocked) {
        std::vector<int> seen(units, 0);
        for (int u = 0; u < units; ++u) {
          const int p = fx::unit_plane(u, units, nj, 0, blocked != 0);
          CHECK(p >= 0 && p < units, "unit_plane out of range nj %d nk %d u %d", nj, nk, u);
          if (p >= 0 && p < units) ++seen[p];
        }
        for (int p = 0; p < units; ++p) CHECK(seen[p] == 1, "plane %d of nj %d nk %d seen %d times", p, nj, nk, seen[p]);
        if (blocked && nj % 4 == 0 && nk % 16 == 0) {
          // whole blocks: each aligned run of 64 units is one block of 4 x 16
          for (int u0 = 0; u0 < units; u0 += 64) {
            int jlo = nj, jhi = -1, klo = nk, khi = -1;
            for (int u = u0; u < u0 + 64 && u < units; ++u) {
              int jj, kk;
              fx::pair_of(fx::unit_plane(u, units, nj, 0, true), nj, 0, &jj, &kk);
              jlo = jj < jlo ? jj : jlo;
              jhi = jj > jhi ? jj : jhi;
              klo = kk < klo ? kk : klo;
              khi = kk > khi ? kk : khi;
            }
            CHECK(jhi - jlo == 3 && khi - klo == 15, "block at %d of nj %d nk %d spans %d x %d", u0, nj, nk,
                  jhi - jlo + 1, khi - klo + 1);
          }
        }
        ++cases;
      }
    }
  // diagonal batches: planes 0 .. K(K+1)/2 - 1, up to K = 3000 (4.5M planes,
  // where the float square root of the inverse needs its integer correction)
  for (int K : {1, 2, 3, 7, 64, 433, 1024, 3000}) {
    int p = 0;
    for (int kk = 0; kk < K; ++kk)
      for (int jj = 0; jj <= kk; ++jj, ++p) {
        CHECK(fx::plane_of(jj, kk, K, 1) == p, "tri plane_of (%d, %d) != %d", jj, kk, p);
        int j2, k2;
        fx::pair_of(p, K, 1, &j2, &k2);
        CHECK(j2 == jj && k2 == kk, "tri plane %d -> (%d, %d), want (%d, %d)", p, j2, k2, jj, kk);
        CHECK(fx::unit_plane(p, p + 1, K, 1, true) == p, "tri unit_plane moved %d", p);
      }
    ++cases;
  }
  if (fails) {
    std::printf("%d failures\n", fails);
    return 1;
  }
  std::printf("ok %ld\n", cases);
  return 0;
}
