// Driver for the sanitized host build of the kernels' geometry: random primitives over the whole
// lattice range the kernels accept, every candidate-range voxel kind (inside, on a face, at the
// grid's edge), all four routines.  Exits 0 when the sanitizers found nothing.
#include <cstdio>
#include <cstdlib>
#include <random>
#include "geom.hpp"

int main(int argc, char** argv) {
  std::mt19937_64 rng(argc > 1 ? strtoull(argv[1], nullptr, 10) : 1);
  const long n = argc > 2 ? atol(argv[2]) : 100000;
  double sink = 0.0;
  for (long it = 0; it < n; ++it) {
    const int Sb = 3 + int(rng() % 18);                 // voxel size 2^3 .. 2^20 lattice units
    const int64_t s = int64_t(1) << Sb, R = int64_t(1) << (23 - Sb);
    const int64_t span = (it % 3 == 0) ? (int64_t(1) << 23) : s * (1 + int64_t(rng() % 4));
    int32_t r[16] = {0};
    const int64_t base = int64_t(rng() % (int64_t(3) << 23)) - (int64_t(1) << 23);   // [-2^23, 2^24)
    for (int k = 0; k < 9; ++k) {
      int64_t x = base + int64_t(rng() % uint64_t(span + 1)) - span / 2;
      if (x < -(int64_t(1) << 23)) x = -(int64_t(1) << 23);
      if (x > (int64_t(1) << 24)) x = int64_t(1) << 24;
      if (it % 5 == 1) x = (x / s) * s;                  // on voxel planes
      r[k] = int32_t(x);
    }
    int64_t v[3];
    bool any = true;
    for (int a = 0; a < 3; ++a) {
      int64_t mn = r[a], mx = r[a];
      for (int i = 1; i < 3; ++i) { mn = mn < r[3 * i + a] ? mn : r[3 * i + a]; mx = mx > r[3 * i + a] ? mx : r[3 * i + a]; }
      int64_t lo = -((-mn) >> Sb) - 1, hi = mx >> Sb;
      lo = lo < 0 ? 0 : lo;
      hi = hi > R - 1 ? R - 1 : hi;
      if (hi < lo) { any = false; break; }
      v[a] = lo + int64_t(rng() % uint64_t(hi - lo + 1));
    }
    if (!any) continue;
    sink += vx::tri_touch(r, v, s, Sb) ? 1.0 : 0.0;
    double a = vx::tri_area_bary(r, v, Sb);
    if (a < 0.0) a = vx::tri_area_exact(r, v[0], v[1], v[2], Sb);
    sink += a;
    const int64_t rho = 1 + int64_t(rng() % uint64_t(s));
    sink += vx::cap_touch(r, v, s, Sb, rho) ? 1.0 : 0.0;
    sink += double(vx::seg_length(r, v, Sb, 1.0f));
  }
  printf("ok %g\n", sink);
  return 0;
}
