// Host build of the kernels' exact geometry (the device header compiled for the CPU), exported
// for tests/test_host_geometry.py, which checks it against the exact-rational brute force.
#include "geom.hpp"

extern "C" {
int hg_tri_touch(const int32_t* q9, const int64_t* v3, int Sb) {
  return vx::tri_touch(q9, v3, int64_t(1) << Sb, Sb) ? 1 : 0;
}
// the piece's area as a fraction of the whole triangle's (whole = 1)
double hg_tri_area_frac(const int32_t* q9, const int64_t* v3, int Sb) {
  double a = vx::tri_area_bary(q9, v3, Sb);
  if (a < 0.0) a = vx::tri_area_exact(q9, v3[0], v3[1], v3[2], Sb);
  return 2.0 * a;
}
int hg_cap_touch(const int32_t* r16, const int64_t* v3, int Sb, int64_t rho) {
  return vx::cap_touch(r16, v3, int64_t(1) << Sb, Sb, rho) ? 1 : 0;
}
double hg_seg_frac(const int32_t* r16, const int64_t* v3, int Sb) {
  return double(vx::seg_length(r16, v3, Sb, 1.0f));
}
}
