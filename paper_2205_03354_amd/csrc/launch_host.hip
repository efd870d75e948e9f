// Routing of a sweep launch to the instantiation part that holds its kernel,
// and the block count (= partial-sum slots) of a sweep.
#include "launch.hpp"

namespace sc {

int sweep_blocks(const SweepLaunch& L) {
  const int R = L.ks->R;
  int blocks = 0;
  if (L.ks->dim == 2) {
    if (L.dtype == SC_F64) {
      SweepArgs<double> a{};
      geom2d<double, 128>(L, R, a, &blocks);
    } else {
      SweepArgs<float> a{};
      geom2d<float, 128>(L, R, a, &blocks);
    }
  } else {
    if (L.dtype == SC_F64) {
      SweepArgs<double> a{};
      geom3d<double, 256>(L, R, a, &blocks);
    } else {
      SweepArgs<float> a{};
      geom3d<float, 256>(L, R, a, &blocks);
    }
  }
  return blocks;
}

hipError_t launch_sweep(const SweepLaunch& L, hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  if (L.ks->dim == 2) {
    if (L.kind == K_APPLY) {
      e = L.dtype == SC_F64 ? part_apply2d_f64(L, st) : part_apply2d_f32(L, st);
    } else if (L.dtype == SC_F32) {
      e = part_solve2d_f32(L, st);
    } else {
      e = L.periodic ? part_solve2d_f64_periodic(L, st) : part_solve2d_f64_ring(L, st);
    }
  } else if (L.ks->dim == 3) {
    if (L.kind == K_APPLY) {
      e = part_apply3d(L, st);
    } else if (L.dtype == SC_F32) {
      e = part_solve3d_f32(L, st);
    } else {
      e = part_solve3d_f64(L, st);
    }
  }
  if (e == hipErrorInvalidValue)
    set_error("no kernel instance for kind %d, %s, %s, %dD pattern %d radius %d", L.kind,
              L.dtype == SC_F64 ? "f64" : "f32", L.periodic ? "periodic" : "ring", L.ks->dim, L.ks->pat,
              L.ks->R);
  return e;
}

}  // namespace sc
