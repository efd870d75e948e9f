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
      geom2d<double>(L, R, a, &blocks, kMaxResidentWaves);
    } else {
      SweepArgs<float> a{};
      geom2d<float>(L, R, a, &blocks, kMaxResidentWaves);
    }
  } else {
    // the symmetric and the general 3D sweeps tile differently: size the
    // partial sums for whichever launches
    int b2 = 0;
    if (L.dtype == SC_F64) {
      SweepArgs<double> a{};
      geom3d<double, 256>(L, R, a, &blocks);
      geom3s<double, 2>(L, R, a, &b2, kMaxResidentWaves);
    } else {
      SweepArgs<float> a{};
      geom3d<float, 256>(L, R, a, &blocks);
      geom3s<float, 2>(L, R, a, &b2, kMaxResidentWaves);
    }
    blocks = blocks > b2 ? blocks : b2;
  }
  return blocks;
}

namespace {

hipError_t route(const SweepLaunch& L, hipStream_t st) {
  if (L.kind == K_SCALE || L.kind == K_ACCUM)
    return L.ks->dim == 2 ? part_varcoef2d(L, st) : part_varcoef3d(L, st);
  if (L.ks->dim == 2) {
    if (L.kind == K_APPLY) return L.dtype == SC_F64 ? part_apply2d_f64(L, st) : part_apply2d_f32(L, st);
    if (L.dtype == SC_F32) return part_solve2d_f32(L, st);
    return L.periodic ? part_solve2d_f64_periodic(L, st) : part_solve2d_f64_ring(L, st);
  }
  if (L.ks->dim == 3) {
    static const bool no3s = std::getenv("SCOMP_NO3S") != nullptr;  // A/B switch to the general kernel
    if (L.ks->sym && !no3s) {
      hipError_t e;
      if (L.kind == K_APPLY)
        e = part_apply3s(L, st);
      else
        e = L.dtype == SC_F32 ? part_solve3s_f32(L, st) : part_solve3s_f64(L, st);
      if (e != hipErrorInvalidValue) return e;
    }
    if (L.kind == K_APPLY) return part_apply3d(L, st);
    if (L.dtype == SC_F32) return part_solve3d_f32(L, st);
    return part_solve3d_f64(L, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace

// Try the stencil's own (pattern, symmetry) kernel, then the generic kernel
// of the same pattern, then the generic box of the same radius.
hipError_t launch_sweep(const SweepLaunch& L, hipStream_t st) {
  hipError_t e = route(L, st);
  if (e == hipErrorInvalidValue && L.ks->sym) {
    KStencil g = *L.ks;
    g.sym = false;
    SweepLaunch L2 = L;
    L2.ks = &g;
    e = route(L2, st);
  }
  if (e == hipErrorInvalidValue && L.ks->pat != PAT_BOX) {
    const KStencil b = to_box(*L.ks);
    SweepLaunch L3 = L;
    L3.ks = &b;
    e = route(L3, st);
  }
  if (e == hipErrorInvalidValue)
    set_error("no kernel instance for kind %d, %s, %s, %dD pattern %d radius %d", L.kind,
              L.dtype == SC_F64 ? "f64" : "f32", L.periodic ? "periodic" : "ring", L.ks->dim, L.ks->pat,
              L.ks->R);
  return e;
}

}  // namespace sc
