// Kernel instantiations, split into parts that compile in parallel. The
// build compiles this file once per part with -DSC_PART=<n>; each part
// defines one dispatcher over (pattern, radius) for a fixed kind, element
// type and boundary handling.
//
// Instantiated (pattern, radius) sets:
//   2D apply : CROSS 1,2  DIAMOND 2  CROSSBOX 4  BOX 1..4   (every stencil
//              of radius <= 4 has a kernel)
//   2D solve : CROSS 1,2  DIAMOND 2  CROSSBOX 4  BOX 1,2
//   3D apply : CROSS 1,2  DIAMOND 2  BOX 1,2                (radius <= 2)
//   3D solve : CROSS 1    DIAMOND 2  BOX 1
//   3D mirror-symmetric (wave-private DMA ring): apply CROSS 1,2 DIAMOND 2
//              BOX 1; solve CROSS 1 DIAMOND 2 BOX 1
//   CH right-hand side (the Laplacian): CROSS 1,2
//   variable coefficient (generic kernels): 2D scale DIAMOND 2 CROSS 2 BOX
//              2,3, accumulate CROSS 1,2 BOX 1; 3D scale DIAMOND 2 BOX 2,
//              accumulate CROSS 1 BOX 1
#include "launch.hpp"

#ifndef SC_PART
#error "SC_PART must be defined"
#endif

namespace sc {

#define SC_KEY2(P, RR, S) ((S) * 256 + (P) * 16 + (RR))
#define SC_CASE2(T, KIND, PER, P, RR, S) \
  case SC_KEY2(P, RR, S): return run2d<T, KIND, P, RR, PER, S>(L, st);
#define SC_CASE3(T, KIND, PER, P, RR) \
  case P * 16 + RR: return run3d<T, KIND, P, RR, PER, 256>(L, st);

// 2D plain apply: symmetric variants of the hot operators, generic kernels
// for every pattern (any stencil of radius <= 4 has a kernel).
#define SC_APPLY2D_SET(T, PER)                     \
  SC_CASE2(T, K_APPLY, PER, PAT_CROSS, 1, true)    \
  SC_CASE2(T, K_APPLY, PER, PAT_CROSS, 2, true)    \
  SC_CASE2(T, K_APPLY, PER, PAT_DIAMOND, 2, true)  \
  SC_CASE2(T, K_APPLY, PER, PAT_CROSSBOX, 4, true) \
  SC_CASE2(T, K_APPLY, PER, PAT_CROSS, 1, false)    \
  SC_CASE2(T, K_APPLY, PER, PAT_CROSS, 2, false)    \
  SC_CASE2(T, K_APPLY, PER, PAT_DIAMOND, 2, false)  \
  SC_CASE2(T, K_APPLY, PER, PAT_CROSSBOX, 4, false) \
  SC_CASE2(T, K_APPLY, PER, PAT_BOX, 1, false)      \
  SC_CASE2(T, K_APPLY, PER, PAT_BOX, 2, false)      \
  SC_CASE2(T, K_APPLY, PER, PAT_BOX, 3, false)      \
  SC_CASE2(T, K_APPLY, PER, PAT_BOX, 4, false)

// 2D solver sweeps: symmetric operators of the hot patterns, plus generic
// radius-1/2 boxes for any other (point-symmetric) operator.
#define SC_SOLVE2D_SET(T, KIND, PER)            \
  SC_CASE2(T, KIND, PER, PAT_CROSS, 1, true)    \
  SC_CASE2(T, KIND, PER, PAT_CROSS, 2, true)    \
  SC_CASE2(T, KIND, PER, PAT_DIAMOND, 2, true)  \
  SC_CASE2(T, KIND, PER, PAT_CROSSBOX, 4, true) \
  SC_CASE2(T, KIND, PER, PAT_BOX, 1, false)     \
  SC_CASE2(T, KIND, PER, PAT_BOX, 2, false)

#define SC_APPLY3D_SET(T, PER)              \
  SC_CASE3(T, K_APPLY, PER, PAT_CROSS, 1)   \
  SC_CASE3(T, K_APPLY, PER, PAT_CROSS, 2)   \
  SC_CASE3(T, K_APPLY, PER, PAT_DIAMOND, 2) \
  SC_CASE3(T, K_APPLY, PER, PAT_BOX, 1)     \
  SC_CASE3(T, K_APPLY, PER, PAT_BOX, 2)

#define SC_SOLVE3D_SET(T, KIND, PER)     \
  SC_CASE3(T, KIND, PER, PAT_CROSS, 1)   \
  SC_CASE3(T, KIND, PER, PAT_DIAMOND, 2) \
  SC_CASE3(T, KIND, PER, PAT_BOX, 1)

#define SC_KEY (L.ks->dim == 2 ? SC_KEY2(L.ks->pat, L.ks->R, L.ks->sym ? 1 : 0) : (L.ks->pat * 16 + L.ks->R))

// symmetric 3D sweep (mirror-symmetric stencils only)
#define SC_CASE3S(T, KIND, PER, P, RR) \
  case P * 16 + RR: return run3s<T, KIND, P, RR, PER>(L, st);
#define SC_APPLY3S_SET(T, PER)               \
  SC_CASE3S(T, K_APPLY, PER, PAT_CROSS, 1)   \
  SC_CASE3S(T, K_APPLY, PER, PAT_CROSS, 2)   \
  SC_CASE3S(T, K_APPLY, PER, PAT_DIAMOND, 2) \
  SC_CASE3S(T, K_APPLY, PER, PAT_BOX, 1)
#define SC_SOLVE3S_SET(T, KIND, PER)          \
  SC_CASE3S(T, KIND, PER, PAT_CROSS, 1)       \
  SC_CASE3S(T, KIND, PER, PAT_DIAMOND, 2)     \
  SC_CASE3S(T, KIND, PER, PAT_BOX, 1)

#if SC_PART == 0
hipError_t part_apply2d_f64(const SweepLaunch& L, hipStream_t st) {
  if (L.periodic) {
    switch (SC_KEY) { SC_APPLY2D_SET(double, true) default: break; }
  } else {
    switch (SC_KEY) { SC_APPLY2D_SET(double, false) default: break; }
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 1
hipError_t part_apply2d_f32(const SweepLaunch& L, hipStream_t st) {
  if (L.periodic) {
    switch (SC_KEY) { SC_APPLY2D_SET(float, true) default: break; }
  } else {
    switch (SC_KEY) { SC_APPLY2D_SET(float, false) default: break; }
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 2
// FP64 periodic solves: CG direction, residual, Cahn-Hilliard right-hand side
hipError_t part_solve2d_f64_periodic(const SweepLaunch& L, hipStream_t st) {
  switch (L.kind) {
    case K_CGDIR: switch (SC_KEY) { SC_SOLVE2D_SET(double, K_CGDIR, true) default: break; } break;
    case K_RESID: switch (SC_KEY) { SC_SOLVE2D_SET(double, K_RESID, true) default: break; } break;
    case K_CHRHS:
      switch (SC_KEY) {
        SC_CASE2(double, K_CHRHS, true, PAT_CROSS, 1, true)
        SC_CASE2(double, K_CHRHS, true, PAT_CROSS, 2, true)
        default: break;
      }
      break;
    default: break;
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 3
// FP64 ring solves: CG direction, residual, biharmonic right-hand side
hipError_t part_solve2d_f64_ring(const SweepLaunch& L, hipStream_t st) {
  switch (L.kind) {
    case K_CGDIR: switch (SC_KEY) { SC_SOLVE2D_SET(double, K_CGDIR, false) default: break; } break;
    case K_RESID: switch (SC_KEY) { SC_SOLVE2D_SET(double, K_RESID, false) default: break; } break;
    case K_BVPRHS: switch (SC_KEY) { SC_SOLVE2D_SET(double, K_BVPRHS, false) default: break; } break;
    default: break;
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 4
hipError_t part_solve2d_f32(const SweepLaunch& L, hipStream_t st) {
  if (L.kind != K_CGDIR) return hipErrorInvalidValue;
  if (L.periodic) {
    switch (SC_KEY) { SC_SOLVE2D_SET(float, K_CGDIR, true) default: break; }
  } else {
    switch (SC_KEY) { SC_SOLVE2D_SET(float, K_CGDIR, false) default: break; }
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 5
hipError_t part_apply3d(const SweepLaunch& L, hipStream_t st) {
  if (L.dtype == SC_F64) {
    if (L.periodic) { switch (SC_KEY) { SC_APPLY3D_SET(double, true) default: break; } }
    else { switch (SC_KEY) { SC_APPLY3D_SET(double, false) default: break; } }
  } else {
    if (L.periodic) { switch (SC_KEY) { SC_APPLY3D_SET(float, true) default: break; } }
    else { switch (SC_KEY) { SC_APPLY3D_SET(float, false) default: break; } }
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 6
hipError_t part_solve3d_f64(const SweepLaunch& L, hipStream_t st) {
  switch (L.kind) {
    case K_CGDIR:
      if (L.periodic) { switch (SC_KEY) { SC_SOLVE3D_SET(double, K_CGDIR, true) default: break; } }
      else { switch (SC_KEY) { SC_SOLVE3D_SET(double, K_CGDIR, false) default: break; } }
      break;
    case K_RESID:
      if (L.periodic) { switch (SC_KEY) { SC_SOLVE3D_SET(double, K_RESID, true) default: break; } }
      else { switch (SC_KEY) { SC_SOLVE3D_SET(double, K_RESID, false) default: break; } }
      break;
    case K_BVPRHS:
      if (!L.periodic) { switch (SC_KEY) { SC_SOLVE3D_SET(double, K_BVPRHS, false) default: break; } }
      break;
    case K_CHRHS:
      if (L.periodic) {
        switch (SC_KEY) {
          SC_CASE3(double, K_CHRHS, true, PAT_CROSS, 1)
          SC_CASE3(double, K_CHRHS, true, PAT_CROSS, 2)
          default: break;
        }
      }
      break;
    default: break;
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 7
hipError_t part_solve3d_f32(const SweepLaunch& L, hipStream_t st) {
  if (L.kind != K_CGDIR) return hipErrorInvalidValue;
  if (L.periodic) {
    switch (SC_KEY) { SC_SOLVE3D_SET(float, K_CGDIR, true) default: break; }
  } else {
    switch (SC_KEY) { SC_SOLVE3D_SET(float, K_CGDIR, false) default: break; }
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 8
hipError_t part_apply3s(const SweepLaunch& L, hipStream_t st) {
  if (L.kind != K_APPLY || !L.ks->sym) return hipErrorInvalidValue;
  if (L.dtype == SC_F64) {
    if (L.periodic) { switch (SC_KEY) { SC_APPLY3S_SET(double, true) default: break; } }
    else { switch (SC_KEY) { SC_APPLY3S_SET(double, false) default: break; } }
  } else {
    if (L.periodic) { switch (SC_KEY) { SC_APPLY3S_SET(float, true) default: break; } }
    else { switch (SC_KEY) { SC_APPLY3S_SET(float, false) default: break; } }
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 9
hipError_t part_solve3s_f64(const SweepLaunch& L, hipStream_t st) {
  if (!L.ks->sym) return hipErrorInvalidValue;
  switch (L.kind) {
    case K_CGDIR:
      if (L.periodic) { switch (SC_KEY) { SC_SOLVE3S_SET(double, K_CGDIR, true) default: break; } }
      else { switch (SC_KEY) { SC_SOLVE3S_SET(double, K_CGDIR, false) default: break; } }
      break;
    case K_RESID:
      if (L.periodic) { switch (SC_KEY) { SC_SOLVE3S_SET(double, K_RESID, true) default: break; } }
      else { switch (SC_KEY) { SC_SOLVE3S_SET(double, K_RESID, false) default: break; } }
      break;
    case K_BVPRHS:
      if (!L.periodic) { switch (SC_KEY) { SC_SOLVE3S_SET(double, K_BVPRHS, false) default: break; } }
      break;
    case K_CHRHS:
      if (L.periodic) {
        switch (SC_KEY) {
          SC_CASE3S(double, K_CHRHS, true, PAT_CROSS, 1)
          SC_CASE3S(double, K_CHRHS, true, PAT_CROSS, 2)
          default: break;
        }
      }
      break;
    default: break;
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 10
hipError_t part_solve3s_f32(const SweepLaunch& L, hipStream_t st) {
  if (L.kind != K_CGDIR || !L.ks->sym) return hipErrorInvalidValue;
  if (L.periodic) {
    switch (SC_KEY) { SC_SOLVE3S_SET(float, K_CGDIR, true) default: break; }
  } else {
    switch (SC_KEY) { SC_SOLVE3S_SET(float, K_CGDIR, false) default: break; }
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 11
// variable-coefficient applies: pointwise coefficient after the inner
// stencil (first derivative of a Laplacian: DIAMOND 2 / BOX 2,3), and the
// accumulating outer first derivative (CROSS 1, BOX 1)
#define SC_VC2D_SET(T, PER)                        \
  SC_CASE2(T, K_SCALE, PER, PAT_DIAMOND, 2, false) \
  SC_CASE2(T, K_SCALE, PER, PAT_CROSS, 2, false)   \
  SC_CASE2(T, K_SCALE, PER, PAT_BOX, 2, false)     \
  SC_CASE2(T, K_SCALE, PER, PAT_BOX, 3, false)     \
  SC_CASE2(T, K_SCALE, PER, PAT_CROSSBOX, 4, false) \
  SC_CASE2(T, K_ACCUM, PER, PAT_CROSS, 1, false)   \
  SC_CASE2(T, K_ACCUM, PER, PAT_CROSS, 2, false)   \
  SC_CASE2(T, K_ACCUM, PER, PAT_BOX, 1, false)
hipError_t part_varcoef2d(const SweepLaunch& L, hipStream_t st) {
  if (L.ks->sym) return hipErrorInvalidValue;
  const int key = SC_KEY2(L.ks->pat, L.ks->R, 0) + (L.kind == K_ACCUM ? 0x10000 : 0);
#define SC_VKEY(P, RR, K) (SC_KEY2(P, RR, 0) + ((K) == K_ACCUM ? 0x10000 : 0))
#undef SC_CASE2
#define SC_CASE2(T, KIND, PER, P, RR, S) \
  case SC_VKEY(P, RR, KIND): return run2d<T, KIND, P, RR, PER, S>(L, st);
  if (L.dtype == SC_F64) {
    if (L.periodic) { switch (key) { SC_VC2D_SET(double, true) default: break; } }
    else { switch (key) { SC_VC2D_SET(double, false) default: break; } }
  } else {
    if (L.periodic) { switch (key) { SC_VC2D_SET(float, true) default: break; } }
    else { switch (key) { SC_VC2D_SET(float, false) default: break; } }
  }
  return hipErrorInvalidValue;
}
#elif SC_PART == 12
#define SC_VKEY3(P, RR, K) ((P) * 16 + (RR) + ((K) == K_ACCUM ? 0x10000 : 0))
#define SC_VC3(T, KIND, PER, P, RR) \
  case SC_VKEY3(P, RR, KIND): return run3d<T, KIND, P, RR, PER, 256>(L, st);
#define SC_VC3D_SET(T, PER)                 \
  SC_VC3(T, K_SCALE, PER, PAT_DIAMOND, 2)   \
  SC_VC3(T, K_SCALE, PER, PAT_BOX, 2)       \
  SC_VC3(T, K_ACCUM, PER, PAT_CROSS, 1)     \
  SC_VC3(T, K_ACCUM, PER, PAT_BOX, 1)
hipError_t part_varcoef3d(const SweepLaunch& L, hipStream_t st) {
  if (L.ks->sym) return hipErrorInvalidValue;
  const int key = SC_VKEY3(L.ks->pat, L.ks->R, L.kind);
  if (L.dtype == SC_F64) {
    if (L.periodic) { switch (key) { SC_VC3D_SET(double, true) default: break; } }
    else { switch (key) { SC_VC3D_SET(double, false) default: break; } }
  } else {
    if (L.periodic) { switch (key) { SC_VC3D_SET(float, true) default: break; } }
    else { switch (key) { SC_VC3D_SET(float, false) default: break; } }
  }
  return hipErrorInvalidValue;
}
#else
#error "unknown SC_PART"
#endif

}  // namespace sc
