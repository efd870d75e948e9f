// Launch helpers shared by the kernel-instantiation translation units.
#pragma once

#include <cstdlib>

#include "internal.hpp"
#include "sweep3d.hpp"
#include "sweep3s.hpp"

namespace sc {

// Output rows (2D) per tile: aim at ~8192 one-wave tiles, about two rounds
// of the waves one MI355X keeps resident (16 per CU), so that the tiles in
// flight at any moment cover a compact band of rows, without making tiles so
// short that the 2R halo rows dominate.
inline int tile_rows_2d(int64_t n1, int64_t strips, int R, int64_t capacity) {
  if (const char* e = std::getenv("SCOMP_TY2D")) {
    const int v = std::atoi(e);
    if (v > 0) return v;
  }
  // as many tiles as the device holds waves of the kernel at once (one
  // round of waves), but tiles of at least max(4R, 12) rows (fewer halo
  // re-reads), unless tiles that tall would leave over half of those waves
  // idle: then max(2R, 4) rows (CH steps at 512^2 and 1024^2 21% and 10%
  // faster, 2048^2 unchanged)
  int64_t ty = (n1 * strips + capacity - 1) / capacity;
  int64_t lo = 4 * R > 12 ? 4 * R : 12;
  if (n1 * strips / lo < capacity / 2) lo = 2 * R > 4 ? 2 * R : 4;
  if (ty < lo) ty = lo;
  if (ty > n1) ty = n1;
  if (ty < 1) ty = 1;
  return (int)ty;
}

// Planes (3D) per tile.
inline int tile_planes_3d(int64_t n2, int64_t xy_tiles, int R) {
  if (const char* e = std::getenv("SCOMP_TZ3D")) {
    const int v = std::atoi(e);
    if (v > 0) return v;
  }
  int64_t tz = (n2 * xy_tiles + 1023) / 1024;
  const int64_t lo = 4 * R > 8 ? 4 * R : 8;
  if (tz < lo) tz = lo;
  if (tz > n2) tz = n2;
  if (tz < 1) tz = 1;
  return (int)tz;
}

template <typename T>
SweepArgs<T> make_args(const SweepLaunch& L) {
  SweepArgs<T> a{};
  a.in = static_cast<const T*>(L.in);
  a.in2 = static_cast<const T*>(L.in2);
  a.aux = static_cast<const T*>(L.aux);
  a.out = static_cast<T*>(L.out);
  a.out2 = static_cast<T*>(L.out2);
  a.pin = L.pin; a.pin2 = L.pin2; a.paux = L.paux; a.pout = L.pout; a.pout2 = L.pout2;
  a.zin = L.zin; a.zin2 = L.zin2; a.zaux = L.zaux; a.zout = L.zout; a.zout2 = L.zout2;
  a.n0 = L.n[0]; a.n1 = L.n[1]; a.n2 = L.n[2];
  a.scal = L.scal;
  a.partials = L.partials;
  a.c0 = L.c0; a.c1 = L.c1; a.c2 = L.c2; a.c3 = L.c3;
  a.flag = L.flag;
  a.fold = L.fold;
  a.fold_n = L.fold_n;
  a.vec_store = L.vec_store ? 1 : 0;
  a.in_aligned = L.in_aligned ? 1 : 0;
  a.alt = 0;
  const int R = L.ks ? L.ks->R : 0;
  a.xlo = L.x_range ? L.in_xlo : -R;
  a.xhi = L.x_range ? L.in_xhi : L.n[0] + R;
  a.axhi = L.x_range ? L.aux_xhi : L.n[0];
  return a;
}

template <typename T, int N>
Taps<T, N> make_taps(const KStencil& ks) {
  Taps<T, N> t{};
  for (int i = 0; i < N; ++i) t.w[i] = (T)ks.w[i];
  return t;
}

// Geometry of a 2D launch: one wave per tile, strips of 64 * VPL columns.
template <typename T>
inline void geom2d(const SweepLaunch& L, int R, SweepArgs<T>& a, int* blocks, int64_t capacity) {
  const int64_t TX = strip_width_2d<T>();
  const int64_t strips = (L.n[0] + TX - 1) / TX;
  a.ty = tile_rows_2d(L.n[1], strips, R, capacity);
  const int64_t ty = (L.n[1] + a.ty - 1) / a.ty;
  a.tiles_a = (int)strips;
  a.tiles_b = (int)ty;
  a.small = (L.n[0] < 2 * R + 8 || L.n[1] < 2 * R + 8) ? 1 : 0;
  *blocks = (int)(strips * ty);
}

template <typename T, int NT>
inline void geom3d(const SweepLaunch& L, int R, SweepArgs<T>& a, int* blocks) {
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int TX = 64;
  constexpr int TY = (NT / (TX / VEC)) * 2;
  const int64_t tx = (L.n[0] + TX - 1) / TX;
  const int64_t ty = (L.n[1] + TY - 1) / TY;
  a.tiles_x2 = (int)tx;
  a.tiles_a = (int)(tx * ty);
  a.ty = tile_planes_3d(L.n[2], tx * ty, R);
  a.tiles_b = (int)((L.n[2] + a.ty - 1) / a.ty);
  a.small = (L.n[0] < 2 * R + 8 || L.n[1] < 2 * R + 8 || L.n[2] < 2 * R + 8) ? 1 : 0;
  *blocks = a.tiles_a * a.tiles_b;
}

// Tile rows and plane look-ahead of the symmetric 3D sweep, by kind: the
// direction sweep holds two input rings, so it takes taller tiles (less
// y-halo re-reading per output) and a shallower look-ahead.
template <int KIND>
constexpr int tile3s_rows() { return KIND == K_CGDIR ? 4 : 2; }
template <int KIND>
constexpr int lookahead3s() { return KIND == K_CGDIR ? 2 : 3; }

// Geometry of the symmetric 3D sweep. Each wave streams a z chunk of one
// x-y tile; the chunk length is chosen so that all tiles are resident at
// once (`capacity` = waves the device holds for this kernel), which avoids a
// partial last round of waves, but no shorter than max(2R, 4) planes.
template <typename T, int TY>
inline void geom3s(const SweepLaunch& L, int R, SweepArgs<T>& a, int* blocks, int64_t capacity) {
  constexpr int VPL = 16 / (int)sizeof(T);
  constexpr int64_t TXW = 64 * VPL;
  const int RA = ((R + VPL - 1) / VPL) * VPL;
  const int64_t tx = (L.n[0] + TXW - 1) / TXW;
  const int64_t ty = (L.n[1] + TY - 1) / TY;
  const int64_t txy = tx * ty;
  int64_t chunks = capacity / txy;
  if (chunks < 1) chunks = 1;
  int64_t tz = (L.n[2] + chunks - 1) / chunks;
  const int64_t lo = 2 * R > 4 ? 2 * R : 4;
  if (const char* e = std::getenv("SCOMP_TZ3S")) {
    const int v = std::atoi(e);
    if (v > 0) tz = v;
  }
  if (tz < lo) tz = lo;
  if (tz > L.n[2]) tz = L.n[2];
  a.tiles_x2 = (int)tx;
  a.tiles_a = (int)txy;
  a.ty = (int)tz;
  a.tiles_b = (int)((L.n[2] + tz - 1) / tz);
  // a single wrap (wrap_once) covers every index the tile touches only when
  // the grid is wider than the tile plus its halo
  a.small = (L.n[0] <= TXW + RA || L.n[1] <= TY + R || L.n[2] <= R) ? 1 : 0;
  *blocks = a.tiles_a * a.tiles_b;
}
// Upper bound on the waves a device holds (partial-sum sizing).
constexpr int64_t kMaxResidentWaves = 8192;

// Class weights (|dx|, |dy|, |dz|) of a 3D mirror-symmetric stencil.
template <typename T, int PAT, int R>
Taps<T, sym3_nweights(R)> make_sym3_taps(const KStencil& ks) {
  Taps<T, sym3_nweights(R)> t{};
  for (int az = 0; az <= R; ++az)
    for (int b = 0; b <= R; ++b)
      for (int d = 0; d <= R; ++d)
        if (in_pattern(PAT, R, d, b, az)) t.w[sym3_index(R, d, b, az)] = (T)ks.w[tap_index(PAT, R, 3, d, b, az)];
  return t;
}

// Class weights (|dx|, |dy|) of a mirror-symmetric stencil.
template <typename T, int PAT, int R>
Taps<T, sym_num_classes(PAT, R)> make_sym_taps(const KStencil& ks) {
  Taps<T, sym_num_classes(PAT, R)> t{};
  for (int aa = 0; aa <= R; ++aa)
    for (int d = 0; d <= R; ++d)
      if (in_pattern(PAT, R, d, aa, 0)) t.w[sym_class_index(PAT, R, d, aa)] = (T)ks.w[tap_index(PAT, R, 2, d, aa, 0)];
  return t;
}

// The finish kernel of a sweep that reduces a dot product (after the sweep's
// own launch on the same stream). The direction sweep has none: the CG
// update that always follows it sums its partials into alpha.
template <int KIND>
hipError_t finish_sweep(const DevScalars* scal, const double* partials, int blocks, double c2, int flag,
                        hipStream_t st) {
  const hipError_t e = hipGetLastError();
  if constexpr (!kind_has_dot(KIND) || KIND == K_CGDIR) {
    return e;
  } else {
    if (e != hipSuccess) return e;
    FinArgs f;
    f.s = const_cast<DevScalars*>(scal);
    f.partials = partials;
    f.n = blocks;
    f.c = c2;
    f.flag = flag;
    const int fk = KIND == K_RESID ? FIN_RESID : FIN_RHS;
    return launch_finish(fk, f, st);
  }
}

// Waves of kernel `kern` (64-thread blocks) the device holds at once.
template <typename K>
int64_t resident_waves(K kern) {
  int per_cu = 0, cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, 0) != hipSuccess || per_cu < 1 || cus < 1)
    return 4096;
  const int64_t c = (int64_t)per_cu * cus;
  return c < kMaxResidentWaves ? c : kMaxResidentWaves;
}

template <typename T, int KIND, int PAT, int R, bool PER, bool SYM>
hipError_t run2d(const SweepLaunch& L, hipStream_t st) {
  const auto kern = sweep2d_kernel<T, KIND, PAT, R, PER, SYM>;
  static const int64_t capacity = resident_waves(kern);
  SweepArgs<T> a = make_args<T>(L);
  int blocks = 0;
  geom2d<T>(L, R, a, &blocks, capacity);
  a.alt = SYM ? 1 : 0;
  if (const char* e = std::getenv("SCOMP_NOALT"))
    if (e[0] == '1') a.alt = 0;
  if constexpr (SYM) {
    const auto taps = make_sym_taps<T, PAT, R>(*L.ks);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64), 0, st, a, taps);
  } else {
    const auto taps = make_taps<T, num_taps(PAT, R, 2)>(*L.ks);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64), 0, st, a, taps);
  }
  return finish_sweep<KIND>(a.scal, a.partials, blocks, a.c2, a.flag, st);
}

template <typename T, int KIND, int PAT, int R, bool PER, int NT>
hipError_t run3d(const SweepLaunch& L, hipStream_t st) {
  SweepArgs<T> a = make_args<T>(L);
  int blocks = 0;
  geom3d<T, NT>(L, R, a, &blocks);
  const auto taps = make_taps<T, num_taps(PAT, R, 3)>(*L.ks);
  hipLaunchKernelGGL((sweep3d_kernel<T, KIND, PAT, R, PER, NT>), dim3(blocks), dim3(NT), 0, st, a,
                     taps);
  return finish_sweep<KIND>(a.scal, a.partials, blocks, a.c2, a.flag, st);
}

template <typename T, int KIND, int PAT, int R, bool PER>
hipError_t run3s(const SweepLaunch& L, hipStream_t st) {
  constexpr int TY = tile3s_rows<KIND>();
  constexpr int D = lookahead3s<KIND>();
  const auto kern = sweep3s_kernel<T, KIND, PAT, R, PER, TY, D>;
  static const int64_t capacity = resident_waves(kern);  // LDS and registers
  SweepArgs<T> a = make_args<T>(L);
  int blocks = 0;
  geom3s<T, TY>(L, R, a, &blocks, capacity);
  const auto taps = make_sym3_taps<T, PAT, R>(*L.ks);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64), 0, st, a, taps);
  return finish_sweep<KIND>(a.scal, a.partials, blocks, a.c2, a.flag, st);
}

}  // namespace sc
