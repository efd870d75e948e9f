// Fused variable-coefficient composition on 2D grids (Sec. 2.2.3):
//   y = sum_t B_t(M * A_t(x)),
// one persistent kernel, no workspace. HBM sees x, M and y once each, plus
// the tiles' overlapping rings (mostly L2 hits), instead of two sweeps per
// term through a grid-sized workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "internal.hpp"

#ifndef VC_WAVES
#define VC_WAVES 4
#endif

namespace sc {

namespace {

// A tile's w = M * A_t(x) covers exactly kWX x kWY points: 64 columns (one
// per lane) and 20 rows (5 per wave, rows wave + 4 j). Its outputs are the
// (kWX - 2 RB) x (kWY - 2 RB) points whose outer stencils stay inside it.
constexpr int kWX = 64, kWY = 20;
constexpr int kNT = 256;
constexpr int kWSlots = kWY / 4;
constexpr int kMaxRA = kVcMaxRing - 1;  // RB >= 1
// x covers w plus a ring of RA; its LDS rows are kVcPitchX apart whatever RA
constexpr int kXW = kVcPitchX, kXH = kWY + 2 * kMaxRA;
constexpr int kXRowSlots = (kXH + 3) / 4, kXSideSlots = (2 * kMaxRA * kXH + kNT - 1) / kNT;
static_assert(kXW >= kWX + 2 * kMaxRA, "x rows hold 64 + 2 RA columns");
static_assert(kVcPitchW == kWX, "outer tap offsets use the w pitch");
// Output row slots past the tile's last output row and lanes past its last
// output column are still summed (and dropped): they read up to 2 RB rows
// below w and 2 RB columns past a row.
constexpr int kWPad = 2 * kVcMaxOuterR * kWX + 2 * kVcMaxOuterR;

// floor(i / d) for 0 <= i < 2^16 and 0 < d < 2^8, with mg = floor((2^32 - 1)
// / d) + 1: the product overshoots i / d by less than i d / 2^32 < 2^-8, which
// never reaches the next integer.
__device__ __forceinline__ int div_small(int i, unsigned mg) { return (int)__umulhi((unsigned)i, mg); }

// a + k n in [0, n): a tile reaches at most kWX + 2 kVcMaxRing past either
// edge, so the loops run once or twice unless the grid is narrower than a
// tile (grid sides are below 2^31, checked at launch)
__device__ __forceinline__ int wrapi(int a, int n) {
  while (a < 0) a += n;
  while (a >= n) a -= n;
  return a;
}

// The region of width 64 + 2 s and height h with corner (x0, y0) into the
// row slots vr (rows wave + 4 k, columns 0..63 by lane) and side slots vs
// (its last 2 s columns, flat over the workgroup) of this thread: wrapped
// (periodic) or read from the caller's ring, zero past it (the ring covers
// [-ring, n + ring) on both axes, and x0, y0 >= -ring). Rows are
// wave-uniform, so a row slot is a scalar row address plus a 32-bit lane
// offset. Issued together and consumed a tile later, so their latency hides
// behind a tile's work.
template <int NR, int NS, bool PER, typename T>
__device__ __forceinline__ void fetch(T (&vr)[NR], T (&vs)[NS], const T* __restrict__ src, int64_t pitch, int x0,
                                      int y0, int s, int h, unsigned mg2s, int ring, int n0, int n1) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int col = PER ? wrapi(x0 + lane, n0) : lane;
  const bool colok = PER || x0 + lane < n0 + ring;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int ly = wv + 4 * k;
    vr[k] = T(0);
    if (ly < h) {
      const int gy = PER ? wrapi(y0 + ly, n1) : y0 + ly;
      const T* row = src + (int64_t)gy * pitch + (PER ? 0 : x0);
      if (PER || (colok && gy < n1 + ring)) vr[k] = row[(unsigned)col];
    }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int i = (int)threadIdx.x + k * kNT;
    vs[k] = T(0);
    if (i < 2 * s * h) {
      const int ly = div_small(i, mg2s), lx = kWX + i - ly * 2 * s;
      const int gx = PER ? wrapi(x0 + lx, n0) : x0 + lx, gy = PER ? wrapi(y0 + ly, n1) : y0 + ly;
      if (PER || (gx < n0 + ring && gy < n1 + ring)) vs[k] = src[(int64_t)gy * pitch + gx];
    }
  }
}

// The tile a block takes in a given round, or -1 when it has none left.
// Blocks are dealt to the 8 XCDs in turn, so block b runs on XCD b % 8; the
// XCD owns the contiguous eighth of all tiles (row-major), which its G / 8
// blocks take in order, so the rings that vertically adjacent tiles share
// meet in one L2, a round or two apart.
__device__ __forceinline__ int tile_of(int round, int b, int G, int ntiles) {
  const int xcd = b % 8, per = G / 8;
  const int lo = (int)((int64_t)ntiles * xcd / 8), hi = (int)((int64_t)ntiles * (xcd + 1) / 8);
  const int q = lo + round * per + b / 8;
  return q < hi ? q : -1;
}

// One workgroup walks its tiles (tile_of). Per tile: x with a ring of
// RA + RB around the outputs goes to LDS, M stays in the registers of the
// threads that form w at its points, w = M * A_t(x) goes to LDS, and B_t(w)
// accumulates in registers; the next tile's x and M are in flight meanwhile.
// Tap loops are outermost, so a tap's offset and weight serve every row a
// wave owns, at immediate LDS offsets.
template <typename T, bool PER>
__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(VC_WAVES, VC_WAVES)))
varcoef_fused_kernel(const T* __restrict__ x, int64_t px,
                                                            const T* __restrict__ m, int64_t pm, T* __restrict__ y,
                                                            int64_t py, int n0, int n1, int tiles_x, int ntiles,
                                                            VcTerms<T> tm) {
  __shared__ T xs[kXH * kXW];
  __shared__ T ws[kWY * kWX + kWPad];
  const int RB = tm.RB, RA = tm.RA;
  const int TX = kWX - 2 * RB, TY = kWY - 2 * RB;  // outputs per tile
  const int XH = kWY + 2 * RA;
  const unsigned mgx = 0xFFFFFFFFu / (unsigned)(2 * RA) + 1u;
  const int G = (int)gridDim.x, b = (int)blockIdx.x;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  int round = 0, q = tile_of(0, b, G, ntiles);
  if (q < 0) return;
  T xr[kXRowSlots], xsd[kXSideSlots], mr[kWSlots], mc[kWSlots], none[1];
  {
    const int X0 = (q % tiles_x) * TX - RB, Y0 = (q / tiles_x) * TY - RB;  // w's corner
    fetch<kXRowSlots, kXSideSlots, PER>(xr, xsd, x, px, X0 - RA, Y0 - RA, RA, XH, mgx, RA + RB, n0, n1);
    fetch<kWSlots, 1, PER>(mr, none, m, pm, X0, Y0, 0, kWY, 1u, RB, n0, n1);
  }
  const T* xrow0 = xs + wv * kXW + lane + RA + RA * kXW;  // x at w row slot 0
  const T* wrow0 = ws + (wv + RB) * kWX + lane + RB;     // w at output row slot 0
  while (true) {
    const int OX = (q % tiles_x) * TX, OY = (q / tiles_x) * TY;  // first output
    __syncthreads();  // the previous tile's LDS reads are done
#pragma unroll
    for (int k = 0; k < kXRowSlots; ++k) {
      const int ly = wv + 4 * k;
      if (ly < XH) xs[ly * kXW + lane] = xr[k];
    }
#pragma unroll
    for (int k = 0; k < kXSideSlots; ++k) {
      const int i = (int)threadIdx.x + k * kNT;
      if (i < 2 * RA * XH) {
        const int ly = div_small(i, mgx);
        xs[ly * kXW + kWX + i - ly * 2 * RA] = xsd[k];
      }
    }
#pragma unroll
    for (int k = 0; k < kWSlots; ++k) mc[k] = mr[k];
    // the next tile of this block, prefetched across this tile's work
    const int qn = tile_of(++round, b, G, ntiles);
    if (qn >= 0) {
      const int X1 = (qn % tiles_x) * TX - RB, Y1 = (qn / tiles_x) * TY - RB;
      fetch<kXRowSlots, kXSideSlots, PER>(xr, xsd, x, px, X1 - RA, Y1 - RA, RA, XH, mgx, RA + RB, n0, n1);
      fetch<kWSlots, 1, PER>(mr, none, m, pm, X1, Y1, 0, kWY, 1u, RB, n0, n1);
    }
    // keep the prefetch ahead of this tile's work (the compiler would
    // otherwise sink the loads to their use, a tile later)
    asm volatile("" ::: "memory");
    T acc[kWSlots];
#pragma unroll
    for (int r = 0; r < kWSlots; ++r) acc[r] = T(0);
    for (int t = 0; t < tm.n; ++t) {
      __syncthreads();  // x staged; the previous term's w fully read
      const int na = tm.na[t];
      T s[kWSlots];
#pragma unroll
      for (int j = 0; j < kWSlots; ++j) s[j] = T(0);
      for (int k = 0; k < na; k += 4) {  // na is a multiple of 4
        // four taps' reads in flight together (the scheduler would
        // otherwise funnel them through one register pair)
        T v[4][kWSlots];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const T* p = xrow0 + tm.aoff[t][k + u];
#pragma unroll
          for (int j = 0; j < kWSlots; ++j) v[u][j] = p[4 * j * kXW];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const T w = tm.aw[t][k + u];
#pragma unroll
          for (int j = 0; j < kWSlots; ++j) s[j] = __builtin_fma(w, v[u][j], s[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < kWSlots; ++j) ws[(wv + 4 * j) * kWX + lane] = mc[j] * s[j];
      __syncthreads();
      const int nb = tm.nb[t];
      for (int k = 0; k < nb; k += 2) {  // nb is even
        T v[2][kWSlots];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const T* p = wrow0 + tm.boff[t][k + u];
#pragma unroll
          for (int r = 0; r < kWSlots; ++r) v[u][r] = p[4 * r * kWX];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const T w = tm.bw[t][k + u];
#pragma unroll
          for (int r = 0; r < kWSlots; ++r) acc[r] = __builtin_fma(w, v[u][r], acc[r]);
        }
      }
    }
    const int gx = OX + lane;
    if (lane < TX && gx < n0) {
#pragma unroll
      for (int r = 0; r < kWSlots; ++r) {
        const int gy = OY + wv + 4 * r;
        if (wv + 4 * r < TY && gy < n1) y[(int64_t)gy * py + gx] = acc[r];
      }
    }
    if (qn < 0) break;
    q = qn;
  }
}

template <typename T>
bool terms_ok(const VcTerms<T>& tm) {
  if (tm.n < 1 || tm.n > kVcMaxTerms || tm.RA < 1 || tm.RB < 1 || tm.RB > kVcMaxOuterR ||
      tm.RA + tm.RB > kVcMaxRing)
    return false;
  for (int t = 0; t < tm.n; ++t) {
    if (tm.na[t] < 0 || tm.na[t] > kVcMaxTapsA || tm.na[t] % 4 || tm.nb[t] < 0 || tm.nb[t] > kVcMaxTapsB ||
        tm.nb[t] % 2)
      return false;
    // every tap stays inside the RA (inner) or RB (outer) box around its point
    for (int k = 0; k < tm.na[t]; ++k) {
      const int o = tm.aoff[t][k] + tm.RA * kXW + tm.RA;
      const int oy = (o + kXW * 8) / kXW - 8, ox = o - oy * kXW;
      if (oy < 0 || oy > 2 * tm.RA || ox < 0 || ox > 2 * tm.RA) return false;
    }
    for (int k = 0; k < tm.nb[t]; ++k) {
      const int o = tm.boff[t][k] + tm.RB * kWX + tm.RB;
      const int oy = (o + kWX * 8) / kWX - 8, ox = o - oy * kWX;
      if (oy < 0 || oy > 2 * tm.RB || ox < 0 || ox > 2 * tm.RB) return false;
    }
  }
  return true;
}

// resident workgroups per CU times the CU count, once per device
template <typename T, bool PER>
int persistent_grid() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, varcoef_fused_kernel<T, PER>, kNT, 0) != hipSuccess)
    return 0;
  const int g = std::max(8, cus * std::max(1, per_cu) / 8 * 8);
  cache[dev] = g;
  return g;
}

template <typename T, bool PER>
hipError_t launch_t(const void* x, int64_t px, const void* m, int64_t pm, void* y, int64_t py, int64_t n0,
                    int64_t n1, const VcTerms<T>& tm, hipStream_t st) {
  const int64_t TX = kWX - 2 * tm.RB, TY = kWY - 2 * tm.RB;
  const int64_t tiles_x = (n0 + TX - 1) / TX, ntiles = tiles_x * ((n1 + TY - 1) / TY);
  if (n0 + 2 * kWX >= INT32_MAX || n1 + 2 * kWX >= INT32_MAX || ntiles + 8 * 4096 >= INT32_MAX)
    return hipErrorInvalidValue;
  const int cap = persistent_grid<T, PER>();
  if (cap <= 0) return hipErrorInvalidValue;
  // a multiple of 8 blocks (whole rounds per XCD), at most the tile count
  // rounded up to 8
  const int64_t g = std::min<int64_t>(cap, (ntiles + 7) / 8 * 8);
  hipLaunchKernelGGL((varcoef_fused_kernel<T, PER>), dim3((unsigned)g), dim3(kNT), 0, st,
                     static_cast<const T*>(x), px, static_cast<const T*>(m), pm, static_cast<T*>(y), py, (int)n0,
                     (int)n1, (int)tiles_x, (int)ntiles, tm);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_t(const void* x, int64_t px, const void* m, int64_t pm, void* y, int64_t py, int64_t n0,
                    int64_t n1, bool periodic, const void* terms, hipStream_t st) {
  const VcTerms<T>& tm = *static_cast<const VcTerms<T>*>(terms);
  if (!terms_ok(tm) || n0 < 1 || n1 < 1) return hipErrorInvalidValue;
  return periodic ? launch_t<T, true>(x, px, m, pm, y, py, n0, n1, tm, st)
                  : launch_t<T, false>(x, px, m, pm, y, py, n0, n1, tm, st);
}

}  // namespace

hipError_t launch_varcoef_fused(int dtype, const void* x, int64_t px, const void* m, int64_t pm, void* y, int64_t py,
                                int64_t n0, int64_t n1, bool periodic, const void* terms, hipStream_t st) {
  return dtype == SC_F64 ? launch_t<double>(x, px, m, pm, y, py, n0, n1, periodic, terms, st)
                         : launch_t<float>(x, px, m, pm, y, py, n0, n1, periodic, terms, st);
}

}  // namespace sc
