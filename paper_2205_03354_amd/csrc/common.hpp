// Shared definitions of the gfx950 stencil-composition library: tap
// patterns, kernel-side weight packs, device scalars of the Krylov solves
// and the deterministic two-kernel grid reduction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace sc {

// ---------------------------------------------------------------------------
// Tap patterns. A kernel is specialised for a pattern P and radius R; the
// taps it evaluates are the offsets of the (2R+1)^d box admitted by the
// pattern, enumerated z-major, then y, then x ascending. A composed stencil
// is run by the smallest instantiated pattern that contains all its offsets;
// missing taps get weight 0.
//   CROSS    : on an axis, |d| <= R                 (5/7-point Laplacians,
//                                                    the 9-point fourth-order cross)
//   DIAMOND  : |dx|+|dy|+|dz| <= R                  (Laplacian o Laplacian:
//                                                    13-point 2D, 25-point 3D)
//   CROSSBOX : on an axis with |d| <= R, or at most two non-zero components
//              each <= R/2                          (fourth-order cross composed
//                                                    with itself: 33-point 2D)
//   BOX      : the full box                          (any stencil of radius R)
// ---------------------------------------------------------------------------
enum Pattern : int { PAT_CROSS = 0, PAT_DIAMOND = 1, PAT_CROSSBOX = 2, PAT_BOX = 3 };

__host__ __device__ constexpr int iabs(int v) { return v < 0 ? -v : v; }
__host__ __device__ constexpr int imax(int a, int b) { return a > b ? a : b; }

__host__ __device__ constexpr bool in_pattern(int pat, int R, int dx, int dy, int dz) {
  const int ax = iabs(dx), ay = iabs(dy), az = iabs(dz);
  const int nz = (ax > 0) + (ay > 0) + (az > 0);
  const int mx = imax(ax, imax(ay, az));
  if (mx > R) return false;
  switch (pat) {
    case PAT_CROSS: return nz <= 1;
    case PAT_DIAMOND: return ax + ay + az <= R;
    case PAT_CROSSBOX: return nz <= 1 || (nz <= 2 && mx <= R / 2);
    default: return true;
  }
}

// Index of tap (dx,dy,dz) in the enumeration of pattern (pat, R) in `dim`
// dimensions, or -1 if the offset is not part of the pattern.
__host__ __device__ constexpr int tap_index(int pat, int R, int dim, int dx, int dy, int dz) {
  int idx = 0;
  const int zr = dim == 3 ? R : 0;
  for (int z = -zr; z <= zr; ++z)
    for (int y = -R; y <= R; ++y)
      for (int x = -R; x <= R; ++x) {
        if (!in_pattern(pat, R, x, y, z)) continue;
        if (x == dx && y == dy && z == dz) return idx;
        ++idx;
      }
  return -1;
}

__host__ __device__ constexpr int num_taps(int pat, int R, int dim) {
  int n = 0;
  const int zr = dim == 3 ? R : 0;
  for (int z = -zr; z <= zr; ++z)
    for (int y = -R; y <= R; ++y)
      for (int x = -R; x <= R; ++x) n += in_pattern(pat, R, x, y, z) ? 1 : 0;
  return n;
}

// Operations that apply a stencil in one sweep (see sweep2d.hpp).
enum SweepKind : int {
  K_APPLY = 0,    // out = S in
  K_CGDIR = 1,    // p = r + beta p_old ; q = S p ; <p, q>  -> alpha
  K_RESID = 2,    // r = b - S x ; <r, r>                   -> rr_true (and a CG (re)start)
  K_BVPRHS = 3,   // b = f - S g_ring ; <b, b>              -> bb, rr_stop
  K_CHRHS = 4,    // rhs = c3 u + c0 S(u^3 - c1 u) ; <rhs, rhs> -> bb, rr_stop
  K_SCALE = 5,    // out = aux * S in   (pointwise coefficient after a stencil)
  K_ACCUM = 6     // out = aux + S in   (aux may be out itself: accumulate)
};

// Kinds that reduce a dot product into DevScalars.
__host__ __device__ constexpr bool kind_has_dot(int kind) {
  return kind == K_CGDIR || kind == K_RESID || kind == K_BVPRHS || kind == K_CHRHS;
}
// Kinds that read `aux` at the output point.
__host__ __device__ constexpr bool kind_reads_aux(int kind) {
  return kind == K_RESID || kind == K_BVPRHS || kind == K_SCALE || kind == K_ACCUM;
}

// Weights of one pattern instance, passed by value as a kernel argument (so
// they live in scalar registers / the kernel-argument segment, with no
// device allocation).
template <typename T, int N>
struct Taps {
  T w[N];
};

// Device scalars of one Krylov solve, written by the one-block finish
// kernels and by thread 0 of block 0 of the CG update and of a direction
// sweep that folds the update's finish in (kernels of one solve are
// serialised on its stream; no kernel reads a field it writes).
struct alignas(64) DevScalars {
  double rr;        // <r, r> of the current recurrence residual
  double pq;        // <p, A p>
  double alpha;     // rr / pq
  double beta;      // rr_new / rr (0 right after a (re)start)
  double rr_stop;   // stop when rr <= rr_stop
  double bb;        // <b, b>
  double rr_true;   // <b - A x, b - A x> of the last residual sweep
  double scale;     // refinement scale s = ||r||
  long long iter;   // iterations performed
  int done;         // 0 running, 1 recurrence converged, 2 breakdown
  int slots;        // partial sums written by the last direction sweep
  double rz;        // preconditioned CG: <r, M^-1 r>
  double rr_prev;   // the rr the last CG update formed alpha with
  double pad[3];
};

// ---------------------------------------------------------------------------
// Compile-time loop helper: f(std::integral_constant<int, I>) for I in [B, E).
// ---------------------------------------------------------------------------
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(static_cast<F&&>(f));
  }
}

__host__ __device__ constexpr int pmod_c(int a, int n) { return ((a % n) + n) % n; }

// Blocks of a launch are dealt round-robin to the 8 XCDs of the MI355X
// (block b runs on XCD b % 8). Remap so that each XCD receives one
// contiguous range of logical tiles: neighbouring tiles, which share halo
// rows/planes, then hit the same XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  constexpr int NX = 8;
  const int q = nb / NX, r = nb % NX;
  const int x = b % NX, i = b / NX;
  return x * q + (x < r ? x : r) + i;
}

// Sum over the block (deterministic tree order); the result is valid in
// thread 0. NT must be a multiple of 64.
template <int NT>
__device__ __forceinline__ double block_sum(double v) {
  static_assert(NT % 64 == 0, "block must be whole waves");
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if constexpr (NT == 64) {
    return v;
  } else {
    __shared__ double red[NT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) t += red[w];
    }
    return t;
  }
}

// Deterministic two-kernel grid reduction. The reducing kernel stores one
// partial sum per block under `slot` (the logical tile, fixed by the data it
// covers, not by the scheduling order); a one-block finish kernel launched
// after it on the same stream (the kernel boundary makes the partials
// visible) sums them in slot order and finalises into DevScalars. A
// single-pass scheme where the last block to arrive finishes needs a
// device-scope release per block, and those serialise: about 25 ns per block
// on this part, 20-100 us for the grids here.
template <int NT>
__device__ __forceinline__ void block_partial(double v, int slot, double* partials) {
  const double bs = block_sum<NT>(v);
  if (threadIdx.x == 0) partials[slot] = bs;
}

// Sum of partials[0 .. n) in a fixed order; valid in thread 0.
template <int NT>
__device__ __forceinline__ double sum_partials(const double* partials, int n) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += partials[i];
  return block_sum<NT>(s);
}

// Threads of the finish kernel (elementwise.hip): its block of partial sums.
constexpr int kFinNT = 256;
// Partial slots a folding sweep loads at once (the CG update writes at most
// this many).
constexpr int kFoldSlots = 1024;

// The update finish (FIN_UPDATE: iteration count, stop test, beta, rr)
// folded into the direction sweep that follows the update: every block of
// NT threads forms the total of the update's <r, r> partials in the finish
// kernel's order (kFinNT threads striding the slots, each wave's butterfly,
// the waves added in order), so beta and the stop test are bit for bit the
// finish kernel's; thread 0 of block 0 records them. Returns false once the
// recurrence has converged (the sweep then has nothing to do).
template <int NT>
__device__ __forceinline__ bool fold_update(DevScalars* s, const double* partials, int n, double* beta) {
  double t = 0.0;
  if constexpr (NT == 64) {
    // lane l plays finish thread w 64 + l for each wave w; the first
    // kFoldSlots slots are loaded in one go (one memory latency), any
    // further ones after them, in the same per-thread order
    constexpr int W = kFinNT / 64;
    double v[W];
#pragma unroll
    for (int w = 0; w < W; ++w) v[w] = 0.0;
#pragma unroll
    for (int k = 0; k < kFoldSlots / kFinNT; ++k) {
      double x[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int i = k * kFinNT + w * 64 + (int)threadIdx.x;
        x[w] = i < n ? partials[i] : 0.0;
      }
#pragma unroll
      for (int w = 0; w < W; ++w)
        if (k * kFinNT + w * 64 + (int)threadIdx.x < n) v[w] += x[w];
    }
    for (int base = kFoldSlots; base < n; base += kFinNT) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int i = base + w * 64 + (int)threadIdx.x;
        if (i < n) v[w] += partials[i];
      }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v[w] += __shfl_xor(v[w], off, 64);
      t += v[w];
    }
  } else {
    static_assert(NT == kFinNT, "a folding sweep runs 64 or kFinNT threads");
    __shared__ double tot;
    const double v = sum_partials<NT>(partials, n);
    if (threadIdx.x == 0) tot = v;
    __syncthreads();
    t = tot;
  }
  const double rr_old = s->rr_prev;
  const bool stop = t <= s->rr_stop;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s->iter += 1;
    if (stop) s->done = 1;
    s->beta = t / rr_old;
    s->rr = t;
  }
  *beta = t / rr_old;
  return !stop;
}

// What the finish kernel does with the total.
// (The direction sweep's <p, Ap> has no finish kernel: the CG update that
// follows it sums those partials itself.)
enum FinKind : int {
  FIN_RESID = 1,   // rr_true (flag: also restart the recurrence: rr, beta, done)
  FIN_RHS = 2,     // bb; rr_stop = c bb
  FIN_UPDATE = 3,  // iteration count, convergence, beta, rr
  FIN_IR = 4,      // FP32 stretch start (flag: keep the direction); c = inner tol^2
  FIN_PCDOT = 5    // rz; beta = rz / rz_old (flag: restart, beta = 0)
};

struct FinArgs {
  DevScalars* s = nullptr;
  const DevScalars* s64 = nullptr;  // FIN_IR: the FP64 scalars (rr_true)
  const double* partials = nullptr;
  int n = 0;           // partial slots
  double c = 0.0;
  int flag = 0;
  int skip_if_done = 0;  // the reducing kernel returned early once s->done was set
};

}  // namespace sc
