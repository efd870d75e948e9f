// Matrix-free stencil sweep over a 2D grid for gfx950 (wave64, LDS).
//
// One kernel template serves every operation that applies a stencil: the
// plain apply, the CG direction sweep, the true residual and the right-hand
// sides of the biharmonic and Cahn-Hilliard problems. They differ only in
// what is fed to the stencil at each input point (`load`) and what is done
// with the stencil value at each output point (`store`).
//
// Work decomposition (one block = one tile of TX columns x TY rows):
//  * Each thread owns VEC = 16 B / sizeof(T) adjacent output columns.
//  * Input rows are streamed top to bottom in batches of B = 2R+1 rows. A
//    batch is staged in LDS with R (rounded up to VEC) halo columns on each
//    side; the next batch's global loads are issued before the current batch
//    is computed, so HBM latency hides behind the arithmetic.
//  * "Push" accumulation along y: an input row contributes to the 2R+1
//    output rows it is a neighbour of, whose partial sums live in a register
//    ring indexed at compile time (the batch length equals the ring length).
//    Each input value is read from HBM once (plus the tile halo) and from
//    LDS (VEC + 2R)/VEC times, as 16-byte conflict-free ds_read_b128.
//  * An output row is complete R rows after its own input row and is then
//    written once, coalesced.
#pragma once

#include "common.hpp"

namespace sc {

// Kernel arguments. Pointers address interior element (0,0[,0]); rings are
// reached with negative indices. p* are row pitches, z* plane pitches
// (elements).
template <typename T>
struct SweepArgs {
  const T* in;    // stencil input (x, r, g, u)
  const T* in2;   // K_CGDIR: p_old
  const T* aux;   // K_RESID / K_BVPRHS: b / f read at the output point
  T* out;         // apply result, p_new, r, b, rhs
  T* out2;        // K_CGDIR: q
  int64_t pin, pin2, paux, pout, pout2;
  int64_t zin, zin2, zaux, zout, zout2;
  int64_t n0, n1, n2;
  int ty;                 // output rows (2D) / planes (3D) per tile
  int tiles_a, tiles_b;   // tile grid: 2D (x, y); 3D (xy tiles, z chunks)
  int tiles_x2;           // 3D: tiles along x
  int small;              // periodic wrap needs a true modulo (grid < radius)
  int vec_store;          // outputs 16-byte aligned for the vector store
  DevScalars* scal;
  double* partials;
  double c0, c1, c2;      // K_CHRHS: dt, 1+S; K_BVPRHS/K_CHRHS: c2 = tol^2
  int flag;               // K_RESID: 1 = also (re)start the CG recurrence
};

template <typename T, int VEC>
struct VecT;
template <>
struct VecT<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <>
struct VecT<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };

__device__ __forceinline__ int64_t wrap_small(int64_t a, int64_t n) {
  int64_t r = a % n;
  return r < 0 ? r + n : r;
}
__device__ __forceinline__ int64_t wrap_once(int64_t a, int64_t n) {
  return a < 0 ? a + n : (a >= n ? a - n : a);
}

// Finalisers run by the last block of a reduction (thread 0).
template <int KIND>
__device__ __forceinline__ void finalize(DevScalars* s, double total, double tol2, int flag) {
  if constexpr (KIND == K_CGDIR) {
    s->pq = total;
    if (!(total > 0.0) || !__builtin_isfinite(total)) {
      s->done = 2;
    } else {
      s->alpha = s->rr / total;
    }
  } else if constexpr (KIND == K_RESID) {
    s->rr_true = total;
    if (flag) {
      s->rr = total;
      s->beta = 0.0;
      s->done = (total <= s->rr_stop) ? 1 : 0;
    }
  } else if constexpr (KIND == K_BVPRHS || KIND == K_CHRHS) {
    s->bb = total;
    s->rr_stop = tol2 * total;
  }
}

template <typename T, int KIND, int PAT, int R, bool PERIODIC, int NT>
__global__ void __launch_bounds__(NT)
    sweep2d_kernel(const SweepArgs<T> a, const Taps<T, num_taps(PAT, R, 2)> w) {
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int TX = NT * VEC;
  constexpr int RA = ((R + VEC - 1) / VEC) * VEC;
  constexpr int W = TX + 2 * RA;
  constexpr int B = 2 * R + 1;
  constexpr int LPR = (W + NT - 1) / NT;
  constexpr int NV = (RA + R + VEC) / VEC + ((RA + R + VEC) % VEC ? 1 : 0);
  constexpr bool HAS_DOT = KIND != K_APPLY;
  using V = typename VecT<T, VEC>::type;
  static_assert((NV - 1) * VEC <= 2 * RA, "window reads must stay inside the LDS row");

  __shared__ __attribute__((aligned(16))) T lds[B * W];

  if constexpr (KIND == K_CGDIR) {
    if (a.scal->done) return;
  }
  const T beta = (KIND == K_CGDIR) ? (T)a.scal->beta : T(0);
  const T c1 = (T)a.c1;

  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int txi = tile / a.tiles_b;
  const int tyi = tile - txi * a.tiles_b;
  const int64_t x0 = (int64_t)txi * TX;
  const int64_t y0 = (int64_t)tyi * a.ty;
  const int rows = (int)((a.n1 - y0) < a.ty ? (a.n1 - y0) : a.ty);
  const int NR = rows + 2 * R;
  const int nb = (NR + B - 1) / B;
  const int l = (int)threadIdx.x;

  // Columns this thread stages into LDS (fixed for the whole tile).
  int64_t gcol[LPR];
  bool gok[LPR];
#pragma unroll
  for (int k = 0; k < LPR; ++k) {
    const int c = l + k * NT;
    int64_t gx = x0 - RA + c;
    gok[k] = (c < W) && (gx >= -R) && (gx < a.n0 + R);
    if constexpr (PERIODIC) gx = a.small ? wrap_small(gx, a.n0) : wrap_once(gx, a.n0);
    gcol[k] = gx;
  }

  auto fetch = [&](int64_t gy_raw, int64_t gx, bool interior) -> T {
    int64_t gy = gy_raw;
    if constexpr (PERIODIC) gy = a.small ? wrap_small(gy, a.n1) : wrap_once(gy, a.n1);
    const T v = a.in[gy * a.pin + gx];
    if constexpr (KIND == K_CGDIR) {
      return v + beta * a.in2[gy * a.pin2 + gx];
    } else if constexpr (KIND == K_BVPRHS) {
      return interior ? T(0) : v;
    } else if constexpr (KIND == K_CHRHS) {
      return v * v * v - c1 * v;
    } else {
      return v;
    }
  };

  T pre[B][LPR];
  auto load_batch = [&](int b) {
    static_for<0, B>([&](auto s_) {
      constexpr int s = decltype(s_)::value;
      const int q = b * B + s;
      if (q < NR) {
        const int64_t gy = y0 - R + q;
        const bool row_in = (gy >= 0) && (gy < a.n1);
#pragma unroll
        for (int k = 0; k < LPR; ++k) {
          if (gok[k]) {
            const bool interior = row_in && (x0 - RA + l + k * NT) >= 0 && (x0 - RA + l + k * NT) < a.n0;
            pre[s][k] = fetch(gy, gcol[k], interior);
          } else {
            pre[s][k] = T(0);
          }
        }
      }
    });
  };

  T acc[B][VEC];
  T cen[B][VEC];
#pragma unroll
  for (int s = 0; s < B; ++s)
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[s][v] = T(0);
  double dot = 0.0;

  const int64_t mycol = x0 + (int64_t)l * VEC;
  const bool full_vec = a.vec_store && (mycol + VEC <= a.n0);

  auto emit = [&](int64_t gy, const T* accv, const T* cenv) {
    if constexpr (KIND == K_APPLY) {
      T* o = a.out + gy * a.pout + mycol;
      if (full_vec) {
        V t;
#pragma unroll
        for (int v = 0; v < VEC; ++v) t[v] = accv[v];
        __builtin_nontemporal_store(t, reinterpret_cast<V*>(o));
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          if (mycol + v < a.n0) o[v] = accv[v];
      }
    } else {
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int64_t col = mycol + v;
        if (col < a.n0) {
          if constexpr (KIND == K_CGDIR) {
            a.out[gy * a.pout + col] = cenv[v];
            a.out2[gy * a.pout2 + col] = accv[v];
            dot += (double)cenv[v] * (double)accv[v];
          } else if constexpr (KIND == K_RESID || KIND == K_BVPRHS) {
            const T r = a.aux[gy * a.paux + col] - accv[v];
            a.out[gy * a.pout + col] = r;
            dot += (double)r * (double)r;
          } else if constexpr (KIND == K_CHRHS) {
            const T r = a.in[gy * a.pin + col] + (T)a.c0 * accv[v];
            a.out[gy * a.pout + col] = r;
            dot += (double)r * (double)r;
          }
        }
      }
    }
  };

  load_batch(0);
  for (int b = 0; b < nb; ++b) {
    __syncthreads();
    static_for<0, B>([&](auto s_) {
      constexpr int s = decltype(s_)::value;
#pragma unroll
      for (int k = 0; k < LPR; ++k) {
        const int c = l + k * NT;
        if (k < LPR - 1 || c < W) lds[s * W + c] = pre[s][k];
      }
    });
    __syncthreads();
    if (b + 1 < nb) load_batch(b + 1);

    static_for<0, B>([&](auto s_) {
      constexpr int s = decltype(s_)::value;
      const int q = b * B + s;
      if (q < NR) {
        // Window of input values: win[j] is column mycol - RA + j.
        T win[NV * VEC];
        const V* rowv = reinterpret_cast<const V*>(lds + s * W) + l;
#pragma unroll
        for (int kv = 0; kv < NV; ++kv) {
          const V t = rowv[kv];
#pragma unroll
          for (int e = 0; e < VEC; ++e) win[kv * VEC + e] = t[e];
        }
        static_for<0, B>([&](auto d_) {
          constexpr int dy = decltype(d_)::value - R;
          constexpr int slot = pmod_c(s - dy, B);
          static_for<0, 2 * R + 1>([&](auto e_) {
            constexpr int dx = decltype(e_)::value - R;
            if constexpr (in_pattern(PAT, R, dx, dy, 0)) {
              constexpr int t = tap_index(PAT, R, 2, dx, dy, 0);
#pragma unroll
              for (int v = 0; v < VEC; ++v)
                acc[slot][v] = __builtin_fma(w.w[t], win[RA + v + dx], acc[slot][v]);
            }
          });
        });
#pragma unroll
        for (int v = 0; v < VEC; ++v) cen[s][v] = win[RA + v];
        constexpr int so = pmod_c(s - R, B);
        if (q >= 2 * R) emit(y0 + q - 2 * R, acc[so], cen[so]);
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[so][v] = T(0);
      }
    });
  }

  if constexpr (HAS_DOT) {
    DevScalars* sc = a.scal;
    const double c2 = a.c2;
    const int flag = a.flag;
    grid_reduce<NT>(dot, tile, (int)gridDim.x, a.partials, &sc->ticket,
                    [&](double total) { finalize<KIND>(sc, total, c2, flag); });
  }
}

}  // namespace sc
