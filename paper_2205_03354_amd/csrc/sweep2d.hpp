// Matrix-free stencil sweep over a 2D grid for gfx950 (wave64).
//
// One kernel template serves every operation that applies a stencil: the
// plain apply, the CG direction sweep, the true residual and the right-hand
// sides of the biharmonic and Cahn-Hilliard problems. They differ only in
// what is fed to the stencil and what is done with the stencil value at each
// output point (`emit`).
//
// Work decomposition: one wavefront per block owns a strip of 64 * VPL
// columns (VPL = one 16-byte chunk per lane) and TY output rows.
//  * Input rows stream through a wave-private LDS ring by direct
//    global->LDS DMA (global_load_lds_dwordx4), D rows ahead of the row
//    being computed; no VGPRs are spent on staging and there is no block
//    barrier. The wave waits with an explicit vmcnt so that D rows stay in
//    flight. Strips whose rows are not 16-byte aligned or that touch the
//    periodic seam use 4-byte DMA with per-element wrapped addresses.
//  * "Push" accumulation along y: every input row adds its contribution to
//    the 2R+1 output rows it neighbours; their partial sums live in a
//    register ring indexed at compile time (the row loop is unrolled by
//    2R+1). An output row is complete R rows after its own input row and is
//    written once.
//  * Mirror-symmetric stencils (w(dx,dy) = w(-dx,dy) = w(dx,-dy), true for
//    every Laplacian / biharmonic / Cahn-Hilliard operator) use one weight
//    per class (|dx|,|dy|): pair sums x[+d] + x[-d] are formed once per
//    input row and each class product is added to the rows above and below.
//    This cuts the arithmetic (25 instead of 33 operations per point for the
//    33-point operator) and keeps the weights in scalar registers.
//  * Tiles are ordered x-fastest in bands, and the 8 XCDs each take a
//    contiguous range of bands, so horizontally adjacent strips (which
//    share partial cache lines) run together on one XCD. For symmetric
//    stencils every other band of tiles streams bottom-up, so two vertically
//    adjacent tiles read their shared halo rows at nearly the same time and
//    the second read hits in L2.
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
  int tiles_a, tiles_b;   // 2D: strips along x, tile rows; 3D: xy tiles, z chunks
  int tiles_x2;           // 3D: tiles along x
  int small;              // periodic wrap needs a true modulo (grid < radius)
  int vec_store;          // outputs 16-byte aligned for the vector store
  int in_aligned;         // 2D: inputs (in, in2, aux) have 16-byte aligned rows
  int alt;                // 2D: alternate the streaming direction by tile row
  int64_t xlo, xhi;       // ring mode: columns [xlo, xhi) of every in / in2 row are readable
  int64_t axhi;           // columns [0, axhi) of every aux row are readable
  DevScalars* scal;
  double* partials;
  double c0, c1, c2;      // K_CHRHS: dt, 1+S; K_BVPRHS/K_CHRHS: c2 = tol^2
  double c3;              // K_CHRHS: weight of the centre value u
  int flag;               // K_RESID: 1 = also (re)start the CG recurrence
  const double* fold;     // K_CGDIR: the CG update's <r, r> partials to finish here (or null)
  int fold_n;             // their count
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

// ---------------------------------------------------------------- weights
// Symmetric stencils carry one weight per class (d, a) = (|dx|, |dy|)
// admitted by the pattern, ordered a-major then d.
__host__ __device__ constexpr int sym_class_index(int pat, int R, int d, int a) {
  int idx = 0;
  for (int aa = 0; aa <= R; ++aa)
    for (int dd = 0; dd <= R; ++dd) {
      if (!in_pattern(pat, R, dd, aa, 0)) continue;
      if (dd == d && aa == a) return idx;
      ++idx;
    }
  return -1;
}
__host__ __device__ constexpr int sym_num_classes(int pat, int R) {
  int n = 0;
  for (int aa = 0; aa <= R; ++aa)
    for (int dd = 0; dd <= R; ++dd) n += in_pattern(pat, R, dd, aa, 0) ? 1 : 0;
  return n;
}
// smallest |dx| present in row |dy| = a of the pattern
__host__ __device__ constexpr int sym_first_d(int pat, int R, int a) {
  for (int dd = 0; dd <= R; ++dd)
    if (in_pattern(pat, R, dd, a, 0)) return dd;
  return R + 1;
}
__host__ __device__ constexpr int sweep2d_nweights(int pat, int R, bool sym) {
  return sym ? sym_num_classes(pat, R) : num_taps(pat, R, 2);
}

// vmcnt-only wait: vector-memory count <= N, no wait on LDS / export.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt is 6 bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

typedef __attribute__((address_space(3))) void lds_void_t;

// Rows in flight per wave (DMA look-ahead) and the strip geometry.
constexpr int kRingDepth = 6;
template <typename T>
__host__ __device__ constexpr int strip_width_2d() { return 64 * (16 / (int)sizeof(T)); }

template <typename T, int KIND, int PAT, int R, bool PER, bool SYM>
__global__ void __launch_bounds__(64)
    sweep2d_kernel(const SweepArgs<T> a, const Taps<T, sweep2d_nweights(PAT, R, SYM)> w) {
  constexpr int VPL = 16 / (int)sizeof(T);   // elements per lane = one 16-byte chunk
  constexpr int TXW = 64 * VPL;              // strip width
  constexpr int RA = ((R + VPL - 1) / VPL) * VPL;
  constexpr int W = TXW + 2 * RA;            // LDS row length (elements)
  constexpr int NCH = W / VPL;               // 16-byte chunks per row
  constexpr int KF = (NCH + 63) / 64;        // chunk DMAs per input row
  constexpr int DPE = (int)sizeof(T) / 4;    // dwords per element
  constexpr int NDW = W * DPE;
  constexpr int KS = (NDW + 63) / 64;        // dword DMAs per input row
  constexpr int NAUXDW = TXW * DPE;
  constexpr int KSA = (NAUXDW + 63) / 64;    // dword DMAs per aux row
  constexpr bool TWO = KIND == K_CGDIR;      // second input (p_old)
  constexpr bool AUX = kind_reads_aux(KIND);
  constexpr bool NEED_CEN = KIND == K_CGDIR || KIND == K_CHRHS;
  constexpr int D = kRingDepth;
  constexpr int NRING = D + 2;
  constexpr int B = 2 * R + 1;
  constexpr int NV = (VPL + 2 * RA) / VPL;   // chunks in a lane's window
  constexpr bool HAS_DOT = kind_has_dot(KIND);
  constexpr int KFAST = KF * (TWO ? 2 : 1) + (AUX ? 1 : 0);
  constexpr int KSLOW = KS * (TWO ? 2 : 1) + (AUX ? KSA : 0);
  using V = typename VecT<T, VPL>::type;

  __shared__ __attribute__((aligned(16))) T ring[NRING * W];
  __shared__ __attribute__((aligned(16))) T ring2[TWO ? NRING * W : VPL];
  __shared__ __attribute__((aligned(16))) T ringa[AUX ? NRING * TXW : VPL];

  if constexpr (KIND == K_CGDIR) {
    if (a.scal->done) return;
  }
  // beta from the finish kernel, or formed here from the CG update's
  // partials (fold_update); a converged recurrence leaves nothing to do
  T beta = T(0);
  if constexpr (KIND == K_CGDIR) {
    if (a.fold) {
      double b = 0.0;
      if (!fold_update<64>(a.scal, a.fold, a.fold_n, &b)) return;
      beta = (T)b;
    } else {
      beta = (T)a.scal->beta;
    }
  }
  const T c1 = (T)a.c1;

  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int sx = tile % a.tiles_a;
  const int syi = tile / a.tiles_a;
  const int64_t x0 = (int64_t)sx * TXW;
  const int64_t y0 = (int64_t)syi * a.ty;
  const int rows = (int)((a.n1 - y0) < a.ty ? (a.n1 - y0) : a.ty);
  const int NR = rows + 2 * R;
  const int lane = (int)threadIdx.x;
  const int64_t lo = x0 - RA;
  // chunk DMA needs 16-byte aligned rows, no periodic seam inside the strip
  // and (ring mode) every loaded column inside the stored ring
  const bool fast = a.in_aligned && !a.small &&
                    (PER ? (lo >= 0 && lo + W <= a.n0) : (lo >= a.xlo && lo + W <= a.xhi)) &&
                    (!AUX || x0 + TXW <= a.axhi);
  const bool rev = SYM && a.alt && (syi & 1);

  // input row index q (0 .. NR-1, streaming order) -> grid row
  auto grid_row = [&](int q) -> int64_t {
    int64_t gy = rev ? (y0 + rows - 1 + R - q) : (y0 - R + q);
    if constexpr (PER) gy = a.small ? wrap_small(gy, a.n1) : wrap_once(gy, a.n1);
    return gy;
  };
  // aux row travelling with input row q: the output emitted when q is the
  // current row (output index q - 2R, clamped into the tile so that every
  // step issues the same number of DMAs)
  auto aux_row = [&](int q) -> int64_t {
    int m = q - 2 * R;
    m = m < 0 ? 0 : (m >= rows ? rows - 1 : m);
    return rev ? (y0 + rows - 1 - m) : (y0 + m);
  };

  auto issue_fast = [&](int q) {
    const int slot = q % NRING;
    const int64_t gy = grid_row(q);
    {
      const T* rp = a.in + gy * a.pin + lo;
      T* lb = ring + slot * W;
#pragma unroll
      for (int k = 0; k < KF; ++k) {
        const int c = lane + 64 * k;
        if (k < KF - 1 || c < NCH)
          __builtin_amdgcn_global_load_lds((const void*)(rp + VPL * c), (lds_void_t*)(lb + 64 * VPL * k), 16,
                                           0, 0);
      }
    }
    if constexpr (TWO) {
      const T* rp = a.in2 + gy * a.pin2 + lo;
      T* lb = ring2 + slot * W;
#pragma unroll
      for (int k = 0; k < KF; ++k) {
        const int c = lane + 64 * k;
        if (k < KF - 1 || c < NCH)
          __builtin_amdgcn_global_load_lds((const void*)(rp + VPL * c), (lds_void_t*)(lb + 64 * VPL * k), 16,
                                           0, 0);
      }
    }
    if constexpr (AUX) {
      const T* rp = a.aux + aux_row(q) * a.paux + x0;
      __builtin_amdgcn_global_load_lds((const void*)(rp + VPL * lane), (lds_void_t*)(ringa + slot * TXW), 16,
                                       0, 0);
    }
  };
  // The look-ahead wait counts KSLOW DMA instructions per row, and a DMA
  // whose lanes are all masked off is skipped by the branch around it, so
  // lane 0 always issues: when its own column is not needed it re-reads
  // column 0 of the row into its LDS slot, which no stored output reads.
  auto issue_slow = [&](int q) {
    const int slot = q % NRING;
    const int64_t gy = grid_row(q);
    auto one = [&](const T* base, int64_t pitch, T* lb) {
      const unsigned int* rp = reinterpret_cast<const unsigned int*>(base + gy * pitch);
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int d = lane + 64 * k;
        const int e = d / DPE;
        int64_t col = lo + e;
        bool ok = (k < KS - 1 || d < NDW) && col < a.n0 + R;
        if constexpr (PER) {
          col = a.small ? wrap_small(col, a.n0) : wrap_once(col, a.n0);
        } else {
          ok = ok && col >= -R;
        }
        const int64_t off = ok ? col * DPE + (d % DPE) : 0;
        if (ok || lane == 0)
          __builtin_amdgcn_global_load_lds((const void*)(rp + off),
                                           (lds_void_t*)(reinterpret_cast<unsigned int*>(lb) + 64 * k), 4, 0, 0);
      }
    };
    one(a.in, a.pin, ring + slot * W);
    if constexpr (TWO) one(a.in2, a.pin2, ring2 + slot * W);
    if constexpr (AUX) {
      const unsigned int* rp = reinterpret_cast<const unsigned int*>(a.aux + aux_row(q) * a.paux + x0);
#pragma unroll
      for (int k = 0; k < KSA; ++k) {
        const int d = lane + 64 * k;
        const bool ok = (k < KSA - 1 || d < NAUXDW) && x0 + d / DPE < a.n0;
        if (ok || lane == 0)
          __builtin_amdgcn_global_load_lds(
              (const void*)(rp + (ok ? d : 0)),
              (lds_void_t*)(reinterpret_cast<unsigned int*>(ringa + slot * TXW) + 64 * k), 4, 0, 0);
      }
    }
  };

  T acc[B][VPL];
  T cen[NEED_CEN ? B : 1][VPL];
#pragma unroll
  for (int s = 0; s < B; ++s)
#pragma unroll
    for (int v = 0; v < VPL; ++v) acc[s][v] = T(0);
  double dot = 0.0;

  const int64_t mycol = x0 + (int64_t)lane * VPL;
  const bool full_vec = a.vec_store && (mycol + VPL <= a.n0);

  // store one finished output row (grid row gy); `slot` is the ring slot of
  // the current input row, which also carries this row's aux values
  auto emit = [&](int64_t gy, int slot, const T* accv, const T* cenv) {
    T res[VPL];
    T res2[VPL];
    if constexpr (KIND == K_APPLY) {
#pragma unroll
      for (int v = 0; v < VPL; ++v) res[v] = accv[v];
    } else if constexpr (KIND == K_CGDIR) {
#pragma unroll
      for (int v = 0; v < VPL; ++v) {
        res[v] = cenv[v];
        res2[v] = accv[v];
      }
    } else if constexpr (AUX) {
      const V t = reinterpret_cast<const V*>(ringa + slot * TXW)[lane];
#pragma unroll
      for (int v = 0; v < VPL; ++v) {
        if constexpr (KIND == K_SCALE)
          res[v] = t[v] * accv[v];
        else if constexpr (KIND == K_ACCUM)
          res[v] = t[v] + accv[v];
        else
          res[v] = t[v] - accv[v];
      }
    } else if constexpr (KIND == K_CHRHS) {
#pragma unroll
      for (int v = 0; v < VPL; ++v) res[v] = __builtin_fma((T)a.c0, accv[v], (T)a.c3 * cenv[v]);
    }
    if constexpr (HAS_DOT) {
#pragma unroll
      for (int v = 0; v < VPL; ++v) {
        if (mycol + v < a.n0) {
          if constexpr (KIND == K_CGDIR)
            dot += (double)res[v] * (double)res2[v];
          else
            dot += (double)res[v] * (double)res[v];
        }
      }
    }
    T* o = a.out + gy * a.pout + mycol;
    T* o2 = (KIND == K_CGDIR) ? a.out2 + gy * a.pout2 + mycol : nullptr;
    if (full_vec) {
      V t;
#pragma unroll
      for (int v = 0; v < VPL; ++v) t[v] = res[v];
      if constexpr (KIND == K_APPLY)
        __builtin_nontemporal_store(t, reinterpret_cast<V*>(o));
      else
        *reinterpret_cast<V*>(o) = t;
      if constexpr (KIND == K_CGDIR) {
        V t2;
#pragma unroll
        for (int v = 0; v < VPL; ++v) t2[v] = res2[v];
        *reinterpret_cast<V*>(o2) = t2;
      }
    } else {
#pragma unroll
      for (int v = 0; v < VPL; ++v) {
        if (mycol + v < a.n0) {
          o[v] = res[v];
          if constexpr (KIND == K_CGDIR) o2[v] = res2[v];
        }
      }
    }
  };

  auto body = [&](auto fast_c) {
    constexpr bool FAST = decltype(fast_c)::value;
    constexpr int K = FAST ? KFAST : KSLOW;
    constexpr int WAITN = K * D < 63 ? K * D : 63;
    const int npro = NR < D ? NR : D;
    for (int q = 0; q < npro; ++q) {
      if constexpr (FAST) issue_fast(q); else issue_slow(q);
    }
    const int nb = (NR + B - 1) / B;
    for (int b = 0; b < nb; ++b) {
      static_for<0, B>([&](auto s_) {
        constexpr int s = decltype(s_)::value;
        const int q = b * B + s;
        if (q < NR) {
          if (q + D < NR) {
            if constexpr (FAST) issue_fast(q + D); else issue_slow(q + D);
            wait_vmcnt<WAITN>();
          } else {
            wait_vmcnt<0>();
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const int slot = q % NRING;
          // window: win[j] is column mycol - RA + j
          T win[NV * VPL];
          {
            const V* rv = reinterpret_cast<const V*>(ring + slot * W) + lane;
#pragma unroll
            for (int kv = 0; kv < NV; ++kv) {
              const V t = rv[kv];
#pragma unroll
              for (int e = 0; e < VPL; ++e) win[kv * VPL + e] = t[e];
            }
          }
          if constexpr (TWO) {
            const V* rv = reinterpret_cast<const V*>(ring2 + slot * W) + lane;
#pragma unroll
            for (int kv = 0; kv < NV; ++kv) {
              const V t = rv[kv];
#pragma unroll
              for (int e = 0; e < VPL; ++e) win[kv * VPL + e] = __builtin_fma(beta, t[e], win[kv * VPL + e]);
            }
          }
          if constexpr (KIND == K_CHRHS) {
#pragma unroll
            for (int v = 0; v < VPL; ++v) cen[s][v] = win[RA + v];
#pragma unroll
            for (int j = 0; j < NV * VPL; ++j) {
              const T u = win[j];
              win[j] = u * u * u - c1 * u;
            }
          } else if constexpr (KIND == K_BVPRHS) {
            const int64_t gy = grid_row(q);
            const bool row_in = gy >= 0 && gy < a.n1;
#pragma unroll
            for (int j = 0; j < NV * VPL; ++j) {
              const int64_t col = mycol - RA + j;
              if (row_in && col >= 0 && col < a.n0) win[j] = T(0);
            }
          } else if constexpr (KIND == K_CGDIR) {
#pragma unroll
            for (int v = 0; v < VPL; ++v) cen[s][v] = win[RA + v];
          }
          // accumulate into the output rows this input row neighbours
          if constexpr (SYM) {
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
              T ps[R + 1];
              ps[0] = win[RA + v];
              static_for<1, R + 1>([&](auto d_) {
                constexpr int d = decltype(d_)::value;
                ps[d] = win[RA + v + d] + win[RA + v - d];
              });
              static_for<0, R + 1>([&](auto a_) {
                constexpr int aa = decltype(a_)::value;
                constexpr int fd = sym_first_d(PAT, R, aa);
                if constexpr (fd <= R) {
                  if constexpr (aa == 0) {
                    static_for<0, R + 1>([&](auto d_) {
                      constexpr int d = decltype(d_)::value;
                      if constexpr (in_pattern(PAT, R, d, 0, 0))
                        acc[s][v] = __builtin_fma(w.w[sym_class_index(PAT, R, d, 0)], ps[d], acc[s][v]);
                    });
                  } else {
                    T t = w.w[sym_class_index(PAT, R, fd, aa)] * ps[fd];
                    static_for<0, R + 1>([&](auto d_) {
                      constexpr int d = decltype(d_)::value;
                      if constexpr (d > fd && in_pattern(PAT, R, d, aa, 0))
                        t = __builtin_fma(w.w[sym_class_index(PAT, R, d, aa)], ps[d], t);
                    });
                    constexpr int sp = pmod_c(s - aa, B);
                    constexpr int sm = pmod_c(s + aa, B);
                    acc[sp][v] += t;
                    acc[sm][v] += t;
                  }
                }
              });
            }
          } else {
            static_for<0, B>([&](auto d_) {
              constexpr int dy = decltype(d_)::value - R;
              constexpr int slot2 = pmod_c(s - dy, B);
              static_for<0, 2 * R + 1>([&](auto e_) {
                constexpr int dx = decltype(e_)::value - R;
                if constexpr (in_pattern(PAT, R, dx, dy, 0)) {
                  constexpr int t = tap_index(PAT, R, 2, dx, dy, 0);
#pragma unroll
                  for (int v = 0; v < VPL; ++v)
                    acc[slot2][v] = __builtin_fma(w.w[t], win[RA + v + dx], acc[slot2][v]);
                }
              });
            });
          }
          constexpr int so = pmod_c(s - R, B);
          if (q >= 2 * R) {
            const int m = q - 2 * R;
            const int64_t gy = rev ? (y0 + rows - 1 - m) : (y0 + m);
            emit(gy, slot, acc[so], cen[NEED_CEN ? so : 0]);
          }
#pragma unroll
          for (int v = 0; v < VPL; ++v) acc[so][v] = T(0);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        }
      });
    }
  };
  if (fast)
    body(std::integral_constant<bool, true>{});
  else
    body(std::integral_constant<bool, false>{});

  if constexpr (HAS_DOT) block_partial<64>(dot, tile, a.partials);
  if constexpr (KIND == K_CGDIR)
    if (blockIdx.x == 0 && threadIdx.x == 0) a.scal->slots = (int)gridDim.x;
}

}  // namespace sc
