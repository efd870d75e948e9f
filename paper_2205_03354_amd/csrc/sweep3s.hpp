// Matrix-free sweep over a 3D grid for mirror-symmetric stencils (gfx950).
//
// One wave64 per workgroup owns an x-y tile of 64 * VPL columns (VPL = 16
// bytes / element) by TY rows and a chunk of planes along z, and streams the
// chunk's input planes (plus R halo planes on either side) through a
// wave-private LDS ring. Each ring slot holds one input plane of the tile
// with R halo rows and RA (R rounded up to VPL) halo columns, filled by
// 16-byte global->LDS DMAs (global_load_lds_dwordx4) packed across the
// slot's rows, D planes ahead of the plane being consumed; the wave waits
// for its own DMAs with an explicit vmcnt and needs no workgroup barrier.
//
// The stencil is pushed along z: an input plane contributes to the 2R + 1
// output planes it neighbours, kept in a register ring; an output plane is
// complete 2R planes after its first contribution and is written once.
// Within a plane, the weights depend only on (|dx|, |dy|, |dz|), so each
// input row is read once into registers, folded into mirror pair sums
// x(+d) + x(-d), and every (|dy|, |dz|) class contributes one short dot
// product to the output rows and planes it reaches.
#pragma once

#include "sweep2d.hpp"

namespace sc {

// Class weight index of (|dx|, |dy|, |dz|) = (d, b, a).
__host__ __device__ constexpr int sym3_index(int R, int d, int b, int a) { return (a * (R + 1) + b) * (R + 1) + d; }
__host__ __device__ constexpr int sym3_nweights(int R) { return (R + 1) * (R + 1) * (R + 1); }
// Any tap of the pattern in row |dy| = b of plane |dz| = a?
__host__ __device__ constexpr bool sym3_row(int pat, int R, int b, int a) {
  for (int d = 0; d <= R; ++d)
    if (in_pattern(pat, R, d, b, a)) return true;
  return false;
}

template <typename T, int KIND, int PAT, int R, bool PER, int TY, int D>
__global__ void __launch_bounds__(64)
    sweep3s_kernel(const SweepArgs<T> a, const Taps<T, sym3_nweights(R)> w) {
  constexpr int VPL = 16 / (int)sizeof(T);
  constexpr int TXW = 64 * VPL;
  constexpr int RA = ((R + VPL - 1) / VPL) * VPL;
  constexpr int W = TXW + 2 * RA;         // LDS row (elements)
  constexpr int NCR = W / VPL;            // 16-byte chunks per LDS row
  constexpr int NYR = TY + 2 * R;         // LDS rows per plane
  constexpr int NCH = NYR * NCR;          // chunks per plane
  constexpr int KF = (NCH + 63) / 64;     // chunk DMAs per plane
  constexpr int PLANE = NYR * W;          // elements per slot
  constexpr bool TWO = KIND == K_CGDIR;
  constexpr bool AUX = kind_reads_aux(KIND);
  constexpr bool NEED_CEN = KIND == K_CGDIR || KIND == K_CHRHS;
  constexpr bool HAS_DOT = kind_has_dot(KIND);
  constexpr int NRING = D + 2;
  constexpr int B = 2 * R + 1;
  constexpr int NV = (VPL + 2 * RA) / VPL;
  constexpr int KFAST = KF * (TWO ? 2 : 1) + (AUX ? TY : 0);
  constexpr int WAITN = KFAST * D < 63 ? KFAST * D : 63;
  using V = typename VecT<T, VPL>::type;
  static_assert(TXW / VPL == 64, "one aux row is one 64-lane chunk DMA");

  __shared__ __attribute__((aligned(16))) T ring[NRING * PLANE];
  __shared__ __attribute__((aligned(16))) T ring2[TWO ? NRING * PLANE : VPL];
  __shared__ __attribute__((aligned(16))) T ringa[AUX ? NRING * TY * TXW : VPL];

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

  // tile order: x fastest, then y, then z chunks
  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int txy = a.tiles_a;  // x tiles * y tiles
  const int zc = tile / txy;
  const int rem = tile - zc * txy;
  const int tyi = rem / a.tiles_x2;
  const int txi = rem - tyi * a.tiles_x2;
  const int64_t x0 = (int64_t)txi * TXW;
  const int64_t y0 = (int64_t)tyi * TY;
  const int64_t z0 = (int64_t)zc * a.ty;
  const int planes = (int)((a.n2 - z0) < a.ty ? (a.n2 - z0) : a.ty);
  const int NQ = planes + 2 * R;
  const int lane = (int)threadIdx.x;
  const int64_t lo = x0 - RA;
  // 16-byte chunk DMA: aligned rows and planes, and (periodic) chunks that
  // never straddle the x seam, or (ring) every chunk inside the stored ring
  const bool fast = a.in_aligned && (PER ? (a.n0 % VPL == 0) : (lo >= a.xlo && lo + W <= a.xhi)) &&
                    (!AUX || x0 + TXW <= a.axhi);

  auto wrap_x = [&](int64_t c) -> int64_t {
    if constexpr (PER) return a.small ? wrap_small(c, a.n0) : wrap_once(c, a.n0);
    return c;
  };
  auto row_of = [&](int r) -> int64_t {  // LDS row r (0 .. NYR-1) -> grid row
    int64_t gy = y0 - R + r;
    if constexpr (PER) {
      gy = a.small ? wrap_small(gy, a.n1) : wrap_once(gy, a.n1);
    } else {
      gy = gy < a.n1 + R ? gy : a.n1 + R - 1;  // rows past the ring only feed masked outputs
    }
    return gy;
  };
  auto plane_of = [&](int q) -> int64_t {  // input plane q (0 .. NQ-1) -> grid plane
    int64_t gz = z0 - R + q;
    if constexpr (PER) gz = a.small ? wrap_small(gz, a.n2) : wrap_once(gz, a.n2);
    return gz;
  };
  // aux plane travelling with input plane q: the output emitted at step q,
  // clamped into the chunk so that every step issues the same DMAs
  auto aux_plane = [&](int q) -> int64_t {
    int m = q - 2 * R;
    m = m < 0 ? 0 : (m >= planes ? planes - 1 : m);
    return z0 + m;
  };

  // In-plane element offsets of this lane's chunks: the same for every plane.
  // Chunk e = lane + 64 k of a slot is row e / NCR, chunk column e % NCR.
  int64_t coff[KF];
  int64_t coff2[TWO ? KF : 1];
#pragma unroll
  for (int k = 0; k < KF; ++k) {
    const int e = lane + 64 * k;
    const int r = e / NCR;
    const int c = e - r * NCR;
    const int64_t gy = row_of(r < NYR ? r : NYR - 1);
    const int64_t gx = wrap_x(lo + (int64_t)VPL * c);
    coff[k] = gy * a.pin + gx;
    if constexpr (TWO) coff2[k] = gy * a.pin2 + gx;
  }

  auto issue_fast = [&](int q) __attribute__((always_inline)) {
    const int slot = q % NRING;
    const int64_t gz = plane_of(q);
    {
      const T* base = a.in + gz * a.zin;
      T* lb = ring + slot * PLANE;
#pragma unroll
      for (int k = 0; k < KF; ++k)
        if (k < KF - 1 || lane + 64 * k < NCH)
          __builtin_amdgcn_global_load_lds((const void*)(base + coff[k]), (lds_void_t*)(lb + 64 * VPL * k), 16, 0, 0);
    }
    if constexpr (TWO) {
      const T* base = a.in2 + gz * a.zin2;
      T* lb = ring2 + slot * PLANE;
#pragma unroll
      for (int k = 0; k < KF; ++k)
        if (k < KF - 1 || lane + 64 * k < NCH)
          __builtin_amdgcn_global_load_lds((const void*)(base + coff2[k]), (lds_void_t*)(lb + 64 * VPL * k), 16, 0, 0);
    }
    if constexpr (AUX) {
      const int64_t az = aux_plane(q);
#pragma unroll
      for (int j = 0; j < TY; ++j) {
        int64_t gy = y0 + j;
        gy = gy < a.n1 ? gy : a.n1 - 1;
        const T* src = a.aux + az * a.zaux + gy * a.paux + x0 + VPL * lane;
        __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_t*)(ringa + (slot * TY + j) * TXW), 16, 0, 0);
      }
    }
  };
  // Slow path (unaligned rows, or strips whose chunks would leave the
  // readable columns): the wave loads plane q element by element with
  // bounds and wrap, writes its slot, and consumes it at once (no look-ahead).
  auto load_slow = [&](int q) __attribute__((always_inline)) {
    const int slot = q % NRING;
    const int64_t gz = plane_of(q);
    auto one = [&](const T* base, int64_t pitch, int64_t zpitch, T* lb) {
      const T* pz = base + gz * zpitch;
#pragma unroll 1
      for (int e = lane; e < PLANE; e += 64) {
        const int r = e / W;
        const int cx = e - r * W;
        int64_t col = lo + cx;
        bool ok = col < a.n0 + R;
        if constexpr (PER) {
          col = a.small ? wrap_small(col, a.n0) : wrap_once(col, a.n0);
        } else {
          ok = ok && col >= -R;
        }
        lb[e] = ok ? pz[row_of(r) * pitch + col] : T(0);
      }
    };
    one(a.in, a.pin, a.zin, ring + slot * PLANE);
    if constexpr (TWO) one(a.in2, a.pin2, a.zin2, ring2 + slot * PLANE);
    if constexpr (AUX) {
      const T* pz = a.aux + aux_plane(q) * a.zaux;
#pragma unroll 1
      for (int e = lane; e < TY * TXW; e += 64) {
        const int j = e / TXW;
        const int cx = e - j * TXW;
        int64_t gy = y0 + j;
        gy = gy < a.n1 ? gy : a.n1 - 1;
        ringa[slot * TY * TXW + e] = x0 + cx < a.n0 ? pz[gy * a.paux + x0 + cx] : T(0);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  };

  // acc[k] accumulates output plane q - 2R + k at input step q (k = 0 is
  // complete after step q); cen[k] holds the centre values of input step
  // q - k (the output plane emitted at step q has its centre at k = R).
  T acc[B][TY][VPL];
  T cen[NEED_CEN ? R + 1 : 1][NEED_CEN ? TY : 1][VPL];
#pragma unroll
  for (int s = 0; s < B; ++s)
#pragma unroll
    for (int j = 0; j < TY; ++j)
#pragma unroll
      for (int v = 0; v < VPL; ++v) acc[s][j][v] = T(0);
  double dot = 0.0;

  const int64_t mycol = x0 + (int64_t)lane * VPL;
  const bool full_vec = a.vec_store && (mycol + VPL <= a.n0);

  // store output plane gz, row j of the tile; `slot` is the ring slot of the
  // current input plane, which also carries this plane's aux values
  auto emit = [&](int64_t gz, int j, int slot, const T* accv, const T* cenv) __attribute__((always_inline)) {
    const int64_t gy = y0 + j;
    if (gy >= a.n1) return;
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
      const V t = reinterpret_cast<const V*>(ringa + (slot * TY + j) * TXW)[lane];
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
    T* o = a.out + gz * a.zout + gy * a.pout + mycol;
    T* o2 = (KIND == K_CGDIR) ? a.out2 + gz * a.zout2 + gy * a.pout2 + mycol : nullptr;
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
    if constexpr (FAST) {
      const int npro = NQ < D ? NQ : D;
      for (int q = 0; q < npro; ++q) issue_fast(q);
    }
    for (int q = 0; q < NQ; ++q) {
      if constexpr (FAST) {
        if (q + D < NQ) {
          issue_fast(q + D);
          wait_vmcnt<WAITN>();
        } else {
          wait_vmcnt<0>();
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else {
        load_slow(q);
      }
      const int slot = q % NRING;
      const int64_t gz_in = z0 - R + q;  // unwrapped: interior test for K_BVPRHS
      if constexpr (NEED_CEN) {
        static_for<0, R>([&](auto k_) {
          constexpr int k = R - decltype(k_)::value;  // R .. 1
          static_for<0, TY>([&](auto j_) {
            constexpr int j = decltype(j_)::value;
            static_for<0, VPL>([&](auto v_) {
              constexpr int v = decltype(v_)::value;
              cen[k][j][v] = cen[k - 1][j][v];
            });
          });
        });
      }
      static_for<0, NYR>([&](auto r_) {
        constexpr int r = decltype(r_)::value;
        // window of LDS row r: win[i] is column mycol - RA + i
        T win[NV * VPL];
        {
          const V* rv = reinterpret_cast<const V*>(ring + slot * PLANE + r * W) + lane;
#pragma unroll
          for (int kv = 0; kv < NV; ++kv) {
            const V t = rv[kv];
#pragma unroll
            for (int e = 0; e < VPL; ++e) win[kv * VPL + e] = t[e];
          }
        }
        if constexpr (TWO) {
          const V* rv = reinterpret_cast<const V*>(ring2 + slot * PLANE + r * W) + lane;
#pragma unroll
          for (int kv = 0; kv < NV; ++kv) {
            const V t = rv[kv];
#pragma unroll
            for (int e = 0; e < VPL; ++e) win[kv * VPL + e] = __builtin_fma(beta, t[e], win[kv * VPL + e]);
          }
        }
        if constexpr (NEED_CEN) {
          if constexpr (r >= R && r < R + TY) {
            static_for<0, VPL>([&](auto v_) {
              constexpr int v = decltype(v_)::value;
              cen[0][r - R][v] = win[RA + v];
            });
          }
        }
        if constexpr (KIND == K_CHRHS) {
#pragma unroll
          for (int i = 0; i < NV * VPL; ++i) {
            const T u = win[i];
            win[i] = u * u * u - c1 * u;
          }
        } else if constexpr (KIND == K_BVPRHS) {
          const int64_t gy = y0 - R + r;
          const bool yz_in = gy >= 0 && gy < a.n1 && gz_in >= 0 && gz_in < a.n2;
#pragma unroll
          for (int i = 0; i < NV * VPL; ++i) {
            const int64_t col = mycol - RA + i;
            if (yz_in && col >= 0 && col < a.n0) win[i] = T(0);
          }
        }
        static_for<0, VPL>([&](auto v_) {
          constexpr int v = decltype(v_)::value;
          T ps[R + 1];
          ps[0] = win[RA + v];
          static_for<1, R + 1>([&](auto d_) {
            constexpr int d = decltype(d_)::value;
            ps[d] = win[RA + v + d] + win[RA + v - d];
          });
          static_for<0, TY>([&](auto j_) {
            constexpr int j = decltype(j_)::value;
            constexpr int dy = r - R - j;
            constexpr int b = dy < 0 ? -dy : dy;
            if constexpr (b <= R) {
              static_for<0, R + 1>([&](auto a_) {
                constexpr int az = decltype(a_)::value;
                if constexpr (sym3_row(PAT, R, b, az)) {
                  T t = T(0);
                  static_for<0, R + 1>([&](auto d_) {
                    constexpr int d = decltype(d_)::value;
                    if constexpr (in_pattern(PAT, R, d, b, az))
                      t = __builtin_fma(w.w[sym3_index(R, d, b, az)], ps[d], t);
                  });
                  // input plane q feeds output planes q - R -/+ az, i.e.
                  // accumulators R -/+ az
                  acc[R - az][j][v] += t;
                  if constexpr (az > 0) acc[R + az][j][v] += t;
                }
              });
            }
          });
        });
      });
      if (q >= 2 * R) {
        const int64_t gz = z0 + q - 2 * R;
        static_for<0, TY>([&](auto j_) {
          constexpr int j = decltype(j_)::value;
          emit(gz, j, slot, acc[0][j], cen[NEED_CEN ? R : 0][NEED_CEN ? j : 0]);
        });
      }
      // shift the accumulator ring by one plane
      static_for<0, B - 1>([&](auto k_) {
        constexpr int k = decltype(k_)::value;
        static_for<0, TY>([&](auto j_) {
          constexpr int j = decltype(j_)::value;
          static_for<0, VPL>([&](auto v_) {
            constexpr int v = decltype(v_)::value;
            acc[k][j][v] = acc[k + 1][j][v];
          });
        });
      });
      static_for<0, TY>([&](auto j_) {
        constexpr int j = decltype(j_)::value;
        static_for<0, VPL>([&](auto v_) { acc[B - 1][j][decltype(v_)::value] = T(0); });
      });
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
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
