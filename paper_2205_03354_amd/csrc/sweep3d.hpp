// Matrix-free stencil sweep over a 3D grid for gfx950 ("2.5D" blocking).
//
// One block owns a TX x TY column of the grid in the xy plane and a chunk of
// TZ planes along z. It streams input planes through a double-buffered LDS
// plane tile (with R halo rows and R, rounded up to VEC, halo columns), one
// barrier per plane, and accumulates along z in a register ring of 2R+1
// partial planes ("push" form, as in the 2D sweep): an input plane adds its
// contribution to the 2R+1 output planes it neighbours; an output plane is
// complete R planes later and is written once.
//
// Each thread owns VEC adjacent columns on RY rows. For every LDS row of its
// window it reads VEC+2R values (16-byte reads) and updates every output
// row / output plane that uses that row, so register use stays at one
// window row at a time.
#pragma once

#include "sweep2d.hpp"

namespace sc {

template <typename T, int KIND, int PAT, int R, bool PERIODIC, int NT>
__global__ void __launch_bounds__(NT)
    sweep3d_kernel(const SweepArgs<T> a, const Taps<T, num_taps(PAT, R, 3)> w) {
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int TX = 64;
  constexpr int NTX = TX / VEC;
  constexpr int NTY = NT / NTX;
  constexpr int RY = 2;
  constexpr int TY = NTY * RY;
  constexpr int RA = ((R + VEC - 1) / VEC) * VEC;
  constexpr int WX = TX + 2 * RA;
  constexpr int WY = TY + 2 * R;
  constexpr int PL = WX * WY;
  constexpr int LPP = (PL + NT - 1) / NT;
  constexpr int B = 2 * R + 1;
  constexpr int NV = (RA + R + VEC) / VEC + ((RA + R + VEC) % VEC ? 1 : 0);
  constexpr bool HAS_DOT = kind_has_dot(KIND);
  using V = typename VecT<T, VEC>::type;
  static_assert(NT % NTX == 0, "block must tile the x extent");
  static_assert((NV - 1) * VEC <= 2 * RA, "window reads must stay inside the LDS row");

  __shared__ __attribute__((aligned(16))) T lds[2 * PL];

  if constexpr (KIND == K_CGDIR) {
    if (a.scal->done) return;
  }
  // beta from the finish kernel, or formed here from the CG update's
  // partials (fold_update); a converged recurrence leaves nothing to do
  T beta = T(0);
  if constexpr (KIND == K_CGDIR) {
    if (a.fold) {
      double b = 0.0;
      if (!fold_update<NT>(a.scal, a.fold, a.fold_n, &b)) return;
      beta = (T)b;
    } else {
      beta = (T)a.scal->beta;
    }
  }
  const T c1 = (T)a.c1;

  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int xy = tile / a.tiles_b;
  const int zc = tile - xy * a.tiles_b;
  const int txi = xy % a.tiles_x2;
  const int tyi = xy / a.tiles_x2;
  const int64_t x0 = (int64_t)txi * TX;
  const int64_t y0 = (int64_t)tyi * TY;
  const int64_t z0 = (int64_t)zc * a.ty;
  const int planes = (int)((a.n2 - z0) < a.ty ? (a.n2 - z0) : a.ty);
  const int NQ = planes + 2 * R;
  const int l = (int)threadIdx.x;
  const int tx = l % NTX, tyt = l / NTX;

  // Staging assignment: element e = l + k NT of the LDS plane tile.
  int64_t goff[LPP];
  bool gok[LPP];
  bool gint[LPP];  // inside the interior in x and y (for K_BVPRHS)
#pragma unroll
  for (int k = 0; k < LPP; ++k) {
    const int e = l + k * NT;
    const int py = e / WX, px = e - py * WX;
    int64_t gx = x0 - RA + px;
    int64_t gy = y0 - R + py;
    gok[k] = (e < PL) && gx >= -R && gx < a.n0 + R && gy >= -R && gy < a.n1 + R;
    gint[k] = gx >= 0 && gx < a.n0 && gy >= 0 && gy < a.n1;
    if constexpr (PERIODIC) {
      gx = a.small ? wrap_small(gx, a.n0) : wrap_once(gx, a.n0);
      gy = a.small ? wrap_small(gy, a.n1) : wrap_once(gy, a.n1);
    }
    goff[k] = gy * a.pin + gx;
  }
  int64_t goff2[LPP];
  if constexpr (KIND == K_CGDIR) {
#pragma unroll
    for (int k = 0; k < LPP; ++k) {
      const int e = l + k * NT;
      const int py = e / WX, px = e - py * WX;
      int64_t gx = x0 - RA + px;
      int64_t gy = y0 - R + py;
      if constexpr (PERIODIC) {
        gx = a.small ? wrap_small(gx, a.n0) : wrap_once(gx, a.n0);
        gy = a.small ? wrap_small(gy, a.n1) : wrap_once(gy, a.n1);
      }
      goff2[k] = gy * a.pin2 + gx;
    }
  }

  T pre[LPP];
  auto load_plane = [&](int q) {
    int64_t gz = z0 - R + q;
    const bool zin = gz >= 0 && gz < a.n2;
    if constexpr (PERIODIC) gz = a.small ? wrap_small(gz, a.n2) : wrap_once(gz, a.n2);
    const T* src = a.in + gz * a.zin;
#pragma unroll
    for (int k = 0; k < LPP; ++k) {
      T v = T(0);
      if (gok[k]) {
        v = src[goff[k]];
        if constexpr (KIND == K_CGDIR) {
          v = v + beta * a.in2[gz * a.zin2 + goff2[k]];
        } else if constexpr (KIND == K_BVPRHS) {
          if (zin && gint[k]) v = T(0);
        } else if constexpr (KIND == K_CHRHS) {
          v = v * v * v - c1 * v;
        }
      }
      pre[k] = v;
    }
  };

  T acc[B][RY][VEC];
  T cen[B][RY][VEC];
#pragma unroll
  for (int s = 0; s < B; ++s)
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[s][r][v] = T(0);
  double dot = 0.0;

  const int64_t mycol = x0 + (int64_t)tx * VEC;
  const int64_t myrow = y0 + (int64_t)tyt * RY;
  const bool full_vec = a.vec_store && (mycol + VEC <= a.n0);

  auto emit = [&](int64_t gz, int r, const T* accv, const T* cenv) {
    const int64_t gy = myrow + r;
    if (gy >= a.n1) return;
    if constexpr (KIND == K_APPLY) {
      T* o = a.out + gz * a.zout + gy * a.pout + mycol;
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
            a.out[gz * a.zout + gy * a.pout + col] = cenv[v];
            a.out2[gz * a.zout2 + gy * a.pout2 + col] = accv[v];
            dot += (double)cenv[v] * (double)accv[v];
          } else if constexpr (KIND == K_RESID || KIND == K_BVPRHS) {
            const T rr = a.aux[gz * a.zaux + gy * a.paux + col] - accv[v];
            a.out[gz * a.zout + gy * a.pout + col] = rr;
            dot += (double)rr * (double)rr;
          } else if constexpr (KIND == K_SCALE) {
            a.out[gz * a.zout + gy * a.pout + col] = a.aux[gz * a.zaux + gy * a.paux + col] * accv[v];
          } else if constexpr (KIND == K_ACCUM) {
            a.out[gz * a.zout + gy * a.pout + col] = a.aux[gz * a.zaux + gy * a.paux + col] + accv[v];
          } else if constexpr (KIND == K_CHRHS) {
            const T rr = __builtin_fma((T)a.c0, accv[v], (T)a.c3 * a.in[gz * a.zin + gy * a.pin + col]);
            a.out[gz * a.zout + gy * a.pout + col] = rr;
            dot += (double)rr * (double)rr;
          }
        }
      }
    }
  };

  const int nb = (NQ + B - 1) / B;
  load_plane(0);
  for (int b = 0; b < nb; ++b) {
    static_for<0, B>([&](auto s_) {
      constexpr int s = decltype(s_)::value;
      const int q = b * B + s;
      if (q < NQ) {
        T* buf = lds + (q & 1) * PL;
#pragma unroll
        for (int k = 0; k < LPP; ++k) {
          const int e = l + k * NT;
          if (k < LPP - 1 || e < PL) buf[e] = pre[k];
        }
        __syncthreads();
        if (q + 1 < NQ) load_plane(q + 1);
        // rows of the window: LDS row tyt*RY + rho, rho in [0, RY + 2R)
        static_for<0, RY + 2 * R>([&](auto rho_) {
          constexpr int rho = decltype(rho_)::value;
          T win[NV * VEC];
          const V* rowv = reinterpret_cast<const V*>(buf + (tyt * RY + rho) * WX) + tx;
#pragma unroll
          for (int kv = 0; kv < NV; ++kv) {
            const V t = rowv[kv];
#pragma unroll
            for (int e = 0; e < VEC; ++e) win[kv * VEC + e] = t[e];
          }
          static_for<0, RY>([&](auto r_) {
            constexpr int r = decltype(r_)::value;
            constexpr int dy = rho - R - r;
            if constexpr (dy >= -R && dy <= R) {
              static_for<0, B>([&](auto dz_) {
                constexpr int dz = decltype(dz_)::value - R;
                constexpr int slot = pmod_c(s - dz, B);
                static_for<0, 2 * R + 1>([&](auto e_) {
                  constexpr int dx = decltype(e_)::value - R;
                  if constexpr (in_pattern(PAT, R, dx, dy, dz)) {
                    constexpr int t = tap_index(PAT, R, 3, dx, dy, dz);
#pragma unroll
                    for (int v = 0; v < VEC; ++v)
                      acc[slot][r][v] = __builtin_fma(w.w[t], win[RA + v + dx], acc[slot][r][v]);
                  }
                });
              });
            }
            if constexpr (dy == 0) {
#pragma unroll
              for (int v = 0; v < VEC; ++v) cen[s][r][v] = win[RA + v];
            }
          });
        });
        constexpr int so = pmod_c(s - R, B);
        if (q >= 2 * R) {
#pragma unroll
          for (int r = 0; r < RY; ++r) emit(z0 + q - 2 * R, r, acc[so][r], cen[so][r]);
        }
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[so][r][v] = T(0);
      }
    });
  }

  if constexpr (HAS_DOT) block_partial<NT>(dot, tile, a.partials);
  if constexpr (KIND == K_CGDIR)
    if (blockIdx.x == 0 && threadIdx.x == 0) a.scal->slots = (int)gridDim.x;
}

}  // namespace sc
