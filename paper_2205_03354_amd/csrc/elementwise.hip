// Element-wise kernels of the Krylov solves (no stencil): the CG update
// sweep, the refinement cast / update, grid copies and the Cahn-Hilliard
// diagnostics, and the one-block finish kernels of every grid reduction. All
// reductions are deterministic (fixed per-thread order, fixed block tree,
// partials summed in slot order by a finish kernel; the diagnostics, run
// once per call, let their last block sum them).
#include "internal.hpp"

namespace sc {

namespace {

constexpr int kNT = 256;
static_assert(kNT == kFinNT, "the update finish folded into a sweep uses this order");

// Rows [r0, r1) of the interior assigned to this block; row rho is
// (j, k) = (rho % n1, rho / n1).
struct RowRange {
  int64_t r0, r1;
};
__device__ __forceinline__ RowRange block_rows(int64_t nrows) {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  return {b * nrows / nb, (b + 1) * nrows / nb};
}
__device__ __forceinline__ int64_t row_offset(int64_t rho, int64_t n1, int64_t pitch, int64_t zpitch) {
  const int64_t k = rho / n1, j = rho - k * n1;
  return k * zpitch + j * pitch;
}

// x += alpha p ; r -= alpha q ; rr_new = <r, r>  (then beta, convergence)
template <typename T>
__global__ void __launch_bounds__(kNT)
    cg_update_kernel(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                     const T* __restrict__ q, int64_t pitch, int64_t zpitch, int64_t n0, int64_t n1,
                     int64_t n2, DevScalars* s, const double* __restrict__ pq_partials, int pc,
                     double* partials) {
  if (s->done) return;
  // alpha = (pc ? <r, z> : <r, r>) / <p, q> from the direction sweep's
  // partials: every block sums them in the same order, so all agree; block
  // 0 records pq and alpha, or the breakdown
  __shared__ double s_alpha;
  __shared__ int s_ok;
  const double pq = sum_partials<kNT>(pq_partials, s->slots);
  if (threadIdx.x == 0) {
    const bool ok = pq > 0.0 && __builtin_isfinite(pq);
    s_ok = ok ? 1 : 0;
    s_alpha = ok ? (pc ? s->rz : s->rr) / pq : 0.0;
    if (blockIdx.x == 0) {
      s->pq = pq;
      s->rr_prev = s->rr;
      if (ok)
        s->alpha = s_alpha;
      else
        s->done = 2;
    }
  }
  __syncthreads();
  if (!s_ok) return;
  const T alpha = (T)s_alpha;
  const RowRange rr = block_rows(n1 * n2);
  double dot = 0.0;
  for (int64_t rho = rr.r0; rho < rr.r1; ++rho) {
    const int64_t o = row_offset(rho, n1, pitch, zpitch);
    for (int64_t i = threadIdx.x; i < n0; i += kNT) {
      const T pv = p[o + i], qv = q[o + i];
      x[o + i] = x[o + i] + alpha * pv;
      const T rv = r[o + i] - alpha * qv;
      r[o + i] = rv;
      dot += (double)rv * (double)rv;
    }
  }
  block_partial<kNT>(dot, (int)blockIdx.x, partials);
}

__global__ void __launch_bounds__(kNT)
    ir_prepare_kernel(const double* __restrict__ r64, int64_t p64, int64_t z64, float* __restrict__ r32,
                      float* __restrict__ d32, int64_t p32, int64_t z32, int64_t n0, int64_t n1,
                      int64_t n2, const DevScalars* s64, DevScalars* s32, double inner_tol2,
                      int keep_direction, double* partials) {
  // A restart scales by the current ||r||; a reliable update keeps the scale
  // of the stretch's restart so that the FP32 direction p stays consistent.
  const double inv = keep_direction ? 1.0 / s32->scale : 1.0 / sqrt(s64->rr_true);
  const RowRange rr = block_rows(n1 * n2);
  double dot = 0.0;
  for (int64_t rho = rr.r0; rho < rr.r1; ++rho) {
    const int64_t o64 = row_offset(rho, n1, p64, z64);
    const int64_t o32 = row_offset(rho, n1, p32, z32);
    for (int64_t i = threadIdx.x; i < n0; i += kNT) {
      const float v = (float)(r64[o64 + i] * inv);
      r32[o32 + i] = v;
      d32[o32 + i] = 0.0f;
      dot += (double)v * (double)v;
    }
  }
  block_partial<kNT>(dot, (int)blockIdx.x, partials);
}

__global__ void __launch_bounds__(kNT)
    ir_update_kernel(double* __restrict__ x64, int64_t p64, int64_t z64, const float* __restrict__ d32,
                     int64_t p32, int64_t z32, int64_t n0, int64_t n1, int64_t n2,
                     const DevScalars* s32) {
  const double scale = s32->scale;
  const RowRange rr = block_rows(n1 * n2);
  for (int64_t rho = rr.r0; rho < rr.r1; ++rho) {
    const int64_t o64 = row_offset(rho, n1, p64, z64);
    const int64_t o32 = row_offset(rho, n1, p32, z32);
    for (int64_t i = threadIdx.x; i < n0; i += kNT) x64[o64 + i] += scale * (double)d32[o32 + i];
  }
}

__global__ void __launch_bounds__(kNT)
    copy_kernel(const double* __restrict__ src, int64_t sp, int64_t sz, double* __restrict__ dst,
                int64_t dp, int64_t dz, int64_t n0, int64_t n1, int64_t n2) {
  const RowRange rr = block_rows(n1 * n2);
  for (int64_t rho = rr.r0; rho < rr.r1; ++rho) {
    const int64_t os = row_offset(rho, n1, sp, sz);
    const int64_t od = row_offset(rho, n1, dp, dz);
    for (int64_t i = threadIdx.x; i < n0; i += kNT) dst[od + i] = src[os + i];
  }
}

// dst = src + add (layouts may differ)
__global__ void __launch_bounds__(kNT)
    copy_shift_kernel(const double* __restrict__ src, int64_t sp, int64_t sz, double* __restrict__ dst,
                      int64_t dp, int64_t dz, int64_t n0, int64_t n1, int64_t n2, double add) {
  const RowRange rr = block_rows(n1 * n2);
  for (int64_t rho = rr.r0; rho < rr.r1; ++rho) {
    const int64_t os = row_offset(rho, n1, sp, sz);
    const int64_t od = row_offset(rho, n1, dp, dz);
    for (int64_t i = threadIdx.x; i < n0; i += kNT) dst[od + i] = src[os + i] + add;
  }
}

// dst = src; <src, src> -> bb, rr_stop = tol2 bb (a given right-hand side)
__global__ void __launch_bounds__(kNT)
    copy_norm_kernel(const double* __restrict__ src, int64_t sp, int64_t sz, double* __restrict__ dst,
                     int64_t dp, int64_t dz, int64_t n0, int64_t n1, int64_t n2, DevScalars* s, double tol2,
                     double* partials) {
  const RowRange rr = block_rows(n1 * n2);
  double dot = 0.0;
  for (int64_t rho = rr.r0; rho < rr.r1; ++rho) {
    const int64_t os = row_offset(rho, n1, sp, sz);
    const int64_t od = row_offset(rho, n1, dp, dz);
    for (int64_t i = threadIdx.x; i < n0; i += kNT) {
      const double v = src[os + i];
      dst[od + i] = v;
      dot += v * v;
    }
  }
  block_partial<kNT>(dot, (int)blockIdx.x, partials);
}

// out = base + sum_k coef_k v_k, all in one layout (k in increasing order)
__global__ void __launch_bounds__(kNT)
    combine_kernel(CombineTerms t, const double* base, double* out, int64_t pitch,
                   int64_t zpitch, int64_t n0, int64_t n1, int64_t n2) {
  const RowRange rr = block_rows(n1 * n2);
  for (int64_t rho = rr.r0; rho < rr.r1; ++rho) {
    const int64_t o = row_offset(rho, n1, pitch, zpitch);
    for (int64_t i = threadIdx.x; i < n0; i += kNT) {
      double acc = base[o + i];
      for (int k = 0; k < t.n; ++k) acc = __builtin_fma(t.coef[k], t.v[k][o + i], acc);
      out[o + i] = acc;
    }
  }
}

// Sums for the free energy: WELL = false, u + the scaled double well
// (u^2 - 1)^2 / 4; WELL = true, (u - wa)^2 (u - wb)^2. Also sum u and the
// squared forward differences (periodic).
template <bool WELL>
__global__ void __launch_bounds__(kNT)
    diagnostics_kernel(const double* __restrict__ u, int64_t pitch, int64_t zpitch, int dim,
                       int64_t n0, int64_t n1, int64_t n2, double* partials, unsigned int* ticket,
                       double* out3, double wa, double wb) {
  const RowRange rr = block_rows(n1 * n2);
  double m = 0.0, bulk = 0.0, grad = 0.0;
  for (int64_t rho = rr.r0; rho < rr.r1; ++rho) {
    const int64_t k = rho / n1, j = rho - k * n1;
    const int64_t o = k * zpitch + j * pitch;
    const int64_t jn = (j + 1 == n1) ? 0 : j + 1;
    const int64_t oy = k * zpitch + jn * pitch;
    const int64_t kn = (k + 1 == n2) ? 0 : k + 1;
    const int64_t oz = kn * zpitch + j * pitch;
    for (int64_t i = threadIdx.x; i < n0; i += kNT) {
      const double v = u[o + i];
      const int64_t in = (i + 1 == n0) ? 0 : i + 1;
      const double dx = u[o + in] - v;
      const double dy = u[oy + i] - v;
      double g = dx * dx + dy * dy;
      if (dim == 3) {
        const double dz = u[oz + i] - v;
        g += dz * dz;
      }
      m += v;
      if constexpr (WELL) {
        const double w = (v - wa) * (v - wb);
        bulk += w * w;
      } else {
        const double w = v * v - 1.0;
        bulk += 0.25 * w * w;
      }
      grad += g;
    }
  }
  __shared__ int is_last;
  const double bm = block_sum<kNT>(m);
  const double bb = block_sum<kNT>(bulk);
  const double bg = block_sum<kNT>(grad);
  const int nb = (int)gridDim.x;
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = bm;
    partials[nb + blockIdx.x] = bb;
    partials[2 * nb + blockIdx.x] = bg;
    const unsigned int prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = prev == (unsigned int)nb - 1u;
  }
  __syncthreads();
  if (!is_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double t[3];
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kNT)
      s += __hip_atomic_load(partials + c * nb + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t[c] = block_sum<kNT>(s);
  }
  if (threadIdx.x == 0) {
    out3[0] = t[0];
    out3[1] = t[1];
    out3[2] = t[2];
    __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

int elem_blocks(const int64_t* n) {
  const int64_t rows = n[1] * n[2];
  return (int)(rows < kElemBlocks ? rows : kElemBlocks);
}


// t /= (lx_i + ly_j + lz_k)^2 : the squared Dirichlet Laplacian in its
// sine eigenbasis (lz = 0 in 2D)
template <typename T>
__global__ void __launch_bounds__(kNT)
    pc_scale_kernel(T* __restrict__ t, int64_t pitch, int64_t zpitch, int64_t n0, int64_t n1, int64_t n2,
                    const double* __restrict__ lx, const double* __restrict__ ly, const double* __restrict__ lz,
                    const DevScalars* s) {
  if (s->done) return;
  const RowRange rr = block_rows(n1 * n2);
  for (int64_t rho = rr.r0; rho < rr.r1; ++rho) {
    const int64_t k = rho / n1, j = rho - k * n1;
    const double lyz = ly[j] + (lz ? lz[k] : 0.0);
    T* row = t + k * zpitch + j * pitch;
    for (int64_t i = threadIdx.x; i < n0; i += kNT) {
      const double l = lx[i] + lyz;
      row[i] = (T)((double)row[i] / (l * l));
    }
  }
}

// rz = <r, z>; beta = rz / rz_old (0 when starting), rz_old = rz
template <typename T>
__global__ void __launch_bounds__(kNT)
    pc_dot_kernel(const T* __restrict__ r, const T* __restrict__ z, int64_t pitch, int64_t zpitch, int64_t n0,
                  int64_t n1, int64_t n2, DevScalars* s, int start, double* partials) {
  if (s->done) return;
  const RowRange rr = block_rows(n1 * n2);
  double dot = 0.0;
  for (int64_t rho = rr.r0; rho < rr.r1; ++rho) {
    const int64_t o = row_offset(rho, n1, pitch, zpitch);
    for (int64_t i = threadIdx.x; i < n0; i += kNT) dot += (double)r[o + i] * (double)z[o + i];
  }
  block_partial<kNT>(dot, (int)blockIdx.x, partials);
}

// S[j][k] = sqrt(2/(m+1)) sin(pi (j+1)(k+1)/(m+1)), the angle reduced
// exactly in integers; lam[k] = -(4/h^2) sin^2(pi (k+1) / (2(m+1)))
template <typename T>
__global__ void __launch_bounds__(kNT) pc_init_kernel(T* __restrict__ S, double* __restrict__ lam, int64_t m, double h) {
  const int64_t tid = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kNT;
  const double c0 = sqrt(2.0 / (double)(m + 1));
  const int64_t period = 2 * (m + 1);
  if (S)
    for (int64_t e = tid; e < m * m; e += stride) {
      const int64_t j = e / m, k = e - j * m;
      const int64_t t = ((j + 1) * (k + 1)) % period;
      S[e] = (T)(c0 * sin(M_PI * (double)t / (double)(m + 1)));
    }
  for (int64_t k = tid; k < m; k += stride) {
    const double sk = sin(M_PI * (double)(k + 1) / (double)period);
    lam[k] = -4.0 / (h * h) * sk * sk;
  }
}

// The sine transform of length m split by its symmetry S(k, m-1-j) =
// (-1)^k S(k, j) (0-based; S(k, j) = sqrt(2/(m+1)) sin(pi (k+1)(j+1)/(m+1))):
// with u+_j = v_j + v_{m-1-j} (and the middle value when m is odd) in the
// first hp = ceil(m/2) entries and u-_j = v_j - v_{m-1-j} stored reversed in
// the last hm = floor(m/2), the transform's even rows are Fo u+ and its odd
// rows FeR u-. F holds Fo (hp x hp, Fo[a][b] = S(2a, b)) then FeR (hm x hm,
// FeR[a][c] = S(2a+1, hm-1-c)), column-major. lam lists the 1D eigenvalues
// in the order the transformed data takes: even k, then odd k.
template <typename T>
__global__ void __launch_bounds__(kNT) pc_init_split_kernel(T* __restrict__ F, double* __restrict__ lam, int64_t m,
                                                            double h) {
  const int64_t tid = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kNT;
  const double c0 = sqrt(2.0 / (double)(m + 1));
  const int64_t period = 2 * (m + 1);
  const int64_t hp = (m + 1) / 2, hm = m / 2;
  if (F) {
    for (int64_t e = tid; e < hp * hp; e += stride) {
      const int64_t b = e / hp, a = e - b * hp;
      const int64_t t = ((2 * a + 1) * (b + 1)) % period;
      F[e] = (T)(c0 * sin(M_PI * (double)t / (double)(m + 1)));
    }
    for (int64_t e = tid; e < hm * hm; e += stride) {
      const int64_t c = e / hm, a = e - c * hm;
      const int64_t t = ((2 * a + 2) * (hm - c)) % period;
      F[hp * hp + e] = (T)(c0 * sin(M_PI * (double)t / (double)(m + 1)));
    }
  }
  for (int64_t i = tid; i < m; i += stride) {
    const int64_t k = i < hp ? 2 * i : 2 * (i - hp) + 1;
    const double sk = sin(M_PI * (double)(k + 1) / (double)period);
    lam[i] = -4.0 / (h * h) * sk * sk;
  }
}

// (v_j, v_{n-1-j}) -> (v_j + v_{n-1-j}, v_j - v_{n-1-j}) along one axis for
// j < floor(n/2), at every position of the other two; the middle value (n
// odd) is copied. The same step folds data before the split transform and
// unfolds it after the transposed one. in may equal out (each pair is read
// and written by one thread).
template <typename T>
__global__ void __launch_bounds__(kNT)
    butterfly_kernel(const T* in, T* out, int64_t p, int64_t zp, int64_t n0, int64_t n1, int64_t n2, int axis) {
  const int64_t n = axis == 0 ? n0 : (axis == 1 ? n1 : n2);
  const int64_t s = axis == 0 ? 1 : (axis == 1 ? p : zp);
  const int64_t hm = n / 2, hp = (n + 1) / 2;
  // the other two extents and strides; the first is the unit-stride one
  // unless the axis itself is x (then pairs along x are the fastest index)
  const int64_t oa = axis == 0 ? n1 : n0, ob = axis == 2 ? n1 : n2;
  const int64_t sa = axis == 0 ? p : 1, sb = axis == 2 ? p : zp;
  const int64_t total = hp * oa * ob;
  for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < total; e += (int64_t)gridDim.x * kNT) {
    int64_t j, ia, ib;
    if (axis == 0) {
      j = e % hp;
      const int64_t r = e / hp;
      ia = r % oa;
      ib = r / oa;
    } else {
      ia = e % oa;
      const int64_t r = e / oa;
      j = r % hp;
      ib = r / hp;
    }
    const int64_t base = ia * sa + ib * sb;
    if (j < hm) {
      const T x = in[base + j * s], y = in[base + (n - 1 - j) * s];
      out[base + j * s] = x + y;
      out[base + (n - 1 - j) * s] = x - y;
    } else {
      out[base + j * s] = in[base + j * s];
    }
  }
}

// Error-free transformations: a + b = s + e exactly (Knuth), a * b = p + e
// exactly (one FMA).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = __builtin_fma(a, b, -p);
}

__global__ void __launch_bounds__(kNT)
    resid_dd_kernel(const double* __restrict__ x, int64_t px, int64_t zx, const double* __restrict__ b,
                    double* __restrict__ r, int64_t pr, int64_t zr, int64_t n0, int64_t n1, int64_t n2,
                    const TapTable taps, DevScalars* s, int flag, double* partials) {
  const RowRange rr = block_rows(n1 * n2);
  double dot = 0.0;
  for (int64_t rho = rr.r0; rho < rr.r1; ++rho) {
    const int64_t k = rho / n1, j = rho - k * n1;
    const int64_t ox = k * zx + j * px, orr = k * zr + j * pr;
    for (int64_t i = threadIdx.x; i < n0; i += kNT) {
      double hi = 0.0, lo = 0.0;  // sum w x as hi + lo
      for (int t = 0; t < taps.n; ++t) {
        const double v = x[ox + i + taps.off[t][0] + taps.off[t][1] * px + taps.off[t][2] * zx];
        double p, pe, sum, se;
        two_prod(taps.w[t], v, p, pe);
        two_sum(hi, p, sum, se);
        hi = sum;
        lo += pe + se;
      }
      double d, de;
      two_sum(b[orr + i], -hi, d, de);
      const double res = d + (de - lo);
      r[orr + i] = res;
      dot += res * res;
    }
  }
  block_partial<kNT>(dot, (int)blockIdx.x, partials);
}

// Second half of every grid reduction here and in the sweeps (one block):
// the total of the partials, in slot order, finalised into DevScalars.
template <int FK>
__global__ void __launch_bounds__(kNT) finish_kernel(FinArgs f) {
  DevScalars* s = f.s;
  if (f.skip_if_done && s->done) return;
  const double total = sum_partials<kNT>(f.partials, f.n);
  if (threadIdx.x != 0) return;
  if constexpr (FK == FIN_RESID) {
    s->rr_true = total;
    if (f.flag) {
      // restart the recurrence from the true residual; flag 2 also sets
      // its stop to c <b, b> (a restart aims below the tolerance)
      s->rr = total;
      s->beta = 0.0;
      if (f.flag == 2) s->rr_stop = f.c * s->bb;
      s->done = (total <= s->rr_stop) ? 1 : 0;
    }
  } else if constexpr (FK == FIN_RHS) {
    s->bb = total;
    s->rr_stop = f.c * total;
  } else if constexpr (FK == FIN_UPDATE) {
    s->iter += 1;
    if (total <= s->rr_stop) s->done = 1;
    s->beta = total / s->rr;
    s->rr = total;
  } else if constexpr (FK == FIN_IR) {
    if (f.flag) {
      // beta = <r', r'> / <r_old, r_old> with r' the replaced residual;
      // the last update left beta = rr / rr_old and rr.
      s->beta = s->rr > 0.0 ? s->beta * (total / s->rr) : 0.0;
    } else {
      s->scale = sqrt(f.s64->rr_true);
      s->beta = 0.0;
    }
    s->rr = total;
    s->rr_stop = f.c * total;
    s->done = total > 0.0 ? 0 : 1;
  } else if constexpr (FK == FIN_PCDOT) {
    s->beta = (f.flag || !(s->rz > 0.0)) ? 0.0 : total / s->rz;
    s->rz = total;
    if (!(total > 0.0)) s->done = 2;  // the preconditioner lost positivity
  }
}

}  // namespace

int update_slots(const int64_t* n) { return elem_blocks(n); }

hipError_t launch_finish(int fk, const FinArgs& f, hipStream_t st) {
  switch (fk) {
    case FIN_RESID: hipLaunchKernelGGL(finish_kernel<FIN_RESID>, dim3(1), dim3(kNT), 0, st, f); break;
    case FIN_RHS: hipLaunchKernelGGL(finish_kernel<FIN_RHS>, dim3(1), dim3(kNT), 0, st, f); break;
    case FIN_UPDATE: hipLaunchKernelGGL(finish_kernel<FIN_UPDATE>, dim3(1), dim3(kNT), 0, st, f); break;
    case FIN_IR: hipLaunchKernelGGL(finish_kernel<FIN_IR>, dim3(1), dim3(kNT), 0, st, f); break;
    case FIN_PCDOT: hipLaunchKernelGGL(finish_kernel<FIN_PCDOT>, dim3(1), dim3(kNT), 0, st, f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

namespace {

hipError_t finish(int fk, DevScalars* s, const double* partials, int n, double c, int flag, int skip,
                  hipStream_t st, const DevScalars* s64 = nullptr) {
  const hipError_t e = hipGetLastError();  // the reducing kernel's launch
  if (e != hipSuccess) return e;
  FinArgs f;
  f.s = s;
  f.s64 = s64;
  f.partials = partials;
  f.n = n;
  f.c = c;
  f.flag = flag;
  f.skip_if_done = skip;
  return launch_finish(fk, f, st);
}

}  // namespace

hipError_t launch_resid_dd(const double* x, const Layout& lx, const double* b, double* r, const Layout& lr,
                           const int64_t* n, const TapTable& taps, DevScalars* s, int flag, double c,
                           double* partials, hipStream_t st) {
  const int nb = elem_blocks(n);
  hipLaunchKernelGGL(resid_dd_kernel, dim3(nb), dim3(kNT), 0, st, x, lx.pitch, lx.zpitch, b, r, lr.pitch, lr.zpitch,
                     n[0], n[1], n[2], taps, s, flag, partials);
  return finish(FIN_RESID, s, partials, nb, c, flag, 0, st);
}

hipError_t launch_pc_init_split(int dtype, void* F, double* lam, int64_t m, double h, hipStream_t st) {
  int64_t nb = (m * m / 2 + kNT - 1) / kNT;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  if (dtype == SC_F64)
    hipLaunchKernelGGL(pc_init_split_kernel<double>, dim3((unsigned)nb), dim3(kNT), 0, st, (double*)F, lam, m, h);
  else
    hipLaunchKernelGGL(pc_init_split_kernel<float>, dim3((unsigned)nb), dim3(kNT), 0, st, (float*)F, lam, m, h);
  return hipGetLastError();
}

hipError_t launch_butterfly(int dtype, const void* in, void* out, const Layout& lay, const int64_t* n, int axis,
                            hipStream_t st) {
  const int64_t na = n[axis];
  const int64_t total = (na + 1) / 2 * (n[0] * n[1] * n[2] / na);
  int64_t nb = (total + kNT - 1) / kNT;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  if (dtype == SC_F64)
    hipLaunchKernelGGL(butterfly_kernel<double>, dim3((unsigned)nb), dim3(kNT), 0, st, (const double*)in,
                       (double*)out, lay.pitch, lay.zpitch, n[0], n[1], n[2], axis);
  else
    hipLaunchKernelGGL(butterfly_kernel<float>, dim3((unsigned)nb), dim3(kNT), 0, st, (const float*)in, (float*)out,
                       lay.pitch, lay.zpitch, n[0], n[1], n[2], axis);
  return hipGetLastError();
}

hipError_t launch_pc_init(int dtype, void* S, double* lam, int64_t m, double h, hipStream_t st) {
  int64_t nb = (m * m + kNT - 1) / kNT;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  if (dtype == SC_F64)
    hipLaunchKernelGGL(pc_init_kernel<double>, dim3((unsigned)nb), dim3(kNT), 0, st, (double*)S, lam, m, h);
  else
    hipLaunchKernelGGL(pc_init_kernel<float>, dim3((unsigned)nb), dim3(kNT), 0, st, (float*)S, lam, m, h);
  return hipGetLastError();
}

hipError_t launch_pc_scale(int dtype, void* t, const Layout& lay, const int64_t* n, const double* lx,
                           const double* ly, const double* lz, const DevScalars* s, hipStream_t st) {
  const int nb = elem_blocks(n);
  if (dtype == SC_F64)
    hipLaunchKernelGGL(pc_scale_kernel<double>, dim3(nb), dim3(kNT), 0, st, (double*)t, lay.pitch, lay.zpitch, n[0],
                       n[1], n[2], lx, ly, lz, s);
  else
    hipLaunchKernelGGL(pc_scale_kernel<float>, dim3(nb), dim3(kNT), 0, st, (float*)t, lay.pitch, lay.zpitch, n[0],
                       n[1], n[2], lx, ly, lz, s);
  return hipGetLastError();
}

hipError_t launch_pc_dot(int dtype, const void* r, const void* z, const Layout& lay, const int64_t* n,
                         DevScalars* s, int start, double* partials, hipStream_t st) {
  const int nb = elem_blocks(n);
  if (dtype == SC_F64)
    hipLaunchKernelGGL(pc_dot_kernel<double>, dim3(nb), dim3(kNT), 0, st, (const double*)r, (const double*)z,
                       lay.pitch, lay.zpitch, n[0], n[1], n[2], s, start, partials);
  else
    hipLaunchKernelGGL(pc_dot_kernel<float>, dim3(nb), dim3(kNT), 0, st, (const float*)r, (const float*)z,
                       lay.pitch, lay.zpitch, n[0], n[1], n[2], s, start, partials);
  return finish(FIN_PCDOT, s, partials, nb, 0.0, start, 1, st);
}

hipError_t launch_cg_update(int dtype, void* x, void* r, const void* p, const void* q,
                            const Layout& lay, const int64_t* n, DevScalars* s, const double* pq_partials,
                            int pc, double* partials, bool fin, hipStream_t st) {
  const int nb = elem_blocks(n);
  if (dtype == SC_F64) {
    hipLaunchKernelGGL(cg_update_kernel<double>, dim3(nb), dim3(kNT), 0, st, (double*)x, (double*)r,
                       (const double*)p, (const double*)q, lay.pitch, lay.zpitch, n[0], n[1], n[2], s,
                       pq_partials, pc, partials);
  } else {
    hipLaunchKernelGGL(cg_update_kernel<float>, dim3(nb), dim3(kNT), 0, st, (float*)x, (float*)r,
                       (const float*)p, (const float*)q, lay.pitch, lay.zpitch, n[0], n[1], n[2], s,
                       pq_partials, pc, partials);
  }
  if (!fin) return hipGetLastError();
  return finish(FIN_UPDATE, s, partials, nb, 0.0, 0, 1, st);
}

hipError_t launch_ir_prepare(const double* r64, const Layout& l64, float* r32, float* d32,
                             const Layout& l32, const int64_t* n, DevScalars* s64, DevScalars* s32,
                             double inner_tol2, int keep_direction, double* partials, hipStream_t st) {
  const int nb = elem_blocks(n);
  hipLaunchKernelGGL(ir_prepare_kernel, dim3(nb), dim3(kNT), 0, st, r64, l64.pitch, l64.zpitch, r32,
                     d32, l32.pitch, l32.zpitch, n[0], n[1], n[2], s64, s32, inner_tol2, keep_direction,
                     partials);
  return finish(FIN_IR, s32, partials, nb, inner_tol2, keep_direction, 0, st, s64);
}

hipError_t launch_ir_update(double* x64, const Layout& l64, const float* d32, const Layout& l32,
                            const int64_t* n, const DevScalars* s32, hipStream_t st) {
  const int nb = elem_blocks(n);
  hipLaunchKernelGGL(ir_update_kernel, dim3(nb), dim3(kNT), 0, st, x64, l64.pitch, l64.zpitch, d32,
                     l32.pitch, l32.zpitch, n[0], n[1], n[2], s32);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, int64_t sp, int64_t sz, double* dst, int64_t dp, int64_t dz,
                       const int64_t* n, hipStream_t st) {
  const int nb = elem_blocks(n);
  hipLaunchKernelGGL(copy_kernel, dim3(nb), dim3(kNT), 0, st, src, sp, sz, dst, dp, dz, n[0], n[1],
                     n[2]);
  return hipGetLastError();
}

hipError_t launch_diagnostics(const double* u, int64_t pitch, int64_t zpitch, int dim,
                              const int64_t* n, double* partials, unsigned int* ticket, double* out3,
                              hipStream_t st, const double* well) {
  const int nb = elem_blocks(n);
  if (well)
    hipLaunchKernelGGL(diagnostics_kernel<true>, dim3(nb), dim3(kNT), 0, st, u, pitch, zpitch, dim, n[0], n[1],
                       n[2], partials, ticket, out3, well[0], well[1]);
  else
    hipLaunchKernelGGL(diagnostics_kernel<false>, dim3(nb), dim3(kNT), 0, st, u, pitch, zpitch, dim, n[0], n[1],
                       n[2], partials, ticket, out3, 0.0, 0.0);
  return hipGetLastError();
}

hipError_t launch_copy_shift(const double* src, int64_t sp, int64_t sz, double* dst, int64_t dp, int64_t dz,
                             const int64_t* n, double add, hipStream_t st) {
  const int nb = elem_blocks(n);
  hipLaunchKernelGGL(copy_shift_kernel, dim3(nb), dim3(kNT), 0, st, src, sp, sz, dst, dp, dz, n[0], n[1], n[2],
                     add);
  return hipGetLastError();
}

hipError_t launch_copy_norm(const double* src, int64_t sp, int64_t sz, double* dst, int64_t dp, int64_t dz,
                            const int64_t* n, DevScalars* s, double tol2, double* partials, hipStream_t st) {
  const int nb = elem_blocks(n);
  hipLaunchKernelGGL(copy_norm_kernel, dim3(nb), dim3(kNT), 0, st, src, sp, sz, dst, dp, dz, n[0], n[1], n[2], s,
                     tol2, partials);
  return finish(FIN_RHS, s, partials, nb, tol2, 0, 0, st);
}

hipError_t launch_combine(const CombineTerms& t, const double* base, double* out, const Layout& lay,
                          const int64_t* n, hipStream_t st) {
  if (t.n < 0 || t.n > kMaxCombine) return hipErrorInvalidValue;
  const int nb = elem_blocks(n);
  hipLaunchKernelGGL(combine_kernel, dim3(nb), dim3(kNT), 0, st, t, base, out, lay.pitch, lay.zpitch, n[0], n[1],
                     n[2]);
  return hipGetLastError();
}

}  // namespace sc
