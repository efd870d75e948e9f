// Batched biharmonic BVPs on small 2D grids (Sec. 3.3), one workgroup per
// problem with every vector on chip.
//
// A grid of up to 512 row segments of 8 points (4096 unknowns; 7936 values
// with its ring) fits one workgroup of 512 threads, each holding one segment
// of x, r, p and b in registers; the search direction is shared through an
// LDS tile that carries a zero ring of the stencil's radius, so each
// iteration is one stencil pass over LDS and two workgroup reductions, with
// no kernel launches or host round trips. The solve is the
// same textbook CG as the large-grid path: x0 from u, b = f - A g_ring,
// stop on the recurrence residual, confirm on the true residual b - A x
// (restarting from it if the check fails), all in FP64. Reductions run in a
// fixed order, so a problem's result does not depend on the rest of the
// batch.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace sc {

namespace {

constexpr int kNT = 512;
constexpr int kWaves = kNT / 64;
constexpr int kSeg = 8;            // consecutive points of a row per thread
constexpr int kMaxTile = 7936;     // LDS tile (unknowns plus ring), doubles: 62 KB
static_assert(kSeg * kNT == kSmallMaxPoints && kMaxTile == kSmallMaxTile, "limits");
constexpr int kMaxRestarts = 64;   // true-residual restarts before giving up

// Sum of a and b over the workgroup, in a fixed order, returned to every
// thread (one barrier). Consecutive calls must alternate between two `red`
// buffers: a buffer is rewritten only after the barrier of the call in
// between, which every thread reaches after reading it.
__device__ __forceinline__ void wg_sum2(double& a, double& b, double (*red)[2]) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = a;
    red[wave][1] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    sa += red[w][0];
    sb += red[w][1];
  }
  a = sa;
  b = sb;
}

// Thread t owns a segment of kSeg consecutive points of one row (the last
// segment of a row may be partly empty). The LDS tile has rows of
// W = ceil(n0 / kSeg) kSeg + 2R doubles, so each segment's stencil reads are
// 2R + 1 aligned row spans of kSeg + 2R values, loaded once into registers
// and shared by every tap of that row (a dense (2R+1)^2 weight table, zero
// where the stencil has no tap).
// The same for one value.
__device__ __forceinline__ double wg_sum1(double a, double (*red)[2]) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave][0] = a;
  __syncthreads();
  double sa = 0.0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) sa += red[w][0];
  return sa;
}

template <int R>
__global__ void __launch_bounds__(kNT) small_cg_kernel(const SmallDesc* __restrict__ descs, SmallTaps taps,
                                                       double tol2, long long max_iter,
                                                       SmallResult* __restrict__ results) {
  constexpr int D = 2 * R + 1;
  constexpr int SPAN = kSeg + 2 * R;
  __shared__ __attribute__((aligned(16))) double tile[kMaxTile];
  __shared__ double red2[2][kWaves][2];
  __shared__ double sw[D * D];
  const SmallDesc& d = descs[blockIdx.x];
  const int tid = threadIdx.x;
  const int n0 = d.n0, n1 = d.n1;
  const int spr = (n0 + kSeg - 1) / kSeg;  // segments per row
  const int W = spr * kSeg + 2 * R;
  const int H = n1 + 2 * R;
  for (int i = tid; i < D * D; i += kNT) sw[i] = 0.0;
  __syncthreads();
  if (tid < taps.n) sw[(taps.dy[tid] + R) * D + taps.dx[tid] + R] = d.w[tid];
  // the ring values of g (zero elsewhere) for b = f - A g_ring; g holds a
  // ring of width R only
  for (int i = tid; i < W * H; i += kNT) {
    const int ty = i / W - R, tx = i % W - R;
    const bool ring = (tx < 0 || tx >= n0 || ty < 0 || ty >= n1) && tx < n0 + R && ty < n1 + R;
    tile[i] = (ring && d.g) ? d.g[(int64_t)ty * d.pg + tx] : 0.0;
  }
  __syncthreads();

  const bool seg = tid < spr * n1;
  const int y = seg ? tid / spr : 0;
  const int x0 = seg ? (tid % spr) * kSeg : 0;
  bool valid[kSeg];
#pragma unroll
  for (int j = 0; j < kSeg; ++j) valid[j] = seg && x0 + j < n0;
  const int own = (y + R) * W + x0 + R;  // tile index of point 0 of the segment

  // q = A (tile) at the segment's points
  auto stencil = [&](double (&q)[kSeg]) {
#pragma unroll
    for (int j = 0; j < kSeg; ++j) q[j] = 0.0;
#pragma unroll
    for (int dy = 0; dy < D; ++dy) {
      double v[SPAN];
      const double2* row = reinterpret_cast<const double2*>(tile + (y + dy) * W + x0);
#pragma unroll
      for (int k = 0; k < SPAN / 2; ++k) {
        const double2 t = row[k];
        v[2 * k] = t.x;
        v[2 * k + 1] = t.y;
      }
#pragma unroll
      for (int dx = 0; dx < D; ++dx) {
        const double w = sw[dy * D + dx];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) q[j] = __builtin_fma(w, v[j + dx], q[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < kSeg; ++j)
      if (!valid[j]) q[j] = 0.0;
  };

  double x[kSeg], r[kSeg], p[kSeg], b[kSeg], q[kSeg];
  stencil(q);  // A g_ring
#pragma unroll
  for (int j = 0; j < kSeg; ++j) {
    const int64_t gx = x0 + j;
    b[j] = valid[j] ? d.f[(int64_t)y * d.pf + gx] - q[j] : 0.0;
    x[j] = valid[j] ? d.u[(int64_t)y * d.pu + gx] : 0.0;
  }
  __syncthreads();
  // the Krylov vectors see a zero ring
  for (int i = tid; i < W * H; i += kNT) tile[i] = 0.0;
  __syncthreads();

  int rb = 0;  // the reduction buffer of the next wg_sum2
  auto reduce2 = [&](double& a, double& c) {
    wg_sum2(a, c, red2[rb]);
    rb ^= 1;
  };
  auto reduce1 = [&](double a) {
    const double t = wg_sum1(a, red2[rb]);
    rb ^= 1;
    return t;
  };
  // q = A v for v in registers. Every call is followed by a reduction,
  // whose barrier orders these tile reads before the next writes.
  auto apply = [&](const double (&v)[kSeg], double (&out)[kSeg]) {
#pragma unroll
    for (int j = 0; j < kSeg; ++j)
      if (valid[j]) tile[own + j] = v[j];
    __syncthreads();
    stencil(out);
  };

  // true residual r = b - A x, <r, r>, <b, b>
  apply(x, q);
  double rr = 0.0, bb = 0.0;
#pragma unroll
  for (int j = 0; j < kSeg; ++j) {
    r[j] = b[j] - q[j];
    p[j] = r[j];
    rr += r[j] * r[j];
    bb += b[j] * b[j];
  }
  reduce2(rr, bb);
  const double rr_stop = tol2 * bb;
  double rr_true = rr;
  long long it = 0;
  int outer = 1, status = SC_OK;
  bool converged = rr_true <= rr_stop;
  // CG in its single-reduction form (Chronopoulos and Gear): each iteration
  // applies A to r (w = A r) and reduces <r, r> and <r, w> together; A p is
  // carried by the recurrence q = w + beta q. The same iterates as the
  // textbook form in exact arithmetic, with two barriers per iteration
  // instead of three. A true-residual restart starts p = r, q = w afresh.
  double w[kSeg];
  bool fresh = true;
  double gamma_old = rr, alpha = 0.0;
  while (!converged) {
    apply(r, w);
    double g = 0.0, dl = 0.0;
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
      g += r[j] * r[j];
      dl += r[j] * w[j];
    }
    reduce2(g, dl);
    if (g <= rr_stop && !fresh) {
      // confirm on the true residual; restart the recurrence from it if not
      apply(x, q);
      double rt = 0.0;
#pragma unroll
      for (int j = 0; j < kSeg; ++j) {
        r[j] = b[j] - q[j];
        rt += r[j] * r[j];
      }
      rt = reduce1(rt);
      rr_true = rt;
      ++outer;
      if (rt <= rr_stop) {
        converged = true;
      } else if (outer > kMaxRestarts) {
        status = SC_ENOTCONV;
        break;
      }
      fresh = true;
      continue;
    }
    if (it >= max_iter) {
      status = SC_ENOTCONV;
      break;
    }
    // beta = <r, r> / <r_old, r_old>; <p, A p> = <r, w> - beta <r, r> / alpha_old
    const double beta = fresh ? 0.0 : g / gamma_old;
    const double pq = fresh ? dl : dl - beta * g / alpha;
    if (!(pq > 0.0) || !__builtin_isfinite(pq)) {
      status = SC_EBREAKDOWN;
      break;
    }
    alpha = g / pq;
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
      p[j] = fresh ? r[j] : __builtin_fma(beta, p[j], r[j]);
      q[j] = fresh ? w[j] : __builtin_fma(beta, q[j], w[j]);
      x[j] = __builtin_fma(alpha, p[j], x[j]);
      r[j] = __builtin_fma(-alpha, q[j], r[j]);
    }
    gamma_old = g;
    fresh = false;
    ++it;
  }
  if (status != SC_OK) {
    // the true residual of the returned iterate
    apply(x, q);
    double rt = 0.0;
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
      const double e = b[j] - q[j];
      rt += e * e;
    }
    rt = reduce1(rt);
    rr_true = rt;
  }
#pragma unroll
  for (int j = 0; j < kSeg; ++j)
    if (valid[j]) d.u[(int64_t)y * d.pu + x0 + j] = x[j];
  if (tid == 0) {
    SmallResult& o = results[blockIdx.x];
    o.iter = it;
    o.rr_true = rr_true;
    o.bb = bb;
    o.status = status;
    o.outer = outer;
  }
}

}  // namespace

int small_class(int64_t n0, int64_t n1, int R) {
  if (n0 < 1 || n1 < 1 || R < 1 || R > 4) return -1;
  const int64_t spr = (n0 + kSeg - 1) / kSeg;
  if (spr * n1 > kNT || (spr * kSeg + 2 * R) * (n1 + 2 * R) > kMaxTile) return -1;
  return R - 1;
}

hipError_t launch_small_cg(const SmallDesc* descs, const SmallTaps& taps, int count, int cls, double tol2,
                           long long max_iter, SmallResult* results, hipStream_t st) {
  if (count < 1) return hipSuccess;
  if (cls != taps.R - 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)count), block(kNT);
  switch (cls) {
    case 0: hipLaunchKernelGGL(small_cg_kernel<1>, grid, block, 0, st, descs, taps, tol2, max_iter, results); break;
    case 1: hipLaunchKernelGGL(small_cg_kernel<2>, grid, block, 0, st, descs, taps, tol2, max_iter, results); break;
    case 2: hipLaunchKernelGGL(small_cg_kernel<3>, grid, block, 0, st, descs, taps, tol2, max_iter, results); break;
    case 3: hipLaunchKernelGGL(small_cg_kernel<4>, grid, block, 0, st, descs, taps, tol2, max_iter, results); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

sc_status solve_biharmonic_batch(const sc_stencil* op, const double* h, int32_t count, const sc_grid* f,
                                 const sc_grid* g, const sc_solve_opts* opts, sc_grid* u, sc_solve_stats* stats,
                                 hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  sc_status r;
  if (!op || !h || !f || !u || count < 0) {
    set_error("NULL operator, spacing or grid arrays, or a negative count");
    return SC_EINVAL;
  }
  if (op->dim != 2) {
    set_error("the batched solver takes 2D operators");
    return SC_EUNSUPPORTED;
  }
  if (count == 0) return SC_OK;
  sc_solve_opts o;
  fill_opts(opts, &o);
  if ((r = check_opts(o)) != SC_OK) return r;
  if (o.precision != SC_PREC_F64 || o.precond != SC_PC_NONE) {
    set_error("the batched solver runs plain CG in FP64");
    return SC_EUNSUPPORTED;
  }
  std::vector<SmallDesc> descs((size_t)count);
  SmallTaps taps{};
  for (int i = 0; i < count; ++i) {
    const sc_grid* gi = g ? &g[i] : nullptr;
    if (gi && !gi->data) gi = nullptr;
    if ((r = check_grid(&f[i], "f")) != SC_OK || (r = check_grid(&u[i], "u")) != SC_OK) return r;
    if (gi && (r = check_grid(gi, "g")) != SC_OK) return r;
    const bool same = f[i].dim == 2 && u[i].dim == 2 && f[i].n[0] == u[i].n[0] && f[i].n[1] == u[i].n[1] &&
                      (!gi || (gi->dim == 2 && gi->n[0] == u[i].n[0] && gi->n[1] == u[i].n[1]));
    if (!same || f[i].dtype != SC_F64 || u[i].dtype != SC_F64 || (gi && gi->dtype != SC_F64)) {
      set_error("problem %d: f, g and u must be 2D FP64 grids of one shape", i);
      return SC_EINVAL;
    }
    KStencil ks;
    if ((r = make_kstencil(op, h[i], &ks)) != SC_OK) return r;
    const TapTable tt = tap_table(ks);
    if (tt.n > kSmallTaps) {
      set_error("the batched solver takes at most %d taps", kSmallTaps);
      return SC_EUNSUPPORTED;
    }
    if (i == 0) {
      taps.n = tt.n;
      taps.R = ks.R;
      for (int t = 0; t < tt.n; ++t) {
        taps.dx[t] = tt.off[t][0];
        taps.dy[t] = tt.off[t][1];
      }
    } else {
      bool ok = tt.n == taps.n && ks.R == taps.R;
      for (int t = 0; ok && t < tt.n; ++t) ok = taps.dx[t] == tt.off[t][0] && taps.dy[t] == tt.off[t][1];
      if (!ok) {
        set_error("problem %d: the operator's taps changed with h", i);
        return SC_EINVAL;
      }
    }
    const int64_t n0 = u[i].n[0], n1 = u[i].n[1];
    const int R = ks.R;
    if (small_class(n0, n1, R) < 0) {
      set_error("problem %d: %lld x %lld unknowns do not fit one workgroup (at most %d rows of %d-point segments, "
                "%d values with the ring)", i, (long long)n0, (long long)n1, kNT, kSeg, kMaxTile);
      return SC_EUNSUPPORTED;
    }
    if (gi && gi->halo < R) {
      set_error("problem %d: g must carry a ring of width >= radius (%d < %d)", i, gi->halo, R);
      return SC_EINVAL;
    }
    SmallDesc& dd = descs[(size_t)i];
    dd.f = static_cast<const double*>(interior(&f[i]));
    dd.g = gi ? static_cast<const double*>(interior(gi)) : nullptr;
    dd.u = static_cast<double*>(interior(&u[i]));
    dd.pf = f[i].pitch[0];
    dd.pg = gi ? gi->pitch[0] : 0;
    dd.pu = u[i].pitch[0];
    dd.n0 = (int)n0;
    dd.n1 = (int)n1;
    for (int t = 0; t < tt.n; ++t) dd.w[t] = tt.w[t];
  }
  // One launch per register class (points per thread), so that a problem
  // always runs in the instantiation its own size selects and its result
  // cannot depend on the rest of the batch.
  auto cls = [&](const SmallDesc& q) { return small_class(q.n0, q.n1, taps.R); };
  std::vector<int> order;
  int first[5] = {0, 0, 0, 0, 0};
  for (int c = 0; c < 4; ++c) {
    first[c] = (int)order.size();
    for (int i = 0; i < count; ++i)
      if (cls(descs[(size_t)i]) == c) order.push_back(i);
  }
  first[4] = count;
  std::vector<SmallDesc> sorted((size_t)count);
  for (int k = 0; k < count; ++k) sorted[(size_t)k] = descs[(size_t)order[(size_t)k]];
  void* ddev = pool_alloc(sorted.size() * sizeof(SmallDesc));
  void* rdev = pool_alloc((size_t)count * sizeof(SmallResult));
  struct Release {
    hipStream_t st;
    void* a;
    void* b;
    ~Release() {
      (void)hipStreamSynchronize(st);
      pool_free(a);
      pool_free(b);
    }
  } rel{st, ddev, rdev};
  if (!ddev || !rdev) {
    set_error("device allocation failed");
    return SC_ENOMEM;
  }
  SC_HIP_CHECK(hipMemcpyAsync(ddev, sorted.data(), sorted.size() * sizeof(SmallDesc), hipMemcpyHostToDevice, st));
  const double tol2 = o.tol * o.tol;
  const auto* dp = static_cast<const SmallDesc*>(ddev);
  auto* rp = static_cast<SmallResult*>(rdev);
  const long long mi = (long long)o.max_iter;
  for (int c = 0; c < 4; ++c) {
    const int k0 = first[c], nk = first[c + 1] - first[c];
    if (nk == 0) continue;
    SC_HIP_CHECK(launch_small_cg(dp + k0, taps, nk, c, tol2, mi, rp + k0, st));
  }
  std::vector<SmallResult> sres((size_t)count), res((size_t)count);
  SC_HIP_CHECK(hipMemcpyAsync(sres.data(), rdev, sres.size() * sizeof(SmallResult), hipMemcpyDeviceToHost, st));
  SC_HIP_CHECK(hipStreamSynchronize(st));
  for (int k = 0; k < count; ++k) res[(size_t)order[(size_t)k]] = sres[(size_t)k];
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  sc_status worst = SC_OK;
  for (int i = 0; i < count; ++i) {
    const SmallResult& q = res[(size_t)i];
    if (stats) {
      stats[i].iterations = q.iter;
      stats[i].outer = q.outer;
      stats[i].bnorm = std::sqrt(q.bb);
      stats[i].rel_residual = q.bb > 0 ? std::sqrt(q.rr_true / q.bb) : 0.0;
      stats[i].seconds = secs;
    }
    if (q.status != SC_OK && worst == SC_OK) worst = (sc_status)q.status;
  }
  if (worst != SC_OK) set_error("at least one problem of the batch did not converge (see its statistics)");
  return worst;
}

}  // namespace sc
