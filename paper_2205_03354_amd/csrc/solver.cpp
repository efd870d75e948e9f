// Krylov drivers: textbook CG (FP64), FP32 CG inside FP64 iterative
// refinement, the biharmonic boundary-value problem and the Cahn-Hilliard
// step. The host only launches kernels and reads the 128-byte scalar block
// every `check_every` iterations; every vector operation and every
// reduction runs on the GPU.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "internal.hpp"

namespace sc {

// ------------------------------------------------------------------ pool
namespace {

std::mutex g_pool_mu;
std::multimap<std::pair<int, size_t>, void*> g_free;      // (device, bytes) -> block
std::map<void*, std::pair<int, size_t>> g_owned;           // block -> (device, bytes)

}  // namespace

void* pool_alloc(size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  bytes = (bytes + 4095) & ~(size_t)4095;
  {
    std::lock_guard<std::mutex> g(g_pool_mu);
    auto it = g_free.lower_bound({dev, bytes});
    if (it != g_free.end() && it->first.first == dev && it->first.second <= 2 * bytes) {
      void* p = it->second;
      g_free.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_pool_mu);
  g_owned[p] = {dev, bytes};
  return p;
}

void pool_free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(g_pool_mu);
  auto it = g_owned.find(p);
  if (it == g_owned.end()) return;
  g_free.insert({it->second, p});
}

namespace {

size_t esize(int dtype) { return dtype == SC_F64 ? 8 : 4; }

// A zeroed workspace vector: `base` addresses the interior (0,0,0) element,
// which is 256-byte aligned, as is every row.
struct DevVec {
  void* alloc = nullptr;
  void* base = nullptr;
  Layout lay;
  int dtype = SC_F64;
};

// Returns workspace to the pool when a call ends, after the stream has
// drained (the pool is shared by every stream of the process).
struct VecGuard {
  hipStream_t st = nullptr;
  std::vector<void*> raw;
  ~VecGuard() {
    if (!raw.empty()) (void)hipStreamSynchronize(st);
    for (auto* r : raw) pool_free(r);
  }
};

sc_status make_vec(int dim, const int64_t* n, int halo, int dtype, hipStream_t st, DevVec* v,
                   VecGuard* guard) {
  const int64_t es = (int64_t)esize(dtype);
  const int64_t align_e = 256 / es;
  const int64_t pitch = (n[0] + 2 * halo + align_e - 1) / align_e * align_e;
  const int64_t rows = n[1] + 2 * halo;
  const int64_t zp = pitch * rows;
  const int64_t planes = dim == 3 ? n[2] + 2 * halo : 1;
  const size_t bytes = (size_t)(zp * planes * es) + 256;
  void* p = pool_alloc(bytes);
  if (!p) {
    set_error("device workspace allocation of %zu bytes failed", bytes);
    return SC_ENOMEM;
  }
  guard->raw.push_back(p);
  v->alloc = p;
  v->dtype = dtype;
  v->lay.pitch = pitch;
  v->lay.zpitch = zp;
  v->lay.halo = halo;
  const int64_t pad = (256 - (halo * es) % 256) % 256;
  const int64_t off_e = (dim == 3 ? halo * zp : 0) + halo * pitch + halo;
  v->base = static_cast<char*>(p) + pad + off_e * es;
  SC_HIP_CHECK(hipMemsetAsync(p, 0, bytes, st));
  return SC_OK;
}

// Scalars: one device block per solve level plus a pinned host mirror.
struct Ctx {
  hipStream_t st = nullptr;
  DevScalars* d64 = nullptr;
  DevScalars* d32 = nullptr;
  DevScalars* h64 = nullptr;
  DevScalars* h32 = nullptr;
  double* partials = nullptr;
};

DevScalars* pinned_scalars() {
  thread_local DevScalars* p = nullptr;
  if (!p) {
    if (hipHostMalloc((void**)&p, 2 * sizeof(DevScalars), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
  }
  return p;
}

sc_status read_scalars(Ctx& c, bool both) {
  SC_HIP_CHECK(hipMemcpyAsync(c.h64, c.d64, sizeof(DevScalars), hipMemcpyDeviceToHost, c.st));
  if (both) SC_HIP_CHECK(hipMemcpyAsync(c.h32, c.d32, sizeof(DevScalars), hipMemcpyDeviceToHost, c.st));
  SC_HIP_CHECK(hipStreamSynchronize(c.st));
  return SC_OK;
}

SweepLaunch sweep_on(int kind, const KStencil& ks, bool periodic, int dtype, const int64_t* n) {
  SweepLaunch L;
  L.kind = kind;
  L.ks = &ks;
  L.periodic = periodic;
  L.dtype = dtype;
  L.n[0] = n[0];
  L.n[1] = n[1];
  L.n[2] = n[2];
  return L;
}

void set_in(SweepLaunch& L, const DevVec& v) {
  L.in = v.base;
  L.pin = v.lay.pitch;
  L.zin = v.lay.zpitch;
}
void set_in2(SweepLaunch& L, const DevVec& v) {
  L.in2 = v.base;
  L.pin2 = v.lay.pitch;
  L.zin2 = v.lay.zpitch;
}
void set_aux(SweepLaunch& L, const DevVec& v) {
  L.aux = v.base;
  L.paux = v.lay.pitch;
  L.zaux = v.lay.zpitch;
}
void set_out(SweepLaunch& L, const DevVec& v) {
  L.out = v.base;
  L.pout = v.lay.pitch;
  L.zout = v.lay.zpitch;
}
void set_out2(SweepLaunch& L, const DevVec& v) {
  L.out2 = v.base;
  L.pout2 = v.lay.pitch;
  L.zout2 = v.lay.zpitch;
}

bool aligned16(const void* p, int64_t pitch, int64_t zpitch, int64_t es, bool three_d) {
  if (!p) return true;
  return (uintptr_t)p % 16 == 0 && (pitch * es) % 16 == 0 && (!three_d || (zpitch * es) % 16 == 0);
}

// Launch a sweep after deriving the alignment flags from its pointers.
sc_status launch(SweepLaunch L, hipStream_t st) {
  const int64_t es = (int64_t)esize(L.dtype);
  const bool d3 = L.ks->dim == 3;
  L.in_aligned = aligned16(L.in, L.pin, L.zin, es, d3) && aligned16(L.in2, L.pin2, L.zin2, es, d3) &&
                 aligned16(L.aux, L.paux, L.zaux, es, d3);
  L.vec_store = aligned16(L.out, L.pout, L.zout, es, d3) && aligned16(L.out2, L.pout2, L.zout2, es, d3);
  const hipError_t e = launch_sweep(L, st);
  if (e == hipErrorInvalidValue) return SC_EUNSUPPORTED;
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return SC_EDEVICE;
  }
  return SC_OK;
}

// CG iterations until the recurrence converges (done = 1), breaks down
// (done = 2) or `cap` iterations have been performed. Requires the scalars
// to hold a fresh (re)start (rr, beta = 0, done = 0) and r = b - A x.
sc_status cg_iterate(const KStencil& ks, bool periodic, int dtype, const int64_t* n, DevVec& x, DevVec& r,
                     DevVec* p, int& cur, DevVec& q, DevScalars* d, DevScalars* h, Ctx& c, int64_t cap,
                     int check_every) {
  const int64_t start = h->iter;
  while (true) {
    const int64_t left = cap - (h->iter - start);
    if (left <= 0) return SC_OK;
    const int64_t k_run = std::min<int64_t>(check_every, left);
    for (int64_t k = 0; k < k_run; ++k) {
      SweepLaunch L = sweep_on(K_CGDIR, ks, periodic, dtype, n);
      set_in(L, r);
      set_in2(L, p[cur]);
      set_out(L, p[1 - cur]);
      set_out2(L, q);
      L.scal = d;
      L.partials = c.partials;
      sc_status s = launch(L, c.st);
      if (s != SC_OK) return s;
      SC_HIP_CHECK(launch_cg_update(dtype, x.base, r.base, p[1 - cur].base, q.base, x.lay, n, d,
                                    c.partials, c.st));
      cur = 1 - cur;
    }
    SC_HIP_CHECK(hipMemcpyAsync(h, d, sizeof(DevScalars), hipMemcpyDeviceToHost, c.st));
    SC_HIP_CHECK(hipStreamSynchronize(c.st));
    if (h->done != 0) return SC_OK;
  }
}

// True residual r = b - A x; flag = 1 also restarts the CG recurrence.
sc_status residual(const KStencil& ks, bool periodic, const int64_t* n, DevVec& x, DevVec& b, DevVec& r,
                   DevScalars* d, Ctx& c, int flag) {
  SweepLaunch L = sweep_on(K_RESID, ks, periodic, SC_F64, n);
  set_in(L, x);
  set_aux(L, b);
  set_out(L, r);
  L.scal = d;
  L.partials = c.partials;
  L.flag = flag;
  return launch(L, c.st);
}

// Plain FP64 CG on A x = b; b's scalars (bb, rr_stop) are set.
sc_status solve_f64(const KStencil& ks, bool periodic, int dim, const int64_t* n, DevVec& x, DevVec& b,
                    const sc_solve_opts& o, Ctx& c, VecGuard& g, sc_solve_stats* stats) {
  DevVec r, p[2], q;
  sc_status s;
  if ((s = make_vec(dim, n, x.lay.halo, SC_F64, c.st, &r, &g)) != SC_OK) return s;
  if ((s = make_vec(dim, n, x.lay.halo, SC_F64, c.st, &p[0], &g)) != SC_OK) return s;
  if ((s = make_vec(dim, n, x.lay.halo, SC_F64, c.st, &p[1], &g)) != SC_OK) return s;
  if ((s = make_vec(dim, n, x.lay.halo, SC_F64, c.st, &q, &g)) != SC_OK) return s;
  int cur = 0;
  int outer = 0;
  int stalled = 0;
  double best = HUGE_VAL;
  sc_status result = SC_OK;
  while (true) {
    if ((s = residual(ks, periodic, n, x, b, r, c.d64, c, 1)) != SC_OK) return s;
    ++outer;
    if ((s = read_scalars(c, false)) != SC_OK) return s;
    if (c.h64->rr_true <= c.h64->rr_stop) break;
    if (c.h64->iter >= o.max_iter) {
      result = SC_ENOTCONV;
      set_error("CG did not reach the tolerance in %lld iterations", (long long)o.max_iter);
      break;
    }
    // restarts that no longer halve the true residual: the tolerance is
    // below the rounding floor of the operator
    stalled = (c.h64->rr_true > 0.25 * best) ? stalled + 1 : 0;
    best = std::min(best, c.h64->rr_true);
    if (stalled >= 3) {
      result = SC_ENOTCONV;
      set_error("CG stagnated at relative residual %g (rounding floor above tol)",
                std::sqrt(c.h64->rr_true / c.h64->bb));
      break;
    }
    s = cg_iterate(ks, periodic, SC_F64, n, x, r, p, cur, q, c.d64, c.h64, c, o.max_iter - c.h64->iter,
                   o.check_every);
    if (s != SC_OK) return s;
    if (c.h64->done == 2) {
      set_error("CG breakdown: <p, Ap> = %g after %lld iterations", c.h64->pq, (long long)c.h64->iter);
      result = SC_EBREAKDOWN;
      if ((s = residual(ks, periodic, n, x, b, r, c.d64, c, 0)) != SC_OK) return s;
      if ((s = read_scalars(c, false)) != SC_OK) return s;
      break;
    }
  }
  if (stats) {
    stats->iterations = c.h64->iter;
    stats->outer = outer;
    stats->bnorm = std::sqrt(c.h64->bb);
    stats->rel_residual = c.h64->bb > 0 ? std::sqrt(c.h64->rr_true / c.h64->bb) : 0.0;
  }
  return result;
}

// FP32 CG (FP64 reductions) inside FP64 iterative refinement.
sc_status solve_ir(const KStencil& ks, bool periodic, int dim, const int64_t* n, DevVec& x, DevVec& b,
                   const sc_solve_opts& o, Ctx& c, VecGuard& g, sc_solve_stats* stats) {
  DevVec r64, r32, d32, p[2], q;
  sc_status s;
  const int halo = x.lay.halo;
  if ((s = make_vec(dim, n, halo, SC_F64, c.st, &r64, &g)) != SC_OK) return s;
  if ((s = make_vec(dim, n, halo, SC_F32, c.st, &r32, &g)) != SC_OK) return s;
  if ((s = make_vec(dim, n, halo, SC_F32, c.st, &d32, &g)) != SC_OK) return s;
  if ((s = make_vec(dim, n, halo, SC_F32, c.st, &p[0], &g)) != SC_OK) return s;
  if ((s = make_vec(dim, n, halo, SC_F32, c.st, &p[1], &g)) != SC_OK) return s;
  if ((s = make_vec(dim, n, halo, SC_F32, c.st, &q, &g)) != SC_OK) return s;
  int cur = 0;
  int outer = 0;
  int stalled = 0;
  double best = HUGE_VAL;
  sc_status result = SC_OK;
  const double inner2 = o.inner_tol * o.inner_tol;
  while (true) {
    if ((s = residual(ks, periodic, n, x, b, r64, c.d64, c, 0)) != SC_OK) return s;
    ++outer;
    if ((s = read_scalars(c, true)) != SC_OK) return s;
    if (c.h64->rr_true <= c.h64->rr_stop) break;
    if (c.h32->iter >= o.max_iter) {
      result = SC_ENOTCONV;
      set_error("refinement did not reach the tolerance in %lld inner iterations", (long long)o.max_iter);
      break;
    }
    stalled = (c.h64->rr_true > 0.25 * best) ? stalled + 1 : 0;
    best = std::min(best, c.h64->rr_true);
    if (stalled >= 3) {
      result = SC_ENOTCONV;
      set_error("refinement stagnated at relative residual %g", std::sqrt(c.h64->rr_true / c.h64->bb));
      break;
    }
    SC_HIP_CHECK(launch_ir_prepare((const double*)r64.base, r64.lay, (float*)r32.base, (float*)d32.base,
                                   r32.lay, n, c.d64, c.d32, inner2, c.partials, c.st));
    const int64_t before = c.h32->iter;
    s = cg_iterate(ks, periodic, SC_F32, n, d32, r32, p, cur, q, c.d32, c.h32, c, o.max_iter - c.h32->iter,
                   o.check_every);
    if (s != SC_OK) return s;
    if (c.h32->done == 2 && c.h32->iter == before) {
      set_error("FP32 CG breakdown at the first inner iteration (<p, Ap> = %g)", c.h32->pq);
      result = SC_EBREAKDOWN;
      break;
    }
    SC_HIP_CHECK(launch_ir_update((double*)x.base, x.lay, (const float*)d32.base, d32.lay, n, c.d64, c.st));
  }
  if (stats) {
    stats->iterations = c.h32->iter;
    stats->outer = outer;
    stats->bnorm = std::sqrt(c.h64->bb);
    stats->rel_residual = c.h64->bb > 0 ? std::sqrt(c.h64->rr_true / c.h64->bb) : 0.0;
  }
  return result;
}

int64_t grid_bytes(const sc_grid* g) {
  const int64_t h = g->halo;
  const int64_t es = (int64_t)esize(g->dtype);
  if (g->dim == 3)
    return ((g->n[2] - 1 + 2 * h) * g->pitch[1] + (g->n[1] - 1 + 2 * h) * g->pitch[0] + g->n[0] + 2 * h) * es;
  return ((g->n[1] - 1 + 2 * h) * g->pitch[0] + g->n[0] + 2 * h) * es;
}

}  // namespace

// Validation shared by the entry points.
sc_status check_grid(const sc_grid* g, const char* what) {
  if (!g || !g->data) {
    set_error("%s: NULL grid or data", what);
    return SC_EINVAL;
  }
  if (g->dim != 2 && g->dim != 3) {
    set_error("%s: dim must be 2 or 3 (got %d)", what, g->dim);
    return SC_EINVAL;
  }
  if (g->dtype != SC_F64 && g->dtype != SC_F32) {
    set_error("%s: unknown dtype %d", what, g->dtype);
    return SC_EINVAL;
  }
  if (g->halo < 0 || g->n[0] < 1 || g->n[1] < 1 || g->n[2] < 1 || (g->dim == 2 && g->n[2] != 1)) {
    set_error("%s: bad extents (%lld, %lld, %lld) or halo %d", what, (long long)g->n[0], (long long)g->n[1],
              (long long)g->n[2], g->halo);
    return SC_EINVAL;
  }
  if (g->pitch[0] < g->n[0] + 2 * g->halo ||
      (g->dim == 3 && g->pitch[1] < g->pitch[0] * (g->n[1] + 2 * g->halo))) {
    set_error("%s: pitch too small", what);
    return SC_EINVAL;
  }
  return SC_OK;
}

void* interior(const sc_grid* g) {
  const int64_t h = g->halo;
  const int64_t es = (int64_t)esize(g->dtype);
  const int64_t off = (g->dim == 3 ? h * g->pitch[1] : 0) + h * g->pitch[0] + h;
  return static_cast<char*>(g->data) + off * es;
}

bool overlaps(const sc_grid* a, const sc_grid* b) {
  const char* a0 = static_cast<const char*>(a->data);
  const char* b0 = static_cast<const char*>(b->data);
  return a0 < b0 + grid_bytes(b) && b0 < a0 + grid_bytes(a);
}

static bool same_shape(const sc_grid* a, const sc_grid* b) {
  return a->dim == b->dim && a->n[0] == b->n[0] && a->n[1] == b->n[1] && a->n[2] == b->n[2];
}

sc_status apply_composed(const sc_stencil* s, double h, const sc_grid* in, sc_grid* out, sc_bc bc,
                         hipStream_t st) {
  sc_status r;
  if (!s) {
    set_error("NULL stencil");
    return SC_EINVAL;
  }
  if ((r = check_grid(in, "in")) != SC_OK || (r = check_grid(out, "out")) != SC_OK) return r;
  if (!same_shape(in, out) || in->dtype != out->dtype) {
    set_error("in and out must share dim, n and dtype");
    return SC_EINVAL;
  }
  if (s->dim != in->dim) {
    set_error("stencil is %dD but the grid is %dD", s->dim, in->dim);
    return SC_EINVAL;
  }
  if (bc != SC_BC_PERIODIC && bc != SC_BC_HALO) {
    set_error("unknown boundary mode %d", (int)bc);
    return SC_EINVAL;
  }
  if (overlaps(in, out)) {
    set_error("in and out overlap in memory");
    return SC_EINVAL;
  }
  KStencil ks;
  if ((r = make_kstencil(s, h, &ks)) != SC_OK) return r;
  const int rad = sc_stencil_radius(s);
  if (bc == SC_BC_HALO && in->halo < rad) {
    set_error("halo mode needs in->halo >= radius (%d < %d)", in->halo, rad);
    return SC_EINVAL;
  }
  SweepLaunch L = sweep_on(K_APPLY, ks, bc == SC_BC_PERIODIC, in->dtype, in->n);
  L.in = interior(in);
  L.pin = in->pitch[0];
  L.zin = in->pitch[1];
  L.out = interior(out);
  L.pout = out->pitch[0];
  L.zout = out->pitch[1];
  return launch(L, st);
}

namespace {

sc_status init_ctx(Ctx& c, hipStream_t st, const KStencil& ks, const int64_t* n, VecGuard& g,
                   const KStencil* ks2 = nullptr) {
  c.st = st;
  DevScalars* h = pinned_scalars();
  if (!h) {
    set_error("pinned host allocation failed");
    return SC_ENOMEM;
  }
  c.h64 = h;
  c.h32 = h + 1;
  void* d = pool_alloc(2 * sizeof(DevScalars));
  if (!d) {
    set_error("device allocation failed");
    return SC_ENOMEM;
  }
  g.raw.push_back(d);
  c.d64 = static_cast<DevScalars*>(d);
  c.d32 = c.d64 + 1;
  SC_HIP_CHECK(hipMemsetAsync(d, 0, 2 * sizeof(DevScalars), st));
  std::memset(c.h64, 0, 2 * sizeof(DevScalars));
  int slots = kElemBlocks;
  for (int dt : {SC_F64, SC_F32}) {
    SweepLaunch L = sweep_on(K_CGDIR, ks, true, dt, n);
    slots = std::max(slots, sweep_blocks(L));
    if (ks2) {
      SweepLaunch L2 = sweep_on(K_CGDIR, *ks2, true, dt, n);
      slots = std::max(slots, sweep_blocks(L2));
    }
  }
  void* p = pool_alloc((size_t)slots * 3 * sizeof(double));
  if (!p) {
    set_error("device allocation failed");
    return SC_ENOMEM;
  }
  g.raw.push_back(p);
  c.partials = static_cast<double*>(p);
  return SC_OK;
}

void fill_opts(const sc_solve_opts* in, sc_solve_opts* o) {
  sc_solve_opts_default(o);
  if (in) *o = *in;
  if (!(o->tol > 0)) o->tol = 1e-10;
  if (o->max_iter <= 0) o->max_iter = 10000000;
  if (!(o->inner_tol > 0)) o->inner_tol = 1e-4;
  if (o->check_every <= 0) o->check_every = 64;
}

}  // namespace

sc_status solve_biharmonic(const sc_stencil* op, double h, const sc_grid* f, const sc_grid* gr,
                           const sc_solve_opts* opts, sc_grid* u, sc_solve_stats* stats, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  sc_status r;
  if (!op) {
    set_error("NULL operator");
    return SC_EINVAL;
  }
  if ((r = check_grid(f, "f")) != SC_OK || (r = check_grid(u, "u")) != SC_OK) return r;
  if (gr && (r = check_grid(gr, "g")) != SC_OK) return r;
  if (!same_shape(f, u) || (gr && !same_shape(gr, u))) {
    set_error("f, g and u must share dim and n");
    return SC_EINVAL;
  }
  if (f->dtype != SC_F64 || u->dtype != SC_F64 || (gr && gr->dtype != SC_F64)) {
    set_error("solver grids must be FP64");
    return SC_EINVAL;
  }
  if (op->dim != u->dim) {
    set_error("operator is %dD but the grid is %dD", op->dim, u->dim);
    return SC_EINVAL;
  }
  sc_solve_opts o;
  fill_opts(opts, &o);
  if (o.precision != SC_PREC_F64 && o.precision != SC_PREC_F32_IR) {
    set_error("unknown precision %d", o.precision);
    return SC_EINVAL;
  }
  KStencil ks;
  if ((r = make_kstencil(op, h, &ks)) != SC_OK) return r;
  const int rad = sc_stencil_radius(op);
  if (gr && gr->halo < rad) {
    set_error("g must carry a ring of width >= radius (%d < %d)", gr->halo, rad);
    return SC_EINVAL;
  }
  const int64_t* n = u->n;
  const int dim = u->dim;
  VecGuard g;
  g.st = st;
  Ctx c;
  if ((r = init_ctx(c, st, ks, n, g)) != SC_OK) return r;
  DevVec x, b, zero;
  if ((r = make_vec(dim, n, ks.R, SC_F64, st, &x, &g)) != SC_OK) return r;
  if ((r = make_vec(dim, n, ks.R, SC_F64, st, &b, &g)) != SC_OK) return r;
  SC_HIP_CHECK(launch_copy((const double*)interior(u), u->pitch[0], u->pitch[1], (double*)x.base,
                           x.lay.pitch, x.lay.zpitch, n, st));
  // b = f - A g_ring
  SweepLaunch L = sweep_on(K_BVPRHS, ks, false, SC_F64, n);
  if (gr) {
    L.in = interior(gr);
    L.pin = gr->pitch[0];
    L.zin = gr->pitch[1];
  } else {
    if ((r = make_vec(dim, n, ks.R, SC_F64, st, &zero, &g)) != SC_OK) return r;
    set_in(L, zero);
  }
  L.aux = interior(f);
  L.paux = f->pitch[0];
  L.zaux = f->pitch[1];
  set_out(L, b);
  L.scal = c.d64;
  L.partials = c.partials;
  L.c2 = o.tol * o.tol;
  if ((r = launch(L, st)) != SC_OK) return r;
  sc_status res = o.precision == SC_PREC_F64 ? solve_f64(ks, false, dim, n, x, b, o, c, g, stats)
                                             : solve_ir(ks, false, dim, n, x, b, o, c, g, stats);
  if (res == SC_OK || res == SC_ENOTCONV || res == SC_EBREAKDOWN) {
    SC_HIP_CHECK(launch_copy((const double*)x.base, x.lay.pitch, x.lay.zpitch, (double*)interior(u), u->pitch[0],
                             u->pitch[1], n, st));
    SC_HIP_CHECK(hipStreamSynchronize(st));
  }
  if (stats)
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return res;
}

sc_status ch_step(const sc_stencil* lap, const sc_ch_params* prm, const sc_solve_opts* opts, sc_grid* u,
                  sc_solve_stats* stats, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  sc_status r;
  if (!lap || !prm) {
    set_error("NULL Laplacian or parameters");
    return SC_EINVAL;
  }
  if ((r = check_grid(u, "u")) != SC_OK) return r;
  if (u->dtype != SC_F64) {
    set_error("u must be FP64");
    return SC_EINVAL;
  }
  if (lap->dim != u->dim || lap->hpow != 2) {
    set_error("lap must be a %dD second-derivative stencil (hpow 2)", u->dim);
    return SC_EINVAL;
  }
  if (!(prm->h > 0) || !(prm->dt > 0) || !(prm->eps >= 0) || !std::isfinite(prm->S)) {
    set_error("invalid Cahn-Hilliard parameters");
    return SC_EINVAL;
  }
  sc_solve_opts o;
  fill_opts(opts, &o);
  const int dim = u->dim;
  const int64_t* n = u->n;
  // A = I + dt eps^2 L o L - dt S L, composed exactly, combined once in
  // extended precision.
  sc_stencil* LL = nullptr;
  if ((r = compose(lap, lap, &LL)) != SC_OK) return r;
  std::map<std::array<int32_t, 3>, long double> wa;
  const long double h = prm->h;
  const long double cLL = (long double)prm->dt * prm->eps * prm->eps / (h * h * h * h);
  const long double cL = -(long double)prm->dt * prm->S / (h * h);
  wa[{0, 0, 0}] += 1.0L;
  for (size_t t = 0; t < LL->num.size(); ++t) wa[LL->off[t]] += cLL * (long double)LL->num[t] / LL->den;
  for (size_t t = 0; t < lap->num.size(); ++t) wa[lap->off[t]] += cL * (long double)lap->num[t] / lap->den;
  delete LL;
  std::vector<std::array<int32_t, 3>> offs;
  std::vector<long double> ws;
  for (auto& kv : wa) {
    offs.push_back(kv.first);
    ws.push_back(kv.second);
  }
  KStencil ksA, ksL;
  if ((r = make_kstencil(dim, offs, ws, &ksA)) != SC_OK) return r;
  if ((r = make_kstencil(lap, prm->h, &ksL)) != SC_OK) return r;
  VecGuard g;
  g.st = st;
  Ctx c;
  if ((r = init_ctx(c, st, ksA, n, g, &ksL)) != SC_OK) return r;
  DevVec x, b;
  if ((r = make_vec(dim, n, 0, SC_F64, st, &x, &g)) != SC_OK) return r;
  if ((r = make_vec(dim, n, 0, SC_F64, st, &b, &g)) != SC_OK) return r;
  SC_HIP_CHECK(launch_copy((const double*)interior(u), u->pitch[0], u->pitch[1], (double*)x.base,
                           x.lay.pitch, x.lay.zpitch, n, st));
  // rhs = u + dt L(u^3 - (1+S) u)
  SweepLaunch L = sweep_on(K_CHRHS, ksL, true, SC_F64, n);
  L.in = interior(u);
  L.pin = u->pitch[0];
  L.zin = u->pitch[1];
  set_out(L, b);
  L.scal = c.d64;
  L.partials = c.partials;
  L.c0 = prm->dt;
  L.c1 = 1.0 + prm->S;
  L.c2 = o.tol * o.tol;
  if ((r = launch(L, st)) != SC_OK) return r;
  sc_status res = o.precision == SC_PREC_F64 ? solve_f64(ksA, true, dim, n, x, b, o, c, g, stats)
                                             : solve_ir(ksA, true, dim, n, x, b, o, c, g, stats);
  if (res == SC_OK) {
    SC_HIP_CHECK(launch_copy((const double*)x.base, x.lay.pitch, x.lay.zpitch, (double*)interior(u), u->pitch[0],
                             u->pitch[1], n, st));
  }
  SC_HIP_CHECK(hipStreamSynchronize(st));
  if (stats)
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return res;
}

sc_status grid_diagnostics(const sc_grid* u, double h, double eps, double* mass, double* energy,
                           hipStream_t st) {
  sc_status r;
  if ((r = check_grid(u, "u")) != SC_OK) return r;
  if (u->dtype != SC_F64 || !(h > 0)) {
    set_error("diagnostics need an FP64 grid and h > 0");
    return SC_EINVAL;
  }
  VecGuard g;
  g.st = st;
  void* p = pool_alloc(kElemBlocks * 3 * sizeof(double));
  void* t = pool_alloc(256);
  if (!p || !t) {
    if (p) pool_free(p);
    if (t) pool_free(t);
    set_error("device allocation failed");
    return SC_ENOMEM;
  }
  g.raw.push_back(p);
  g.raw.push_back(t);
  SC_HIP_CHECK(hipMemsetAsync(t, 0, 256, st));
  double* out3 = reinterpret_cast<double*>(static_cast<char*>(t) + 64);
  SC_HIP_CHECK(launch_diagnostics((const double*)interior(u), u->pitch[0], u->pitch[1], u->dim, u->n,
                                  (double*)p, (unsigned int*)t, out3, st));
  double host[3];
  SC_HIP_CHECK(hipMemcpyAsync(host, out3, sizeof(host), hipMemcpyDeviceToHost, st));
  SC_HIP_CHECK(hipStreamSynchronize(st));
  const double hd = u->dim == 3 ? h * h * h : h * h;
  if (mass) *mass = hd * host[0];
  if (energy) *energy = hd * (host[1] + 0.5 * eps * eps * host[2] / (h * h));
  return SC_OK;
}

}  // namespace sc
