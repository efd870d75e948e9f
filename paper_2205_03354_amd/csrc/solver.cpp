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

#include "task.hpp"

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

size_t esize(int dtype) { return dtype == SC_F64 ? 8 : 4; }

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

static bool aligned16(const void* p, int64_t pitch, int64_t zpitch, int64_t es, bool three_d) {
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

// Rows are padded so that the sweeps' 16-byte chunk DMAs of a strip
// (64 x 16 bytes plus halo chunks) stay inside the row even where the strip
// runs past the last column: the padding is zero and feeds no output.
Layout make_layout(int dim, const int64_t* n, int halo, int dtype) {
  const int64_t es = (int64_t)esize(dtype);
  const int64_t align_e = 256 / es;
  const int64_t vpl = 16 / es;
  const int64_t txw = 64 * vpl;
  const int64_t ra = halo ? (halo + vpl - 1) / vpl * vpl : 0;
  int64_t width = n[0] + 2 * halo;
  if (halo) width = std::max<int64_t>(width, halo + (n[0] + txw - 1) / txw * txw + ra);
  Layout lay;
  lay.pitch = (width + align_e - 1) / align_e * align_e;
  lay.zpitch = lay.pitch * (n[1] + 2 * halo);
  lay.halo = halo;
  lay.halo_x = (int)ra;
  lay.xhi = lay.pitch - halo;
  (void)dim;
  return lay;
}

size_t vec_bytes(int dim, const int64_t* n, int halo, int dtype) {
  const Layout lay = make_layout(dim, n, halo, dtype);
  const int64_t planes = dim == 3 ? n[2] + 2 * halo : 1;
  const size_t raw = (size_t)(lay.zpitch * planes) * esize(dtype) + 256;
  return (raw + 4095) & ~(size_t)4095;
}

namespace {

int partial_slots(const TaskSpec& sp) {
  int slots = kElemBlocks;
  for (int dt : {SC_F64, SC_F32}) {
    SweepLaunch L = sweep_on(K_CGDIR, sp.ksA, true, dt, sp.n);
    slots = std::max(slots, sweep_blocks(L));
    if (sp.kind == TASK_CH) {
      SweepLaunch L2 = sweep_on(K_CHRHS, sp.ksL, true, dt, sp.n);
      slots = std::max(slots, sweep_blocks(L2));
    }
  }
  return slots;
}

// ------------------------------------------------------- pinned host slots
std::mutex g_pin_mu;
std::vector<DevScalars*> g_pin_free;

}  // namespace

DevScalars* pinned_pair_alloc() {
  std::lock_guard<std::mutex> g(g_pin_mu);
  if (g_pin_free.empty()) {
    constexpr int kPairs = 1024;
    DevScalars* arena = nullptr;
    if (hipHostMalloc((void**)&arena, sizeof(DevScalars) * 2 * kPairs, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    for (int i = kPairs - 1; i >= 0; --i) g_pin_free.push_back(arena + 2 * i);
  }
  DevScalars* p = g_pin_free.back();
  g_pin_free.pop_back();
  std::memset(p, 0, 2 * sizeof(DevScalars));
  return p;
}

void pinned_pair_free(DevScalars* p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(g_pin_mu);
  g_pin_free.push_back(p);
}

bool task_onchip(const TaskSpec& sp) {
  if (sp.kind != TASK_BVP || sp.dim != 2 || sp.o.precision != SC_PREC_F64 || sp.o.precond != SC_PC_NONE ||
      !sp.o.onchip)
    return false;
  return tap_table(sp.ksA).n <= kSmallTaps && small_class(sp.n[0], sp.n[1], sp.ksA.R) >= 0;
}

size_t task_footprint(const TaskSpec& sp) {
  const int halo = sp.kind == TASK_BVP ? sp.ksA.R : 0;
  if (task_onchip(sp)) return vec_bytes(sp.dim, sp.n, halo, SC_F64) + 4096;
  const bool f32 = sp.o.precision != SC_PREC_F64;
  size_t b = 0;
  const size_t v64 = vec_bytes(sp.dim, sp.n, halo, SC_F64);
  const size_t v32 = vec_bytes(sp.dim, sp.n, halo, SC_F32);
  if (f32)
    b = 6 * v64 + 5 * v32;  // x b r64 (+ p0 p1 q if it falls back to FP64) | r d p0 p1 q
  else
    b = 6 * v64;            // x b r p0 p1 q
  if (sp.kind == TASK_BVP && sp.o.precond == SC_PC_FASTPOISSON) {  // z and scratch, tables
    b += 2 * v64 + fastpoisson_bytes(sp.dim, sp.n, SC_F64);
    if (f32) b += 2 * v32 + fastpoisson_bytes(sp.dim, sp.n, SC_F32);
  }
  b += 4096 + (size_t)partial_slots(sp) * 3 * sizeof(double);
  return b;
}

// ------------------------------------------------------------------ task
SolveTask::~SolveTask() {
  if (st_ && !allocs_.empty()) (void)hipStreamSynchronize(st_);
  for (auto& gp : graph_)
    for (auto& g : gp)
      if (g) (void)hipGraphExecDestroy(g);
  for (void* p : allocs_) pool_free(p);
  if (h64_) pinned_pair_free(h64_);
}

sc_status SolveTask::make(Vec* v, int dtype) {
  const size_t bytes = vec_bytes(spec_.dim, spec_.n, halo_, dtype);
  void* p = pool_alloc(bytes);
  if (!p) {
    set_error("device workspace allocation of %zu bytes failed", bytes);
    return SC_ENOMEM;
  }
  allocs_.push_back(p);
  bytes_ += bytes;
  v->alloc = p;
  v->lay = make_layout(spec_.dim, spec_.n, halo_, dtype);
  const int64_t es = (int64_t)esize(dtype);
  const int64_t pad = (256 - (halo_ * es) % 256) % 256;
  const int64_t off_e = (spec_.dim == 3 ? halo_ * v->lay.zpitch : 0) + halo_ * v->lay.pitch + halo_;
  v->base = static_cast<char*>(p) + pad + off_e * es;
  SC_HIP_CHECK(hipMemsetAsync(p, 0, bytes, st_));
  return SC_OK;
}

sc_status SolveTask::init(const TaskSpec& spec, hipStream_t st) {
  spec_ = spec;
  st_ = st;
  periodic_ = spec.kind == TASK_CH || spec.kind == TASK_LIN;
  f32_ = spec.o.precision != SC_PREC_F64;
  ru_ = spec.o.precision == SC_PREC_F32_RU;
  restart_ = true;
  pc_ = spec.kind == TASK_BVP && spec.o.precond == SC_PC_FASTPOISSON;
  taps_ = tap_table(spec.ksA);
  halo_ = periodic_ ? 0 : spec.ksA.R;
  h64_ = pinned_pair_alloc();
  if (!h64_) {
    set_error("pinned host allocation failed");
    return SC_ENOMEM;
  }
  h32_ = h64_ + 1;
  onchip_ = task_onchip(spec);
  if (onchip_) {
    // x, the problem descriptor and the result; the kernel does the rest
    static_assert(sizeof(SmallResult) <= sizeof(DevScalars), "result slot");
    dev_block_ = pool_alloc(4096);
    if (!dev_block_) {
      set_error("device allocation failed");
      return SC_ENOMEM;
    }
    allocs_.push_back(dev_block_);
    bytes_ += 4096;
    sdesc_dev_ = static_cast<SmallDesc*>(dev_block_);
    sres_dev_ = reinterpret_cast<SmallResult*>(static_cast<char*>(dev_block_) + 2048);
    staps_.n = taps_.n;
    staps_.R = spec.ksA.R;
    for (int t = 0; t < taps_.n; ++t) {
      staps_.dx[t] = taps_.off[t][0];
      staps_.dy[t] = taps_.off[t][1];
      sdesc_.w[t] = taps_.w[t];
    }
    sc_status s;
    if ((s = make(&x_, SC_F64)) != SC_OK) return s;
    phase_ = P_NONE;
    return SC_OK;
  }
  const size_t slots = (size_t)partial_slots(spec_);
  const size_t blk = 2 * sizeof(DevScalars) + 256 + slots * 3 * sizeof(double);
  dev_block_ = pool_alloc(blk);
  if (!dev_block_) {
    set_error("device allocation failed");
    return SC_ENOMEM;
  }
  allocs_.push_back(dev_block_);
  bytes_ += (blk + 4095) & ~(size_t)4095;
  SC_HIP_CHECK(hipMemsetAsync(dev_block_, 0, 2 * sizeof(DevScalars), st_));
  d64_ = static_cast<DevScalars*>(dev_block_);
  d32s_ = d64_ + 1;
  partials_ = reinterpret_cast<double*>(static_cast<char*>(dev_block_) + 2 * sizeof(DevScalars) + 256);
  upd_partials_ = partials_ + slots;  // the update's partials (room for 3 x slots)
  sc_status s;
  if ((s = make(&x_, SC_F64)) != SC_OK || (s = make(&b_, SC_F64)) != SC_OK || (s = make(&r64_, SC_F64)) != SC_OK)
    return s;
  const int vt = f32_ ? SC_F32 : SC_F64;
  if (f32_) {
    if ((s = make(&r32_, SC_F32)) != SC_OK || (s = make(&d32_, SC_F32)) != SC_OK) return s;
  }
  if ((s = make(&p_[0], vt)) != SC_OK || (s = make(&p_[1], vt)) != SC_OK || (s = make(&q_, vt)) != SC_OK) return s;
  if (pc_ && (s = make_pc(f32_)) != SC_OK) return s;
  phase_ = P_NONE;
  return SC_OK;
}

sc_status SolveTask::make_pc(bool f32) {
  sc_status s;
  if (f32) {
    if ((s = make(&z32_, SC_F32)) != SC_OK || (s = make(&t32_, SC_F32)) != SC_OK) return s;
    return pc32_.init(spec_.dim, spec_.n, spec_.h, SC_F32, st_);
  }
  if ((s = make(&z64_, SC_F64)) != SC_OK || (s = make(&t64_, SC_F64)) != SC_OK) return s;
  return pc64_.init(spec_.dim, spec_.n, spec_.h, SC_F64, st_);
}

// z = M^-1 r and <r, z> (beta = <r, z> / <r_old, z_old>, or 0 when starting)
sc_status SolveTask::precondition(bool f32, int start) {
  sc_status s;
  if (f32) {
    if ((s = pc32_.apply(r32_.base, z32_.base, t32_.base, r32_.lay, d32s_, st_)) != SC_OK) return s;
    SC_HIP_CHECK(launch_pc_dot(SC_F32, r32_.base, z32_.base, r32_.lay, spec_.n, d32s_, start, partials_, st_));
    return SC_OK;
  }
  if ((s = pc64_.apply(r64_.base, z64_.base, t64_.base, r64_.lay, d64_, st_)) != SC_OK) return s;
  SC_HIP_CHECK(launch_pc_dot(SC_F64, r64_.base, z64_.base, r64_.lay, spec_.n, d64_, start, partials_, st_));
  return SC_OK;
}

sc_status SolveTask::sweep(int kind, int dtype, const KStencil& ks, const void* in, const Layout* lin,
                           const void* in2, const void* aux, void* out, void* out2, const Layout& lout, int flag,
                           double c0, double c1, double c2, DevScalars* scal, const GridView* in_view,
                           const GridView* aux_view, const double* fold) {
  SweepLaunch L = sweep_on(kind, ks, periodic_, dtype, spec_.n);
  if (fold) {
    L.fold = fold;
    L.fold_n = update_slots(spec_.n);
  }
  if (in_view) {
    L.in = in_view->p;
    L.pin = in_view->pitch;
    L.zin = in_view->zpitch;
  } else {
    L.in = in;
    L.pin = lin->pitch;
    L.zin = lin->zpitch;
  }
  // workspace vectors carry padded rows (see make_layout); views do not
  if (!periodic_ && !in_view && !aux_view) {
    L.x_range = true;
    L.in_xlo = -lin->halo_x;
    L.in_xhi = lin->xhi;
    L.aux_xhi = lout.xhi;
  }
  L.in2 = in2;
  L.pin2 = lout.pitch;
  L.zin2 = lout.zpitch;
  if (aux_view) {
    L.aux = aux_view->p;
    L.paux = aux_view->pitch;
    L.zaux = aux_view->zpitch;
  } else {
    L.aux = aux;
    L.paux = lout.pitch;
    L.zaux = lout.zpitch;
  }
  L.out = out;
  L.pout = lout.pitch;
  L.zout = lout.zpitch;
  L.out2 = out2;
  L.pout2 = lout.pitch;
  L.zout2 = lout.zpitch;
  L.scal = scal;
  L.partials = partials_;
  L.flag = flag;
  L.c0 = c0;
  L.c1 = c1;
  L.c2 = c2;
  return launch(L, st_);
}

// The host copies carry an iteration count of -1 until the copy has landed.
sc_status SolveTask::enqueue_read(bool both) {
  h64_->iter = -1;
  if (both) h32_->iter = -1;
  SC_HIP_CHECK(hipMemcpyAsync(h64_, d64_, sizeof(DevScalars), hipMemcpyDeviceToHost, st_));
  if (both) SC_HIP_CHECK(hipMemcpyAsync(h32_, d32s_, sizeof(DevScalars), hipMemcpyDeviceToHost, st_));
  return SC_OK;
}

// The true residual. With a boundary ring (the BVP) |A| |x| exceeds |b| by
// many orders in the interior (weights ~ 1/h^4, the solution O(1)), so an
// FP64 stencil sum would round the residual at ~1e-10 relative to |b| on
// 2048^2 grids; the ring-mode residual is summed in double-double instead.
sc_status SolveTask::enqueue_residual(int flag, double c) {
  if (!periodic_) {
    SC_HIP_CHECK(launch_resid_dd((const double*)x_.base, x_.lay, (const double*)b_.base, (double*)r64_.base, r64_.lay,
                                 spec_.n, taps_, d64_, flag, c, partials_, st_));
    return SC_OK;
  }
  return sweep(K_RESID, SC_F64, spec_.ksA, x_.base, &x_.lay, nullptr, b_.base, r64_.base, nullptr, x_.lay, flag, 0,
               0, c, d64_);
}

// K CG iterations (direction sweep + update each), replayed from a graph
// captured on first use, one graph per ping-pong parity of the p buffers.
sc_status SolveTask::enqueue_block(bool f32) {
  const int dtype = f32 ? SC_F32 : SC_F64;
  DevScalars* ds = f32 ? d32s_ : d64_;
  const DevScalars* hs = f32 ? h32_ : h64_;
  Vec& x = f32 ? d32_ : x_;
  Vec& r = f32 ? r32_ : r64_;
  const int gi = f32 ? 1 : 0;
  const int K = std::max(1, spec_.o.check_every);
  const int64_t left = spec_.o.max_iter - hs->iter;
  block_cur0_ = cur_;
  block_iter0_ = hs->iter;
  // One CG iteration. On grids of up to kFoldPoints points, where launches
  // rather than bytes set an iteration's time, the update's finish (beta,
  // stop test) is folded into the next iteration's direction sweep within a
  // block; the block's last update keeps its finish kernel, so the host
  // reads final scalars. (At 256^3 the one-block finish is about 1% of an
  // iteration and the fold's partial sums at every sweep block's start cost
  // as much; at 1024^2 folding makes CH steps 12-14% faster.) Results are
  // the same bit for bit either way.
  constexpr int64_t kFoldPoints = int64_t(1) << 23;
  const bool fold_ok = spec_.n[0] * spec_.n[1] * spec_.n[2] <= kFoldPoints;
  auto one = [&](bool fold, bool fin) -> sc_status {
    fold = fold && fold_ok;
    fin = fin || !fold_ok;
    sc_status s = sweep(K_CGDIR, dtype, spec_.ksA, r.base, &r.lay, p_[cur_].base, nullptr, p_[1 - cur_].base,
                        q_.base, r.lay, 0, 0, 0, 0, ds, nullptr, nullptr, fold ? upd_partials_ : nullptr);
    if (s != SC_OK) return s;
    SC_HIP_CHECK(launch_cg_update(dtype, x.base, r.base, p_[1 - cur_].base, q_.base, x.lay, spec_.n, ds, partials_,
                                  0, upd_partials_, fin, st_));
    cur_ = 1 - cur_;
    return SC_OK;
  };
  if (pc_) {
    // p = z + beta p; q = A p; alpha = <r, z> / <p, q>; x, r update; z = M^-1 r.
    // The transforms are library GEMMs that ignore the device stop flag,
    // so blocks are short and are not captured.
    Vec& z = f32 ? z32_ : z64_;
    const int64_t k_run = std::min<int64_t>(std::min(K, 4), left);
    for (int64_t k = 0; k < k_run; ++k) {
      sc_status s = sweep(K_CGDIR, dtype, spec_.ksA, z.base, &z.lay, p_[cur_].base, nullptr, p_[1 - cur_].base,
                          q_.base, r.lay, 1, 0, 0, 0, ds);
      if (s != SC_OK) return s;
      SC_HIP_CHECK(launch_cg_update(dtype, x.base, r.base, p_[1 - cur_].base, q_.base, x.lay, spec_.n, ds,
                                    partials_, 1, upd_partials_, true, st_));
      cur_ = 1 - cur_;
      if ((s = precondition(f32, 0)) != SC_OK) return s;
    }
    return enqueue_read(f32);
  }
  if (spec_.o.use_graph && left >= K) {
    hipGraphExec_t& ge = graph_[gi][cur_];
    const int cur0 = cur_;
    if (!ge) {
      SC_HIP_CHECK(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
      sc_status s = SC_OK;
      for (int k = 0; k < K && s == SC_OK; ++k) s = one(k > 0, k == K - 1);
      hipGraph_t captured = nullptr;
      const hipError_t e = hipStreamEndCapture(st_, &captured);
      cur_ = cur0;
      if (s != SC_OK) {
        if (captured) (void)hipGraphDestroy(captured);
        return s;
      }
      if (e != hipSuccess) {
        set_error("graph capture failed: %s", hipGetErrorString(e));
        return SC_EDEVICE;
      }
      const hipError_t ei = hipGraphInstantiate(&ge, captured, nullptr, nullptr, 0);
      (void)hipGraphDestroy(captured);
      if (ei != hipSuccess) {
        ge = nullptr;
        set_error("graph instantiation failed: %s", hipGetErrorString(ei));
        return SC_EDEVICE;
      }
    }
    SC_HIP_CHECK(hipGraphLaunch(ge, st_));
    cur_ = cur0 ^ (K & 1);
  } else {
    const int64_t k_run = std::min<int64_t>(K, left);
    for (int64_t k = 0; k < k_run; ++k) {
      sc_status s = one(k > 0, k == k_run - 1);
      if (s != SC_OK) return s;
    }
  }
  return enqueue_read(f32);
}

sc_status SolveTask::start(const GridView& u0, const GridView& f, const GridView* g) {
  SC_HIP_CHECK(launch_copy(u0.p, u0.pitch, u0.zpitch, (double*)x_.base, x_.lay.pitch, x_.lay.zpitch, spec_.n, st_));
  if (onchip_) {
    sdesc_.f = f.p;
    sdesc_.pf = f.pitch;
    sdesc_.g = g ? g->p : nullptr;
    sdesc_.pg = g ? g->pitch : 0;
    sdesc_.u = static_cast<double*>(x_.base);
    sdesc_.pu = x_.lay.pitch;
    sdesc_.n0 = (int)spec_.n[0];
    sdesc_.n1 = (int)spec_.n[1];
    SC_HIP_CHECK(hipMemcpyAsync(sdesc_dev_, &sdesc_, sizeof(SmallDesc), hipMemcpyHostToDevice, st_));
    SC_HIP_CHECK(launch_small_cg(sdesc_dev_, staps_, 1, small_class(spec_.n[0], spec_.n[1], spec_.ksA.R),
                                 spec_.o.tol * spec_.o.tol, (long long)spec_.o.max_iter, sres_dev_, st_));
    // the result lands in the (otherwise unused) FP32 host slot; iter < 0 until then
    SmallResult* hr = reinterpret_cast<SmallResult*>(h32_);
    __atomic_store_n(&hr->iter, -1LL, __ATOMIC_RELEASE);
    SC_HIP_CHECK(hipMemcpyAsync(hr, sres_dev_, sizeof(SmallResult), hipMemcpyDeviceToHost, st_));
    phase_ = P_ONCHIP;
    return SC_OK;
  }
  const double tol2 = spec_.o.tol * spec_.o.tol;
  sc_status s;
  if (spec_.kind == TASK_BVP) {
    // b = f - A g_ring (the zero ring of q when g is absent)
    GridView zero{(const double*)q_.base, q_.lay.pitch, q_.lay.zpitch};
    if (f32_) zero = GridView{(const double*)r64_.base, r64_.lay.pitch, r64_.lay.zpitch};
    const GridView& gv = g ? *g : zero;
    s = sweep(K_BVPRHS, SC_F64, spec_.ksA, nullptr, nullptr, nullptr, nullptr, b_.base, nullptr, b_.lay, 0, 0, 0,
              tol2, d64_, &gv, &f);
  } else if (spec_.kind == TASK_LIN) {
    // the given right-hand side and its norm
    SC_HIP_CHECK(launch_copy_norm(f.p, f.pitch, f.zpitch, (double*)b_.base, b_.lay.pitch, b_.lay.zpitch, spec_.n,
                                  d64_, tol2, partials_, st_));
    s = SC_OK;
  } else {
    // rhs = u + dt L(u^3 - (1+S) u), from x0 = u
    s = sweep(K_CHRHS, SC_F64, spec_.ksL, x_.base, &x_.lay, nullptr, nullptr, b_.base, nullptr, b_.lay, 0,
              spec_.dt, 1.0 + spec_.S, tol2, d64_);
  }
  if (s != SC_OK) return s;
  outer_ = 1;
  stalled_ = 0;
  best_ = HUGE_VAL;
  if (!f32_) {
    if ((s = enqueue_residual(1)) != SC_OK) return s;
    if (pc_ && (s = precondition(false, 1)) != SC_OK) return s;
    phase_ = P_CHECK64;
    return enqueue_read(false);
  }
  if ((s = enqueue_residual(0)) != SC_OK) return s;
  phase_ = P_OUTER;
  return enqueue_read(true);
}

sc_status SolveTask::restart(const GridView& u0, const GridView& f) {
  if (spec_.kind != TASK_LIN || !d64_) {
    set_error("only an initialised linear-solve task can be restarted");
    return SC_EINVAL;
  }
  // a mixed-precision task that fell back to FP64 keeps solving in FP64
  f32_ = spec_.o.precision != SC_PREC_F64 && !fell_back_;
  ru_ = f32_ && spec_.o.precision == SC_PREC_F32_RU;
  restart_ = true;
  cur_ = 0;
  block_cur0_ = 0;
  block_iter0_ = 0;
  pending_ = SC_OK;
  status_ = SC_OK;
  outer_ = 0;
  stalled_ = 0;
  best_ = 0.0;
  inner_start_ = 0;
  inner_keep_ = 0;
  stretch_best_ = 0.0;
  stretch_idle_ = 0;
  stats_ = sc_solve_stats{};
  SC_HIP_CHECK(hipMemsetAsync(dev_block_, 0, 2 * sizeof(DevScalars), st_));
  std::memset(h64_, 0, 2 * sizeof(DevScalars));
  phase_ = P_NONE;
  return start(u0, f, nullptr);
}

void SolveTask::finish(sc_status s) {
  status_ = s;
  phase_ = P_DONE;
  stats_.iterations = h64_->iter + (spec_.o.precision != SC_PREC_F64 ? h32_->iter : 0);
  stats_.outer = outer_;
  stats_.bnorm = std::sqrt(h64_->bb);
  stats_.rel_residual = h64_->bb > 0 ? std::sqrt(h64_->rr_true / h64_->bb) : 0.0;
}

// The FP32 stretches stopped reducing the FP64 residual (the operator is
// too ill-conditioned for an FP32 Krylov recurrence): continue with FP64 CG
// from the current x, in FP64 direction buffers allocated now.
sc_status SolveTask::fall_back_to_f64() {
  sc_status s;
  Vec p0, p1, q;
  if ((s = make(&p0, SC_F64)) != SC_OK || (s = make(&p1, SC_F64)) != SC_OK || (s = make(&q, SC_F64)) != SC_OK)
    return s;
  p_[0] = p0;
  p_[1] = p1;
  q_ = q;
  cur_ = 0;
  f32_ = false;
  fell_back_ = true;
  stalled_ = 0;
  best_ = HUGE_VAL;
  if (pc_ && (s = make_pc(false)) != SC_OK) return s;
  if ((s = enqueue_residual(1)) != SC_OK) return s;
  if (pc_ && (s = precondition(false, 1)) != SC_OK) return s;
  if ((s = enqueue_read(false)) != SC_OK) return s;
  phase_ = P_CHECK64;
  return SC_OK;
}

sc_status SolveTask::advance(bool* done) {
  *done = false;
  if (__atomic_load_n(&h64_->iter, __ATOMIC_ACQUIRE) < 0 || __atomic_load_n(&h32_->iter, __ATOMIC_ACQUIRE) < 0)
    return SC_OK;  // the last host copy has not landed yet: call again later
  const sc_solve_opts& o = spec_.o;
  sc_status s;
  auto stagnated = [&]() {
    stalled_ = (h64_->rr_true > 0.25 * best_) ? stalled_ + 1 : 0;
    best_ = std::min(best_, h64_->rr_true);
    return stalled_ >= 3;
  };
  switch (phase_) {
    case P_ONCHIP: {
      const SmallResult* hr = reinterpret_cast<const SmallResult*>(h32_);
      if (__atomic_load_n(&hr->iter, __ATOMIC_ACQUIRE) < 0) return SC_OK;  // not landed yet
      h64_->iter = hr->iter;
      h64_->bb = hr->bb;
      h64_->rr_true = hr->rr_true;
      outer_ = hr->outer;
      const sc_status st = (sc_status)hr->status;
      if (st == SC_ENOTCONV)
        set_error("CG did not reach the tolerance (relative residual %g after %lld iterations)",
                  hr->bb > 0 ? std::sqrt(hr->rr_true / hr->bb) : 0.0, hr->iter);
      else if (st == SC_EBREAKDOWN)
        set_error("CG breakdown: <p, Ap> <= 0 after %lld iterations", hr->iter);
      finish(st);
      break;
    }
    case P_CHECK64:
      if (h64_->rr_true <= o.tol * o.tol * h64_->bb) {  // the tolerance itself, not a restart's stop
        finish(SC_OK);
      } else if (h64_->iter >= o.max_iter) {
        set_error("CG did not reach the tolerance in %lld iterations", (long long)o.max_iter);
        finish(SC_ENOTCONV);
      } else if (stagnated()) {
        set_error("CG stagnated at relative residual %g (rounding floor above tol)",
                  std::sqrt(h64_->rr_true / h64_->bb));
        finish(SC_ENOTCONV);
      } else {
        if ((s = enqueue_block(false)) != SC_OK) return s;
        phase_ = P_ITER64;
      }
      break;
    case P_ITER64:
      if (h64_->done == 2) {
        set_error("CG breakdown: <p, Ap> = %g after %lld iterations", h64_->pq, (long long)h64_->iter);
        pending_ = SC_EBREAKDOWN;
        if ((s = enqueue_residual(0)) != SC_OK || (s = enqueue_read(false)) != SC_OK) return s;
        phase_ = P_FINAL;
      } else if (h64_->done == 1) {
        // the recurrence met the tolerance: confirm with the true residual,
        // and should CG go on from it, let that run aim at half the
        // tolerance (near the rounding floor a run that stops at the
        // tolerance itself barely moves the true residual)
        if ((s = enqueue_residual(2, 0.25 * o.tol * o.tol)) != SC_OK) return s;
        if (pc_ && (s = precondition(false, 1)) != SC_OK) return s;
        if ((s = enqueue_read(false)) != SC_OK) return s;
        ++outer_;
        phase_ = P_CHECK64;
      } else if (h64_->iter >= o.max_iter) {
        set_error("CG did not reach the tolerance in %lld iterations", (long long)o.max_iter);
        pending_ = SC_ENOTCONV;
        if ((s = enqueue_residual(0)) != SC_OK || (s = enqueue_read(false)) != SC_OK) return s;
        phase_ = P_FINAL;
      } else {
        if ((s = enqueue_block(false)) != SC_OK) return s;
      }
      break;
    case P_FINAL:
      finish(pending_);
      break;
    case P_OUTER:
      if (h64_->rr_true <= o.tol * o.tol * h64_->bb) {
        finish(SC_OK);
      } else if (h32_->iter >= o.max_iter) {
        set_error("refinement did not reach the tolerance in %lld inner iterations", (long long)o.max_iter);
        finish(SC_ENOTCONV);
      } else if (stagnated()) {
        return fall_back_to_f64();
      } else {
        const int keep = (ru_ && !restart_) ? 1 : 0;
        SC_HIP_CHECK(launch_ir_prepare((const double*)r64_.base, r64_.lay, (float*)r32_.base, (float*)d32_.base,
                                       r32_.lay, spec_.n, d64_, d32s_, o.inner_tol * o.inner_tol, keep, partials_,
                                       st_));
        if (pc_ && (s = precondition(true, keep ? 0 : 1)) != SC_OK) return s;
        restart_ = false;
        inner_keep_ = keep;
        inner_start_ = h32_->iter;
        stretch_best_ = HUGE_VAL;
        stretch_idle_ = 0;
        if ((s = enqueue_block(true)) != SC_OK) return s;
        phase_ = P_INNER;
      }
      break;
    case P_INNER: {
      const bool first_breakdown = h32_->done == 2 && h32_->iter == inner_start_ && !inner_keep_;
      bool end = h32_->done != 0 || h32_->iter >= o.max_iter;
      if (!end) {
        // a stretch whose FP32 residual has not halved in 8 blocks ends early
        if (h32_->rr < 0.25 * stretch_best_) {
          stretch_best_ = h32_->rr;
          stretch_idle_ = 0;
        } else if (++stretch_idle_ >= 8) {
          end = true;
        }
      }
      if (first_breakdown) {
        return fall_back_to_f64();  // FP32 lost positivity of <p, Ap> at once
      } else if (end) {
        // the latest direction sits in the buffer the executed iterations
        // of the last block wrote (the skipped ones did not toggle it)
        cur_ = block_cur0_ ^ (int)((h32_->iter - block_iter0_) & 1);
        if (h32_->done == 2) restart_ = true;  // a lost direction: restart from p = r
        SC_HIP_CHECK(launch_ir_update((double*)x_.base, x_.lay, (const float*)d32_.base, d32_.lay, spec_.n, d32s_,
                                      st_));
        if ((s = enqueue_residual(0)) != SC_OK || (s = enqueue_read(true)) != SC_OK) return s;
        ++outer_;
        phase_ = P_OUTER;
      } else {
        if ((s = enqueue_block(true)) != SC_OK) return s;
      }
      break;
    }
    default:
      break;
  }
  *done = phase_ == P_DONE;
  return SC_OK;
}

sc_status SolveTask::enqueue_copy_out(double* dst, int64_t pitch, int64_t zpitch) {
  SC_HIP_CHECK(launch_copy((const double*)x_.base, x_.lay.pitch, x_.lay.zpitch, dst, pitch, zpitch, spec_.n, st_));
  return SC_OK;
}

// ---------------------------------------------------------- validation
namespace {

int64_t grid_bytes(const sc_grid* g) {
  const int64_t h = g->halo;
  const int64_t es = (int64_t)esize(g->dtype);
  if (g->dim == 3)
    return ((g->n[2] - 1 + 2 * h) * g->pitch[1] + (g->n[1] - 1 + 2 * h) * g->pitch[0] + g->n[0] + 2 * h) * es;
  return ((g->n[1] - 1 + 2 * h) * g->pitch[0] + g->n[0] + 2 * h) * es;
}

}  // namespace

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

GridView view_of(const sc_grid* g) {
  return GridView{static_cast<const double*>(interior(g)), g->pitch[0], g->pitch[1]};
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
  std::shared_ptr<void> cached;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->cached_h == h && s->cached_ks) cached = s->cached_ks;
  }
  if (!cached) {
    auto fresh = std::make_shared<KStencil>();
    if ((r = make_kstencil(s, h, fresh.get())) != SC_OK) return r;
    cached = fresh;
    std::lock_guard<std::mutex> g(s->mu);
    s->cached_h = h;
    s->cached_ks = cached;
  }
  const KStencil& ks = *static_cast<const KStencil*>(cached.get());
  const int rad = ks.R;  // the radius the kernel reads
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

// nonzero taps of a stencil, weights num / (den h^p) rounded as the sweeps
// round them (extended precision, then double, then the grid's dtype)
template <typename T>
int vc_taps(const sc_stencil* s, double h, int W, int cap, int pad, int* off, T* w) {
  long double hp = 1.0L;
  for (int i = 0; i < std::abs(s->hpow); ++i) hp *= (long double)h;
  if (s->hpow < 0) hp = 1.0L / hp;
  int n = 0;
  for (size_t t = 0; t < s->num.size(); ++t) {
    if (s->num[t] == 0) continue;
    if (n == cap) return -1;
    off[n] = s->off[t][1] * W + s->off[t][0];
    w[n++] = (T)(double)((long double)s->num[t] / ((long double)s->den * hp));
  }
  while (n % pad) {  // pad with zero weights at the point itself
    off[n] = 0;
    w[n++] = T(0);
  }
  return n;
}

// The fused kernel takes terms of at most kVcMaxTapsA inner and kVcMaxTapsB
// outer taps (after padding to multiples of 4 and 2), rA + rB <= kVcMaxRing
// and rB <= kVcMaxOuterR.
// SCOMP_VARCOEF=twosweep keeps the two-sweep form (for comparisons).
bool varcoef_fusable(int nterms, const sc_stencil* const* inner, const sc_stencil* const* outer, int rA, int rB,
                     const int64_t* n) {
  if (const char* e = std::getenv("SCOMP_VARCOEF"))
    if (std::strcmp(e, "twosweep") == 0) return false;
  if (nterms > kVcMaxTerms || rB > kVcMaxOuterR || rA + rB > kVcMaxRing || (n[1] + 15) / 16 > 65535) return false;
  auto padded = [](const sc_stencil* s, int64_t pad) {
    int64_t c = 0;
    for (int64_t v : s->num) c += v != 0;
    return (c + pad - 1) / pad * pad;
  };
  for (int t = 0; t < nterms; ++t)
    if (padded(inner[t], 4) > kVcMaxTapsA || padded(outer[t], 2) > kVcMaxTapsB) return false;
  return true;
}

template <typename T>
hipError_t varcoef_fused(int nterms, const sc_stencil* const* inner, const sc_stencil* const* outer, double h, int rA,
                         int rB, const sc_grid* M, const sc_grid* in, sc_grid* out, bool per, hipStream_t st) {
  VcTerms<T> tm;
  tm.n = nterms;
  tm.RA = rA;
  tm.RB = rB;
  for (int t = 0; t < nterms; ++t) {
    tm.na[t] = vc_taps(inner[t], h, kVcPitchX, kVcMaxTapsA, 4, tm.aoff[t], tm.aw[t]);
    tm.nb[t] = vc_taps(outer[t], h, kVcPitchW, kVcMaxTapsB, 2, tm.boff[t], tm.bw[t]);
    if (tm.na[t] < 0 || tm.nb[t] < 0) return hipErrorInvalidValue;
  }
  return launch_varcoef_fused(in->dtype, interior(in), in->pitch[0], interior(M), M->pitch[0], interior(out),
                              out->pitch[0], in->n[0], in->n[1], per, &tm, st);
}

}  // namespace

// y = sum_t B_t(M * A_t(x)). On 2D grids with few, small terms one fused
// kernel does it (varcoef.hip). Otherwise, per term, one sweep writes
// w = M * A_t(x) on the grid plus the ring B_t reads (a library workspace),
// and one sweep applies B_t to w, writing (first term) or accumulating into y.
sc_status apply_varcoef(int nterms, const sc_stencil* const* inner, const sc_stencil* const* outer, double h,
                        const sc_grid* M, const sc_grid* in, sc_grid* out, sc_bc bc, hipStream_t st) {
  sc_status r;
  if (nterms < 1 || nterms > 16 || !inner || !outer) {
    set_error("nterms must be in 1..16 with inner and outer arrays");
    return SC_EINVAL;
  }
  if ((r = check_grid(in, "in")) != SC_OK || (r = check_grid(out, "out")) != SC_OK ||
      (r = check_grid(M, "mobility")) != SC_OK)
    return r;
  if (!same_shape(in, out) || !same_shape(in, M) || in->dtype != out->dtype || in->dtype != M->dtype) {
    set_error("in, out and the coefficient grid must share dim, n and dtype");
    return SC_EINVAL;
  }
  if (bc != SC_BC_PERIODIC && bc != SC_BC_HALO) {
    set_error("unknown boundary mode %d", (int)bc);
    return SC_EINVAL;
  }
  if (overlaps(in, out) || overlaps(M, out)) {
    set_error("out overlaps an input in memory");
    return SC_EINVAL;
  }
  int rA = 0, rB = 0;
  std::vector<KStencil> ka(nterms), kb(nterms);
  for (int t = 0; t < nterms; ++t) {
    if (!inner[t] || !outer[t] || inner[t]->dim != in->dim || outer[t]->dim != in->dim) {
      set_error("term %d: NULL stencil or dimension mismatch", t);
      return SC_EINVAL;
    }
    if ((r = make_kstencil(inner[t], h, &ka[t])) != SC_OK || (r = make_kstencil(outer[t], h, &kb[t])) != SC_OK)
      return r;
    rA = std::max(rA, ka[t].R);
    rB = std::max(rB, kb[t].R);
  }
  const bool per = bc == SC_BC_PERIODIC;
  if (!per && (in->halo < rA + rB || M->halo < rB)) {
    set_error("halo mode needs in->halo >= %d (inner + outer radius) and coefficient halo >= %d", rA + rB, rB);
    return SC_EINVAL;
  }
  const int dim = in->dim;
  if (dim == 2 && varcoef_fusable(nterms, inner, outer, rA, rB, in->n)) {
    const hipError_t e = in->dtype == SC_F64 ? varcoef_fused<double>(nterms, inner, outer, h, rA, rB, M, in, out, per, st)
                                             : varcoef_fused<float>(nterms, inner, outer, h, rA, rB, M, in, out, per, st);
    if (e != hipSuccess) {
      set_error("device error: %s", hipGetErrorString(e));
      return SC_EDEVICE;
    }
    return SC_OK;
  }
  const int wr = per ? 0 : rB;  // ring of the workspace
  int64_t ne[3] = {in->n[0], in->n[1], in->n[2]};
  for (int a = 0; a < dim; ++a) ne[a] += 2 * wr;
  const Layout lay = make_layout(dim, in->n, wr, in->dtype);
  const size_t bytes = vec_bytes(dim, in->n, wr, in->dtype);
  void* wbuf = pool_alloc(bytes);
  if (!wbuf) {
    set_error("workspace allocation of %zu bytes failed", bytes);
    return SC_ENOMEM;
  }
  const int64_t es = (int64_t)esize(in->dtype);
  const int64_t pad = (256 - (wr * es) % 256) % 256;
  const int64_t off_w = (dim == 3 ? wr * lay.zpitch : 0) + wr * lay.pitch + wr;
  char* w_int = static_cast<char*>(wbuf) + pad + off_w * es;  // workspace interior
  char* w_org = w_int - off_w * es;                            // its ring's first element
  auto shifted = [&](const sc_grid* g) {                       // interior moved back by the ring
    const int64_t o = (dim == 3 ? wr * g->pitch[1] : 0) + wr * g->pitch[0] + wr;
    return static_cast<const char*>(interior(g)) - o * es;
  };
  sc_status res = SC_OK;
  for (int t = 0; t < nterms && res == SC_OK; ++t) {
    SweepLaunch L1 = sweep_on(K_SCALE, ka[t], per, in->dtype, ne);
    L1.in = shifted(in);
    L1.pin = in->pitch[0];
    L1.zin = in->pitch[1];
    L1.aux = shifted(M);
    L1.paux = M->pitch[0];
    L1.zaux = M->pitch[1];
    L1.out = w_org;
    L1.pout = lay.pitch;
    L1.zout = lay.zpitch;
    if ((res = launch(L1, st)) != SC_OK) break;
    SweepLaunch L2 = sweep_on(t == 0 ? K_APPLY : K_ACCUM, kb[t], per, in->dtype, in->n);
    L2.in = w_int;
    L2.pin = lay.pitch;
    L2.zin = lay.zpitch;
    L2.out = interior(out);
    L2.pout = out->pitch[0];
    L2.zout = out->pitch[1];
    L2.aux = interior(out);
    L2.paux = out->pitch[0];
    L2.zaux = out->pitch[1];
    if (!per) {  // the workspace rows are padded (see make_layout); out is not
      L2.x_range = true;
      L2.in_xlo = -lay.halo_x;
      L2.in_xhi = lay.xhi;
      L2.aux_xhi = in->n[0];
    }
    res = launch(L2, st);
  }
  const hipError_t e = hipStreamSynchronize(st);  // the workspace goes back to the pool
  pool_free(wbuf);
  if (res == SC_OK && e != hipSuccess) {
    set_error("device error: %s", hipGetErrorString(e));
    res = SC_EDEVICE;
  }
  return res;
}

void fill_opts(const sc_solve_opts* in, sc_solve_opts* o) {
  sc_solve_opts_default(o);
  if (in) *o = *in;
  if (!(o->tol > 0)) o->tol = 1e-10;
  if (o->max_iter <= 0) o->max_iter = 10000000;
  if (!(o->inner_tol > 0)) o->inner_tol = o->precision == SC_PREC_F32_RU ? 0.1 : 1e-4;
  if (o->check_every <= 0) o->check_every = 64;
}

sc_status check_precision(int precision) {
  if (precision != SC_PREC_F64 && precision != SC_PREC_F32_IR && precision != SC_PREC_F32_RU) {
    set_error("unknown precision %d", precision);
    return SC_EINVAL;
  }
  return SC_OK;
}

sc_status check_opts(const sc_solve_opts& o) {
  if (o.precond != SC_PC_NONE && o.precond != SC_PC_FASTPOISSON) {
    set_error("unknown preconditioner %d", o.precond);
    return SC_EINVAL;
  }
  return check_precision(o.precision);
}

// The operator of one Cahn-Hilliard step, I + dt eps^2 L o L - dt S L,
// composed exactly and combined once in extended precision.
sc_status lap_operator(const sc_stencil* lap, long double cI, long double cLL, long double cL, KStencil* out) {
  sc_status r;
  sc_stencil* LL = nullptr;
  if ((r = compose(lap, lap, &LL)) != SC_OK) return r;
  std::map<std::array<int32_t, 3>, long double> wa;
  if (cI != 0.0L) wa[{0, 0, 0}] += cI;
  for (size_t t = 0; t < LL->num.size(); ++t) wa[LL->off[t]] += cLL * (long double)LL->num[t] / LL->den;
  if (cL != 0.0L)
    for (size_t t = 0; t < lap->num.size(); ++t) wa[lap->off[t]] += cL * (long double)lap->num[t] / lap->den;
  delete LL;
  std::vector<std::array<int32_t, 3>> offs;
  std::vector<long double> ws;
  for (auto& kv : wa) {
    offs.push_back(kv.first);
    ws.push_back(kv.second);
  }
  return make_kstencil(lap->dim, offs, ws, out);
}

sc_status ch_operator(const sc_stencil* lap, const sc_ch_params* prm, KStencil* ksA, KStencil* ksL) {
  sc_status r;
  const long double h = prm->h;
  const long double cLL = (long double)prm->dt * prm->eps * prm->eps / (h * h * h * h);
  const long double cL = -(long double)prm->dt * prm->S / (h * h);
  if ((r = lap_operator(lap, 1.0L, cLL, cL, ksA)) != SC_OK) return r;
  return make_kstencil(lap, prm->h, ksL);
}

sc_status check_ch(const sc_stencil* lap, const sc_ch_params* prm, int dim) {
  if (!lap || !prm) {
    set_error("NULL Laplacian or parameters");
    return SC_EINVAL;
  }
  if (lap->dim != dim || lap->hpow != 2) {
    set_error("lap must be a %dD second-derivative stencil (hpow 2)", dim);
    return SC_EINVAL;
  }
  if (!(prm->h > 0) || !(prm->dt > 0) || !(prm->eps >= 0) || !std::isfinite(prm->S)) {
    set_error("invalid Cahn-Hilliard parameters");
    return SC_EINVAL;
  }
  return SC_OK;
}

// Drive a task to completion on its stream.
// The blocking entry points run on the caller's stream. The legacy null
// stream cannot be captured into a graph, so a call made on it runs on a
// per-thread, per-device non-blocking stream that first waits for the work
// already queued on the null stream; the call returns only after that stream
// has drained, so later null-stream work is ordered after it.
sc_status blocking_stream(hipStream_t caller, hipStream_t* out) {
  *out = caller;
  if (caller) return SC_OK;
  struct Cached {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
  };
  thread_local std::map<int, Cached> cache;
  int dev = 0;
  SC_HIP_CHECK(hipGetDevice(&dev));
  Cached& c = cache[dev];
  if (!c.st) {
    SC_HIP_CHECK(hipStreamCreateWithFlags(&c.st, hipStreamNonBlocking));
    SC_HIP_CHECK(hipEventCreateWithFlags(&c.ev, hipEventDisableTiming));
  }
  SC_HIP_CHECK(hipEventRecord(c.ev, nullptr));
  SC_HIP_CHECK(hipStreamWaitEvent(c.st, c.ev, 0));
  *out = c.st;
  return SC_OK;
}

sc_status run_blocking(SolveTask& t) {
  bool done = false;
  while (!done) {
    SC_HIP_CHECK(hipStreamSynchronize(t.stream()));
    sc_status s = t.advance(&done);
    if (s != SC_OK) return s;
  }
  return t.status();
}

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
  TaskSpec sp;
  fill_opts(opts, &sp.o);
  if ((r = check_opts(sp.o)) != SC_OK) return r;
  if ((r = make_kstencil(op, h, &sp.ksA)) != SC_OK) return r;
  const int rad = sp.ksA.R;
  if (gr && gr->halo < rad) {
    set_error("g must carry a ring of width >= radius (%d < %d)", gr->halo, rad);
    return SC_EINVAL;
  }
  if ((r = blocking_stream(st, &st)) != SC_OK) return r;
  sp.kind = TASK_BVP;
  sp.h = h;
  sp.dim = u->dim;
  for (int a = 0; a < 3; ++a) sp.n[a] = u->n[a];
  SolveTask t;
  if ((r = t.init(sp, st)) != SC_OK) return r;
  const GridView gv = gr ? view_of(gr) : GridView{};
  if ((r = t.start(view_of(u), view_of(f), gr ? &gv : nullptr)) != SC_OK) return r;
  const sc_status res = run_blocking(t);
  if (res == SC_OK || res == SC_ENOTCONV || res == SC_EBREAKDOWN) {
    if ((r = t.enqueue_copy_out(static_cast<double*>(interior(u)), u->pitch[0], u->pitch[1])) != SC_OK) return r;
    SC_HIP_CHECK(hipStreamSynchronize(st));
  }
  if (stats) {
    *stats = t.stats();
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return res;
}

sc_status ch_step(const sc_stencil* lap, const sc_ch_params* prm, const sc_solve_opts* opts, sc_grid* u,
                  sc_solve_stats* stats, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  sc_status r;
  if ((r = check_grid(u, "u")) != SC_OK) return r;
  if (u->dtype != SC_F64) {
    set_error("u must be FP64");
    return SC_EINVAL;
  }
  if ((r = check_ch(lap, prm, u->dim)) != SC_OK) return r;
  TaskSpec sp;
  fill_opts(opts, &sp.o);
  if ((r = check_opts(sp.o)) != SC_OK) return r;
  if ((r = ch_operator(lap, prm, &sp.ksA, &sp.ksL)) != SC_OK) return r;
  sp.kind = TASK_CH;
  sp.dim = u->dim;
  for (int a = 0; a < 3; ++a) sp.n[a] = u->n[a];
  sp.dt = prm->dt;
  sp.S = prm->S;
  sp.h = prm->h;
  if ((r = blocking_stream(st, &st)) != SC_OK) return r;
  SolveTask t;
  if ((r = t.init(sp, st)) != SC_OK) return r;
  if ((r = t.start(view_of(u), GridView{}, nullptr)) != SC_OK) return r;
  const sc_status res = run_blocking(t);
  if (res == SC_OK) {
    if ((r = t.enqueue_copy_out(static_cast<double*>(interior(u)), u->pitch[0], u->pitch[1])) != SC_OK) return r;
  }
  SC_HIP_CHECK(hipStreamSynchronize(st));
  if (stats) {
    *stats = t.stats();
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
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
  void* p = pool_alloc(kElemBlocks * 3 * sizeof(double));
  void* t = pool_alloc(256);
  if (!p || !t) {
    if (p) pool_free(p);
    if (t) pool_free(t);
    set_error("device allocation failed");
    return SC_ENOMEM;
  }
  struct Release {
    hipStream_t st;
    void* a;
    void* b;
    ~Release() {
      (void)hipStreamSynchronize(st);
      pool_free(a);
      pool_free(b);
    }
  } rel{st, p, t};
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
