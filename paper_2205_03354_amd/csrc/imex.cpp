// IMEX Runge-Kutta steps of the spinodal-decomposition benchmark (Sec. 4.1,
// eq. (cahn) with constant mobility M) on a periodic grid:
//   c' = N(c) + K(c),  N(c) = M L f'(c) (explicit),  K(c) = -M kappa (L o L) c (implicit).
//
// With m = (c_alpha + c_beta) / 2, d = (c_beta - c_alpha) / 2 and w = c - m,
// f'(c) = 2 rho (c - c_alpha)(c - c_beta)(2c - c_alpha - c_beta) = 4 rho (w^3 - d^2 w),
// so N is one Cahn-Hilliard right-hand-side sweep on w (the cube formed in
// registers, centre weight 0), and K, L o L and the stage operators act on w
// as on c (a periodic L annihilates constants). A call therefore shifts c to
// w once, runs every stage on w, and shifts back.
//
// Stage i of a pair (Ahat explicit, A implicit; stage 0 explicit):
//   (I + dt A_ii M kappa L o L) Y_i = w^n + dt sum_{j<i} (Ahat_ij N(Y_j) + A_ij K(Y_j)),
// a CG solve started from Y_{i-1}. The pairs are stiffly accurate, so the
// last stage is w^{n+1}.
#include <chrono>
#include <cmath>

#include "task.hpp"

namespace sc {

namespace {

constexpr int kMaxStages = 5;

struct ImexPair {
  int s = 0;  // stages 0 .. s-1
  double Ah[kMaxStages][kMaxStages] = {};
  double A[kMaxStages][kMaxStages] = {};
};

// The L-stable pairs of Ascher, Ruuth and Spiteri (Appl. Numer. Math. 25,
// 1997): forward/backward Euler, ARS(2,2,2) and ARS(4,4,3). In each, column 0
// of A is zero, the diagonal of A is constant and the last rows are the
// weights.
bool imex_pair(int order, ImexPair* t) {
  *t = ImexPair{};
  if (order == 1) {
    t->s = 2;
    t->Ah[1][0] = 1.0;
    t->A[1][1] = 1.0;
    return true;
  }
  if (order == 2) {
    const double g = 1.0 - 1.0 / std::sqrt(2.0);
    const double d = 1.0 - 1.0 / (2.0 * g);
    t->s = 3;
    t->Ah[1][0] = g;
    t->Ah[2][0] = d;
    t->Ah[2][1] = 1.0 - d;
    t->A[1][1] = g;
    t->A[2][1] = 1.0 - g;
    t->A[2][2] = g;
    return true;
  }
  if (order == 3) {
    static const double Ah[5][5] = {{0, 0, 0, 0, 0},
                                    {1.0 / 2, 0, 0, 0, 0},
                                    {11.0 / 18, 1.0 / 18, 0, 0, 0},
                                    {5.0 / 6, -5.0 / 6, 1.0 / 2, 0, 0},
                                    {1.0 / 4, 7.0 / 4, 3.0 / 4, -7.0 / 4, 0}};
    static const double A[5][5] = {{0, 0, 0, 0, 0},
                                   {0, 1.0 / 2, 0, 0, 0},
                                   {0, 1.0 / 6, 1.0 / 2, 0, 0},
                                   {0, -1.0 / 2, 1.0 / 2, 1.0 / 2, 0},
                                   {0, 3.0 / 2, -3.0 / 2, 1.0 / 2, 1.0 / 2}};
    t->s = 5;
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) {
        t->Ah[i][j] = Ah[i][j];
        t->A[i][j] = A[i][j];
      }
    return true;
  }
  return false;
}

sc_status check_params(const sc_stencil* lap, const sc_spinodal_params* p, int dim) {
  if (!lap || !p) {
    set_error("NULL Laplacian or parameters");
    return SC_EINVAL;
  }
  if (lap->dim != dim || lap->hpow != 2) {
    set_error("lap must be a %dD second-derivative stencil (hpow 2)", dim);
    return SC_EINVAL;
  }
  const bool ok = p->h > 0 && std::isfinite(p->h) && p->dt > 0 && std::isfinite(p->dt) && p->mobility > 0 &&
                  std::isfinite(p->mobility) && p->kappa >= 0 && std::isfinite(p->kappa) &&
                  std::isfinite(p->rho) && std::isfinite(p->c_alpha) && std::isfinite(p->c_beta);
  if (!ok) {
    set_error("invalid spinodal parameters (need h, dt, M > 0, kappa >= 0, finite rho and minima)");
    return SC_EINVAL;
  }
  if (p->order < 1 || p->order > 3) {
    set_error("IMEX order must be 1, 2 or 3 (got %d)", p->order);
    return SC_EINVAL;
  }
  return SC_OK;
}

// Device vectors of one layout (periodic, no ring), released on scope exit
// after the stream has drained.
struct Work {
  hipStream_t st = nullptr;
  std::vector<void*> allocs;
  ~Work() {
    if (st && !allocs.empty()) (void)hipStreamSynchronize(st);
    for (void* a : allocs) pool_free(a);
  }
  void* get(size_t bytes) {
    void* p = pool_alloc(bytes);
    if (p) allocs.push_back(p);
    return p;
  }
};

}  // namespace

sc_status spinodal_steps(const sc_stencil* lap, const sc_spinodal_params* p, int32_t nsteps,
                         const sc_solve_opts* opts, sc_grid* c, sc_spinodal_stats* stats, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  sc_status r;
  if ((r = check_grid(c, "c")) != SC_OK) return r;
  if (c->dtype != SC_F64) {
    set_error("c must be FP64");
    return SC_EINVAL;
  }
  if ((r = check_params(lap, p, c->dim)) != SC_OK) return r;
  if (nsteps < 0) {
    set_error("nsteps must be >= 0");
    return SC_EINVAL;
  }
  TaskSpec sp;
  fill_opts(opts, &sp.o);
  if ((r = check_opts(sp.o)) != SC_OK) return r;
  if (sp.o.precond != SC_PC_NONE) {
    set_error("the stage solves take no preconditioner");
    return SC_EINVAL;
  }
  ImexPair T;
  imex_pair(p->order, &T);
  const double m = 0.5 * (p->c_alpha + p->c_beta);
  const double d = 0.5 * (p->c_beta - p->c_alpha);
  const long double h = p->h;
  const long double h4 = h * h * h * h;
  const long double Mk = (long double)p->mobility * p->kappa;
  KStencil ksL, ksK;
  if ((r = make_kstencil(lap, p->h, &ksL)) != SC_OK) return r;
  if ((r = lap_operator(lap, 0.0L, -Mk / h4, 0.0L, &ksK)) != SC_OK) return r;
  if ((r = lap_operator(lap, 1.0L, (long double)p->dt * T.A[1][1] * Mk / h4, 0.0L, &sp.ksA)) != SC_OK) return r;
  sp.kind = TASK_LIN;
  sp.dim = c->dim;
  for (int a = 0; a < 3; ++a) sp.n[a] = c->n[a];
  sp.h = p->h;
  if ((r = blocking_stream(st, &st)) != SC_OK) return r;

  // explicit and implicit stage terms, intermediate stages, the rhs
  const Layout lay = make_layout(sp.dim, sp.n, 0, SC_F64);
  const size_t vb = vec_bytes(sp.dim, sp.n, 0, SC_F64);
  Work work;
  work.st = st;
  double *w = nullptr, *rhs = nullptr;
  double *Y[kMaxStages] = {}, *N[kMaxStages] = {}, *K[kMaxStages] = {};
  auto vec = [&](double** out) -> sc_status {
    void* v = work.get(vb);
    if (!v) {
      set_error("device workspace allocation of %zu bytes failed", vb);
      return SC_ENOMEM;
    }
    *out = static_cast<double*>(v);
    SC_HIP_CHECK(hipMemsetAsync(v, 0, vb, st));
    return SC_OK;
  };
  if ((r = vec(&w)) != SC_OK || (r = vec(&rhs)) != SC_OK) return r;
  for (int i = 0; i + 1 < T.s; ++i) {
    if ((r = vec(&N[i])) != SC_OK) return r;
    if (i >= 1 && ((r = vec(&Y[i])) != SC_OK || (r = vec(&K[i])) != SC_OK)) return r;
  }
  Y[0] = w;
  Y[T.s - 1] = w;  // stiffly accurate: the last stage is the new state
  SweepLaunch LN = sweep_on(K_CHRHS, ksL, true, SC_F64, sp.n);
  const int slots = std::max(sweep_blocks(LN), kElemBlocks);
  void* blk = work.get(sizeof(DevScalars) + 256 + (size_t)slots * sizeof(double));
  if (!blk) {
    set_error("device allocation failed");
    return SC_ENOMEM;
  }
  SC_HIP_CHECK(hipMemsetAsync(blk, 0, sizeof(DevScalars), st));
  DevScalars* dsc = static_cast<DevScalars*>(blk);
  double* partials = reinterpret_cast<double*>(static_cast<char*>(blk) + sizeof(DevScalars) + 256);

  // N(y) = 4 rho M L(y^3 - d^2 y); K(y) = -M kappa (L o L) y
  auto explicit_part = [&](const double* y, double* out) -> sc_status {
    SweepLaunch L = LN;
    L.in = y;
    L.pin = lay.pitch;
    L.zin = lay.zpitch;
    L.out = out;
    L.pout = lay.pitch;
    L.zout = lay.zpitch;
    L.scal = dsc;
    L.partials = partials;
    L.c0 = 4.0 * p->rho * p->mobility;
    L.c1 = d * d;
    L.c2 = 0.0;
    L.c3 = 0.0;
    return launch(L, st);
  };
  auto implicit_part = [&](const double* y, double* out) -> sc_status {
    SweepLaunch L = sweep_on(K_APPLY, ksK, true, SC_F64, sp.n);
    L.in = y;
    L.pin = lay.pitch;
    L.zin = lay.zpitch;
    L.out = out;
    L.pout = lay.pitch;
    L.zout = lay.zpitch;
    return launch(L, st);
  };

  const GridView cv = view_of(c);
  SC_HIP_CHECK(launch_copy_shift(cv.p, cv.pitch, cv.zpitch, w, lay.pitch, lay.zpitch, sp.n, -m, st));
  sc_spinodal_stats acc{};
  sc_status res = SC_OK;
  SolveTask t;  // one workspace and one set of graphs for every stage solve
  if ((r = t.init(sp, st)) != SC_OK) return r;
  for (int step = 0; step < nsteps && res == SC_OK; ++step) {
    if ((r = explicit_part(w, N[0])) != SC_OK) return r;
    for (int i = 1; i < T.s; ++i) {
      CombineTerms ct;
      for (int j = 0; j < i; ++j) {
        if (T.Ah[i][j] != 0.0) {
          ct.v[ct.n] = N[j];
          ct.coef[ct.n++] = p->dt * T.Ah[i][j];
        }
        if (j >= 1 && T.A[i][j] != 0.0) {
          ct.v[ct.n] = K[j];
          ct.coef[ct.n++] = p->dt * T.A[i][j];
        }
      }
      SC_HIP_CHECK(launch_combine(ct, w, rhs, lay, sp.n, st));
      const double* x0 = i == 1 ? w : Y[i - 1];
      if ((r = t.restart(GridView{x0, lay.pitch, lay.zpitch}, GridView{rhs, lay.pitch, lay.zpitch})) != SC_OK)
        return r;
      res = run_blocking(t);
      acc.solves += 1;
      acc.iterations += t.stats().iterations;
      acc.max_rel_residual = std::max(acc.max_rel_residual, t.stats().rel_residual);
      if (res != SC_OK) break;  // w still holds the last completed step
      if ((r = t.enqueue_copy_out(Y[i], lay.pitch, lay.zpitch)) != SC_OK) return r;
      if (i + 1 < T.s) {
        if ((r = explicit_part(Y[i], N[i])) != SC_OK) return r;
        if ((r = implicit_part(Y[i], K[i])) != SC_OK) return r;
      }
    }
    if (res == SC_OK) acc.steps += 1;
  }
  SC_HIP_CHECK(launch_copy_shift(w, lay.pitch, lay.zpitch, static_cast<double*>(interior(c)), c->pitch[0],
                                 c->pitch[1], sp.n, m, st));
  SC_HIP_CHECK(hipStreamSynchronize(st));
  if (stats) {
    acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *stats = acc;
  }
  return res;
}

sc_status spinodal_energy(const sc_grid* c, const sc_spinodal_params* p, double* mass, double* energy,
                          hipStream_t st) {
  sc_status r;
  if ((r = check_grid(c, "c")) != SC_OK) return r;
  if (c->dtype != SC_F64) {
    set_error("c must be FP64");
    return SC_EINVAL;
  }
  if (!p || !(p->h > 0) || !std::isfinite(p->rho) || !std::isfinite(p->kappa) || !std::isfinite(p->c_alpha) ||
      !std::isfinite(p->c_beta)) {
    set_error("invalid spinodal parameters");
    return SC_EINVAL;
  }
  if ((r = blocking_stream(st, &st)) != SC_OK) return r;
  Work work;
  work.st = st;
  void* part = work.get(kElemBlocks * 3 * sizeof(double));
  void* t = work.get(256);
  if (!part || !t) {
    set_error("device allocation failed");
    return SC_ENOMEM;
  }
  SC_HIP_CHECK(hipMemsetAsync(t, 0, 256, st));
  double* out3 = reinterpret_cast<double*>(static_cast<char*>(t) + 64);
  const double well[2] = {p->c_alpha, p->c_beta};
  SC_HIP_CHECK(launch_diagnostics(static_cast<const double*>(interior(c)), c->pitch[0], c->pitch[1], c->dim, c->n,
                                  static_cast<double*>(part), static_cast<unsigned int*>(t), out3, st, well));
  double host[3];
  SC_HIP_CHECK(hipMemcpyAsync(host, out3, sizeof(host), hipMemcpyDeviceToHost, st));
  SC_HIP_CHECK(hipStreamSynchronize(st));
  const double hd = c->dim == 3 ? p->h * p->h * p->h : p->h * p->h;
  if (mass) *mass = hd * host[0];
  if (energy) *energy = hd * (p->rho * host[1] + 0.5 * p->kappa * host[2] / (p->h * p->h));
  return SC_OK;
}

}  // namespace sc
