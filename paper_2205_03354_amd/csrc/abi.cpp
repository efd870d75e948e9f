// extern "C" entry points declared in include/scomp.h. They translate
// arguments, catch every C++ exception and record the error message; the
// work itself lives in stencil.cpp, solver.cpp and the kernels.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.hpp"

namespace sc {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

const char* last_error_message() { return g_err; }

}  // namespace sc

#define SC_GUARD(body)                         \
  try {                                        \
    body                                       \
  } catch (const std::bad_alloc&) {            \
    ::sc::set_error("host allocation failed"); \
    return SC_ENOMEM;                          \
  } catch (...) {                              \
    ::sc::set_error("internal error");         \
    return SC_EINVAL;                          \
  }

extern "C" {

sc_status sc_stencil_create(int32_t dim, int32_t npts, const int32_t* offsets, const int64_t* num,
                            int64_t den, int32_t hpow, sc_stencil** out) {
  SC_GUARD(return sc::stencil_create(dim, npts, offsets, num, den, hpow, out);)
}

sc_status sc_compose_stencil(const sc_stencil* a, const sc_stencil* b, sc_stencil** out) {
  SC_GUARD(return sc::compose(a, b, out);)
}

sc_status sc_stencil_lincomb(int32_t n, const sc_stencil* const* terms, const int64_t* cnum,
                             const int64_t* cden, const int32_t* chpow, sc_stencil** out) {
  SC_GUARD(return sc::lincomb(n, terms, cnum, cden, chpow, out);)
}

sc_status sc_stencil_get(const sc_stencil* s, int32_t* dim, int32_t* npts, int32_t capacity,
                         int32_t* offsets, int64_t* num, int64_t* den, int32_t* hpow) {
  if (!s) {
    sc::set_error("NULL stencil");
    return SC_EINVAL;
  }
  const int32_t np = (int32_t)s->off.size();
  if (dim) *dim = s->dim;
  if (npts) *npts = np;
  if (den) *den = s->den;
  if (hpow) *hpow = s->hpow;
  if (capacity >= np) {
    for (int32_t t = 0; t < np; ++t) {
      if (offsets) {
        offsets[3 * t] = s->off[t][0];
        offsets[3 * t + 1] = s->off[t][1];
        offsets[3 * t + 2] = s->off[t][2];
      }
      if (num) num[t] = s->num[t];
    }
  } else if (offsets || num) {
    sc::set_error("capacity %d < %d taps", capacity, np);
    return SC_EINVAL;
  }
  return SC_OK;
}

int32_t sc_stencil_radius(const sc_stencil* s) {
  if (!s) return -1;
  int32_t r = 0;
  for (const auto& o : s->off)
    for (int d = 0; d < 3; ++d) r = std::max<int32_t>(r, o[d] < 0 ? -o[d] : o[d]);
  return r;
}

void sc_stencil_free(sc_stencil* s) { delete s; }

sc_status sc_apply_composed(const sc_stencil* s, double h, const sc_grid* in, sc_grid* out, sc_bc bc,
                            sc_stream_t stream) {
  SC_GUARD(return sc::apply_composed(s, h, in, out, bc, reinterpret_cast<hipStream_t>(stream));)
}

sc_status sc_apply_varcoef(int32_t nterms, const sc_stencil* const* inner, const sc_stencil* const* outer,
                           double h, const sc_grid* mob, const sc_grid* in, sc_grid* out, sc_bc bc,
                           sc_stream_t stream) {
  SC_GUARD(return sc::apply_varcoef(nterms, inner, outer, h, mob, in, out, bc, reinterpret_cast<hipStream_t>(stream));)
}

sc_status sc_spinodal_steps(const sc_stencil* lap, const sc_spinodal_params* p, int32_t nsteps,
                            const sc_solve_opts* opts, sc_grid* c, sc_spinodal_stats* stats,
                            sc_stream_t stream) {
  SC_GUARD(return sc::spinodal_steps(lap, p, nsteps, opts, c, stats, reinterpret_cast<hipStream_t>(stream));)
}

sc_status sc_spinodal_energy(const sc_grid* c, const sc_spinodal_params* p, double* mass, double* energy,
                             sc_stream_t stream) {
  SC_GUARD(return sc::spinodal_energy(c, p, mass, energy, reinterpret_cast<hipStream_t>(stream));)
}

sc_status sc_csr_assemble(const sc_stencil* s, double h, int32_t dim, const int64_t* n, int32_t bc,
                          int32_t dtype, int32_t alg, sc_stream_t stream, sc_csr** out) {
  SC_GUARD(return sc::csr_assemble(s, h, dim, n, bc, dtype, alg, reinterpret_cast<hipStream_t>(stream), out);)
}

sc_status sc_csr_info(const sc_csr* m, int64_t* rows, int64_t* nnz, uint64_t* bytes) {
  SC_GUARD(return sc::csr_info(m, rows, nnz, bytes);)
}

sc_status sc_csr_spmv(sc_csr* m, const sc_grid* x, sc_grid* y, sc_stream_t stream) {
  SC_GUARD(return sc::csr_spmv(m, x, y, reinterpret_cast<hipStream_t>(stream));)
}

sc_status sc_csr_export(const sc_csr* m, int64_t* row_ptr, int32_t* col, void* val) {
  SC_GUARD(return sc::csr_export(m, row_ptr, col, val);)
}

void sc_csr_free(sc_csr* m) {
  try {
    sc::csr_free(m);
  } catch (...) {
  }
}

void sc_solve_opts_default(sc_solve_opts* o) {
  if (!o) return;
  o->tol = 1e-10;
  o->max_iter = 10000000;
  o->precision = SC_PREC_F64;
  o->inner_tol = 0.0;
  o->check_every = 64;
  o->use_graph = 1;
  o->precond = SC_PC_NONE;
  o->onchip = 1;
}

sc_status sc_solve_biharmonic(const sc_stencil* op, double h, const sc_grid* f, const sc_grid* g,
                              const sc_solve_opts* opts, sc_grid* u, sc_solve_stats* stats,
                              sc_stream_t stream) {
  SC_GUARD(return sc::solve_biharmonic(op, h, f, g, opts, u, stats, reinterpret_cast<hipStream_t>(stream));)
}

sc_status sc_solve_biharmonic_batch(const sc_stencil* op, const double* h, int32_t count, const sc_grid* f,
                                    const sc_grid* g, const sc_solve_opts* opts, sc_grid* u,
                                    sc_solve_stats* stats, sc_stream_t stream) {
  SC_GUARD(return sc::solve_biharmonic_batch(op, h, count, f, g, opts, u, stats,
                                             reinterpret_cast<hipStream_t>(stream));)
}

sc_status sc_ch_step(const sc_stencil* lap, const sc_ch_params* prm, const sc_solve_opts* opts, sc_grid* u,
                     sc_solve_stats* stats, sc_stream_t stream) {
  SC_GUARD(return sc::ch_step(lap, prm, opts, u, stats, reinterpret_cast<hipStream_t>(stream));)
}

sc_status sc_grid_diagnostics(const sc_grid* u, double h, double eps, double* mass, double* energy,
                              sc_stream_t stream) {
  SC_GUARD(return sc::grid_diagnostics(u, h, eps, mass, energy, reinterpret_cast<hipStream_t>(stream));)
}

sc_status sc_server_create(const sc_server_opts* opts, sc_server** out) {
  SC_GUARD(return sc::server_create(opts, out);)
}

sc_status sc_server_submit(sc_server* s, const sc_request* r, uint64_t* id) {
  SC_GUARD(return sc::server_submit(s, r, id);)
}

sc_status sc_server_poll(sc_server* s, sc_result* out, int32_t max, int32_t* n, int32_t wait_ms) {
  SC_GUARD(return sc::server_poll(s, out, max, n, wait_ms);)
}

sc_status sc_server_cancel(sc_server* s, uint64_t id) { SC_GUARD(return sc::server_cancel(s, id);) }

sc_status sc_server_load(sc_server* s, int32_t* queued, int32_t* active, int32_t* finished,
                         uint64_t* device_bytes) {
  SC_GUARD(return sc::server_load(s, queued, active, finished, device_bytes);)
}

void sc_server_destroy(sc_server* s) {
  try {
    sc::server_destroy(s);
  } catch (...) {
  }
}

const char* sc_status_str(sc_status s) {
  switch (s) {
    case SC_OK: return "ok";
    case SC_EINVAL: return "invalid argument";
    case SC_EOVERFLOW: return "rational overflow";
    case SC_EDEVICE: return "device error";
    case SC_ENOMEM: return "out of memory";
    case SC_ENOTCONV: return "not converged";
    case SC_EBREAKDOWN: return "CG breakdown";
    case SC_EUNSUPPORTED: return "unsupported";
    case SC_ECANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char* sc_last_error(void) { return sc::last_error_message(); }

const char* sc_version(void) { return "scomp 0.1.0 (gfx950)"; }

}  // extern "C"
