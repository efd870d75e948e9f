// Host-side internals of the stencil-composition library: the stencil
// object, kernel-pattern selection, launch descriptors and error handling.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/scomp.h"
#include "common.hpp"

// Exact stencil: weight of tap t is num[t] / (den * h^hpow). Taps are in
// canonical order (z, y, x ascending), without duplicates or zero weights,
// and gcd(num..., den) == 1 with den > 0.
struct sc_stencil {
  int dim = 0;
  int hpow = 0;
  int64_t den = 1;
  std::vector<std::array<int32_t, 3>> off;
  std::vector<int64_t> num;
  // kernel-ready weights for the last grid spacing used (host cache, guarded
  // by `mu`; a stencil handle may be shared between threads)
  mutable std::mutex mu;
  mutable double cached_h = -1.0;
  mutable std::shared_ptr<void> cached_ks;
};

namespace sc {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();
const char* last_error_message();

#define SC_HIP_CHECK(expr)                                                        \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess) {                                                       \
      ::sc::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                      __LINE__);                                                  \
      return SC_EDEVICE;                                                          \
    }                                                                             \
  } while (0)

// ------------------------------------------------------- kernel stencils
constexpr int kMaxTaps = 128;

// The stencil arranged for one kernel instance: pattern, radius and the
// weights (already divided by den * h^p) in the pattern's tap order.
struct KStencil {
  int dim = 0;
  int pat = 0;
  int R = 0;
  int ntaps = 0;
  bool sym = false;  // w(dx,dy,dz) unchanged by negating any one component
  double w[kMaxTaps] = {};
};

// The same weights re-indexed for the BOX pattern of the same radius
// (sym cleared): the fallback for a (kind, pattern) without its own kernel.
KStencil to_box(const KStencil& ks);

// Choose the cheapest instantiated (pattern, radius) containing every tap of
// the (already scaled) stencil given by offsets and weights.
sc_status make_kstencil(int dim, const std::vector<std::array<int32_t, 3>>& off,
                        const std::vector<long double>& w, KStencil* out);
// Same, from an exact stencil and a grid spacing.
sc_status make_kstencil(const sc_stencil* s, double h, KStencil* out);

// ------------------------------------------------------------- launches
struct SweepLaunch {
  int kind = 0;        // SweepKind
  int dtype = SC_F64;  // SC_F64 / SC_F32
  bool periodic = true;
  const KStencil* ks = nullptr;
  const void* in = nullptr;
  const void* in2 = nullptr;
  const void* aux = nullptr;
  void* out = nullptr;
  void* out2 = nullptr;
  int64_t pin = 0, pin2 = 0, paux = 0, pout = 0, pout2 = 0;
  int64_t zin = 0, zin2 = 0, zaux = 0, zout = 0, zout2 = 0;
  int64_t n[3] = {1, 1, 1};
  DevScalars* scal = nullptr;
  double* partials = nullptr;
  double c0 = 0.0, c1 = 0.0, c2 = 0.0;
  double c3 = 1.0;  // K_CHRHS: weight of the centre value
  int flag = 0;
  const double* fold = nullptr;  // K_CGDIR: finish the CG update here from these partials
  int fold_n = 0;
  bool vec_store = false;
  bool in_aligned = false;  // in / in2 / aux rows start on 16-byte boundaries
  // Ring mode: columns [in_xlo, in_xhi) of every in / in2 row and [0, aux_xhi)
  // of every aux row may be read (values outside the ring feed no output).
  // Unset (x_range false): the ring itself, [-R, n0 + R) and [0, n0).
  bool x_range = false;
  int64_t in_xlo = 0, in_xhi = 0, aux_xhi = 0;
};

// Number of blocks (= partial-sum slots) the sweep will launch.
int sweep_blocks(const SweepLaunch& L);
// Launch; returns hipErrorInvalidValue (with sc_last_error set) for a
// (kind, dtype, boundary, pattern, radius) combination with no kernel.
hipError_t launch_sweep(const SweepLaunch& L, hipStream_t st);

// Instantiation parts (dispatch.hip compiled once per part).
hipError_t part_apply2d_f64(const SweepLaunch& L, hipStream_t st);
hipError_t part_apply2d_f32(const SweepLaunch& L, hipStream_t st);
hipError_t part_solve2d_f64_periodic(const SweepLaunch& L, hipStream_t st);
hipError_t part_solve2d_f64_ring(const SweepLaunch& L, hipStream_t st);
hipError_t part_solve2d_f32(const SweepLaunch& L, hipStream_t st);
hipError_t part_apply3d(const SweepLaunch& L, hipStream_t st);
hipError_t part_solve3d_f64(const SweepLaunch& L, hipStream_t st);
hipError_t part_solve3d_f32(const SweepLaunch& L, hipStream_t st);
hipError_t part_apply3s(const SweepLaunch& L, hipStream_t st);
hipError_t part_solve3s_f64(const SweepLaunch& L, hipStream_t st);
hipError_t part_solve3s_f32(const SweepLaunch& L, hipStream_t st);
hipError_t part_varcoef2d(const SweepLaunch& L, hipStream_t st);
hipError_t part_varcoef3d(const SweepLaunch& L, hipStream_t st);

// Vector layout of solver workspace: pointers address the interior
// (0,0,0) element, rows of `pitch` elements, planes of `zpitch`.
struct Layout {
  int64_t pitch = 0;
  int64_t zpitch = 0;
  int halo = 0;
  int64_t xhi = 0;  // columns [-halo_x, xhi) of every row lie inside the allocation
  int halo_x = 0;
};

constexpr int kElemBlocks = 1024;  // blocks of the element-wise kernels
static_assert(kElemBlocks <= kFoldSlots, "a folding sweep loads the update's partials at once");

// The one-block second half of a grid reduction (see FinKind): sums the
// partials of the kernel launched just before on `st` and finalises.
hipError_t launch_finish(int fk, const FinArgs& f, hipStream_t st);

// x += alpha p; r -= alpha q; <r, r> partials, with alpha = (pc ? rz : rr)
// / <p, q> formed by every block from the s->slots partials of the direction
// sweep just before (pq_partials must differ from partials). fin: the
// finish kernel turns the partials into beta and the stop test; otherwise
// the next direction sweep folds that in (update_slots(n) partials).
hipError_t launch_cg_update(int dtype, void* x, void* r, const void* p, const void* q,
                            const Layout& lay, const int64_t* n, DevScalars* s, const double* pq_partials,
                            int pc, double* partials, bool fin, hipStream_t st);
int update_slots(const int64_t* n);
// r32 = r64 / s; d32 = 0; rr = <r32, r32>, rr_stop = inner_tol^2 rr. A
// restart (keep_direction 0) sets s = sqrt(s64->rr_true) and beta = 0; a
// reliable update (keep_direction 1) keeps s and rescales beta so that the
// next direction continues the FP32 recurrence from the replaced residual.
hipError_t launch_ir_prepare(const double* r64, const Layout& l64, float* r32, float* d32,
                             const Layout& l32, const int64_t* n, DevScalars* s64,
                             DevScalars* s32, double inner_tol2, int keep_direction,
                             double* partials, hipStream_t st);
// Preconditioner pieces: t /= (lx_i + ly_j + lz_k)^2 (lz may be null), and
// rz = <r, z>, beta = rz / rz_old (0 when start), both skipped once done.
hipError_t launch_pc_init(int dtype, void* S, double* lam, int64_t m, double h, hipStream_t st);
// The split sine transform of length m (even rows from the folded sums,
// odd rows from the folded differences; see elementwise.hip): F holds the
// two half matrices, lam the 1D eigenvalues in the transformed data's order.
hipError_t launch_pc_init_split(int dtype, void* F, double* lam, int64_t m, double h, hipStream_t st);
// The fold / unfold step of the split transform along `axis` (in may equal out).
hipError_t launch_butterfly(int dtype, const void* in, void* out, const Layout& lay, const int64_t* n, int axis,
                            hipStream_t st);
hipError_t launch_pc_scale(int dtype, void* t, const Layout& lay, const int64_t* n, const double* lx,
                           const double* ly, const double* lz, const DevScalars* s, hipStream_t st);
hipError_t launch_pc_dot(int dtype, const void* r, const void* z, const Layout& lay, const int64_t* n,
                         DevScalars* s, int start, double* partials, hipStream_t st);
// Nonzero taps of a stencil as (offset, weight) pairs (kernel argument).
struct TapTable {
  int n = 0;
  int off[kMaxTaps][3];
  double w[kMaxTaps];
};
TapTable tap_table(const KStencil& ks);
// Ring-mode residual r = b - A x with the stencil sum carried in double-double
// (error-free products and sums), so that the residual is accurate relative
// to |b - A x| rather than to |A| |x|; then <r, r> -> rr_true (and a CG
// restart when flag; flag 2 also sets rr_stop = c <b, b>). x has a ring of
// width >= the taps' radius.
hipError_t launch_resid_dd(const double* x, const Layout& lx, const double* b, double* r, const Layout& lr,
                           const int64_t* n, const TapTable& taps, DevScalars* s, int flag, double c,
                           double* partials, hipStream_t st);
// x64 += s32->scale * d32
hipError_t launch_ir_update(double* x64, const Layout& l64, const float* d32, const Layout& l32,
                            const int64_t* n, const DevScalars* s32, hipStream_t st);
// Copy the interior of one FP64 grid view to another.
hipError_t launch_copy(const double* src, int64_t sp, int64_t sz, double* dst, int64_t dp,
                       int64_t dz, const int64_t* n, hipStream_t st);
// mass = sum u, grad = sum_axes (u_{i+e} - u_i)^2, bulk = sum (u^2-1)^2/4,
// periodic; results into out[3] (device) via a deterministic reduction.
hipError_t launch_diagnostics(const double* u, int64_t pitch, int64_t zpitch, int dim,
                              const int64_t* n, double* partials, unsigned int* ticket, double* out3,
                              hipStream_t st, const double* well = nullptr);
// dst = src + add over the interior (FP64, layouts may differ).
hipError_t launch_copy_shift(const double* src, int64_t sp, int64_t sz, double* dst, int64_t dp, int64_t dz,
                             const int64_t* n, double add, hipStream_t st);
// dst = src; s->bb = <src, src>, s->rr_stop = tol2 s->bb.
hipError_t launch_copy_norm(const double* src, int64_t sp, int64_t sz, double* dst, int64_t dp, int64_t dz,
                            const int64_t* n, DevScalars* s, double tol2, double* partials, hipStream_t st);
// out = base + sum_k coef[k] v[k] (FP64, one layout; out may alias base).
constexpr int kMaxCombine = 10;
struct CombineTerms {
  int n = 0;
  const double* v[kMaxCombine] = {};
  double coef[kMaxCombine] = {};
};
hipError_t launch_combine(const CombineTerms& t, const double* base, double* out, const Layout& lay,
                          const int64_t* n, hipStream_t st);

// Fused 2D variable-coefficient composition (varcoef.hip): a term list
// whose taps are given as offsets into the kernel's LDS tiles (rows of x
// kVcPitchX apart, rows of w kVcPitchW apart; w is kVcTileX wide), inner
// lists padded with zero weights to a multiple of four taps and outer lists
// to an even count.
constexpr int kVcTileX = 64;
constexpr int kVcMaxTerms = 4, kVcMaxTapsA = 40, kVcMaxTapsB = 16;
constexpr int kVcMaxRing = 6, kVcMaxOuterR = 2;  // RA + RB, RB
constexpr int kVcPitchX = kVcTileX + 2 * kVcMaxRing, kVcPitchW = kVcTileX;
template <typename T>
struct VcTerms {
  int n = 0, RA = 0, RB = 0;
  int na[kVcMaxTerms] = {}, nb[kVcMaxTerms] = {};
  int aoff[kVcMaxTerms][kVcMaxTapsA] = {};
  int boff[kVcMaxTerms][kVcMaxTapsB] = {};
  T aw[kVcMaxTerms][kVcMaxTapsA] = {};
  T bw[kVcMaxTerms][kVcMaxTapsB] = {};
};
// y (interior, row pitch py) = sum_t B_t(M * A_t(x)); x and M point at
// their interiors. periodic: indices wrap; else x carries a ring of RA + RB
// and M one of RB. terms points at a VcTerms<double> or VcTerms<float>.
hipError_t launch_varcoef_fused(int dtype, const void* x, int64_t px, const void* m, int64_t pm, void* y, int64_t py,
                                int64_t n0, int64_t n1, bool periodic, const void* terms, hipStream_t st);

// ------------------------------------------------------ entry-point bodies
sc_status stencil_create(int32_t dim, int32_t npts, const int32_t* offsets, const int64_t* num,
                         int64_t den, int32_t hpow, sc_stencil** out);
sc_status compose(const sc_stencil* a, const sc_stencil* b, sc_stencil** out);
sc_status lincomb(int32_t n, const sc_stencil* const* terms, const int64_t* cnum, const int64_t* cden,
                  const int32_t* chpow, sc_stencil** out);
sc_status apply_composed(const sc_stencil* s, double h, const sc_grid* in, sc_grid* out, sc_bc bc,
                         hipStream_t st);
sc_status solve_biharmonic(const sc_stencil* op, double h, const sc_grid* f, const sc_grid* g,
                           const sc_solve_opts* opts, sc_grid* u, sc_solve_stats* stats, hipStream_t st);
sc_status ch_step(const sc_stencil* lap, const sc_ch_params* prm, const sc_solve_opts* opts, sc_grid* u,
                  sc_solve_stats* stats, hipStream_t st);
sc_status grid_diagnostics(const sc_grid* u, double h, double eps, double* mass, double* energy,
                           hipStream_t st);
sc_status server_create(const sc_server_opts* opts, sc_server** out);
sc_status server_submit(sc_server* s, const sc_request* r, uint64_t* id);
sc_status server_poll(sc_server* s, sc_result* out, int32_t max, int32_t* n, int32_t wait_ms);
sc_status server_cancel(sc_server* s, uint64_t id);
sc_status server_load(sc_server* s, int32_t* queued, int32_t* active, int32_t* fin, uint64_t* bytes);
void server_destroy(sc_server* s);
// shared validation / set-up helpers (solver.cpp)
sc_status check_grid(const sc_grid* g, const char* what);
void* interior(const sc_grid* g);
sc_status apply_varcoef(int nterms, const sc_stencil* const* inner, const sc_stencil* const* outer, double h,
                        const sc_grid* M, const sc_grid* in, sc_grid* out, sc_bc bc, hipStream_t st);
void fill_opts(const sc_solve_opts* in, sc_solve_opts* o);
sc_status check_precision(int precision);
sc_status check_opts(const sc_solve_opts& o);
sc_status check_ch(const sc_stencil* lap, const sc_ch_params* prm, int dim);
sc_status ch_operator(const sc_stencil* lap, const sc_ch_params* prm, KStencil* ksA, KStencil* ksL);

// --------------------------------------------------------- workspace pool
// Grow-only per-device cache of device allocations (never returned to the
// driver before process exit).
void* pool_alloc(size_t bytes);
void pool_free(void* p);
size_t esize(int dtype);

// On-chip CG for small 2D BVPs, one workgroup per problem (small.hip).
constexpr int kSmallTaps = 64;
constexpr int kSmallMaxPoints = 4096;  // unknowns per problem (512 segments of 8)
constexpr int kSmallMaxTile = 7936;    // unknowns plus the ring of the pattern radius
struct SmallDesc {
  const double* f;  // interiors
  const double* g;  // NULL: zero ring
  double* u;        // initial guess in, solution out
  int64_t pf, pg, pu;
  int n0, n1;
  double w[kSmallTaps];
};
struct SmallTaps {
  int n;
  int R;
  int dx[kSmallTaps];
  int dy[kSmallTaps];
};
struct SmallResult {
  long long iter;
  double rr_true;
  double bb;
  int status;
  int outer;
};
// Kernel class (R - 1) of an n0 x n1 problem of pattern radius R, or -1
// when it does not fit one workgroup.
int small_class(int64_t n0, int64_t n1, int R);
// Solve `count` problems of one class (descs and results in device memory).
hipError_t launch_small_cg(const SmallDesc* descs, const SmallTaps& taps, int count, int cls, double tol2,
                           long long max_iter, SmallResult* results, hipStream_t st);

// Batched small 2D BVPs, one workgroup per problem (small.hip).
sc_status solve_biharmonic_batch(const sc_stencil* op, const double* h, int32_t count, const sc_grid* f,
                                 const sc_grid* g, const sc_solve_opts* opts, sc_grid* u, sc_solve_stats* stats,
                                 hipStream_t st);

// IMEX steps of the spinodal-decomposition benchmark (imex.cpp).
sc_status spinodal_steps(const sc_stencil* lap, const sc_spinodal_params* p, int32_t nsteps,
                         const sc_solve_opts* opts, sc_grid* c, sc_spinodal_stats* stats, hipStream_t st);
sc_status spinodal_energy(const sc_grid* c, const sc_spinodal_params* p, double* mass, double* energy,
                          hipStream_t st);

// Assembled CSR form of a stencil (csr.hip).
sc_status csr_assemble(const sc_stencil* s, double h, int32_t dim, const int64_t* n, int32_t bc, int32_t dtype,
                       int32_t alg, hipStream_t st, sc_csr** out);
sc_status csr_info(const sc_csr* m, int64_t* rows, int64_t* nnz, uint64_t* bytes);
sc_status csr_spmv(sc_csr* m, const sc_grid* x, sc_grid* y, hipStream_t st);
sc_status csr_export(const sc_csr* m, int64_t* row_ptr, int32_t* col, void* val);
void csr_free(sc_csr* m);

}  // namespace sc
