/*
 * scomp.h - C ABI of the MI355X stencil-composition library.
 *
 * The library forms finite-difference stencils by composition and applies
 * them matrix-free on structured 2D/3D grids on a gfx950 GPU, inside
 * conjugate-gradient solves of a biharmonic boundary-value problem and of an
 * implicit Cahn-Hilliard step.
 *
 * Paper: A. Mishra, D. Salac, M. G. Knepley, "On the order of accuracy for
 * finite difference approximations of partial differential equations using
 * stencil composition".
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns an sc_status; SC_OK (0) is success. Nothing is thrown
 *   across the ABI. sc_last_error() gives a human-readable message for the
 *   most recent failure on the calling thread.
 * - Stencils are opaque, library-owned, immutable handles created by
 *   sc_stencil_create / sc_compose_stencil / sc_stencil_lincomb and released
 *   with sc_stencil_free. They live in host memory only.
 * - Grids (sc_grid) describe caller-owned DEVICE memory. The library never
 *   frees or reallocates it. Axis 0 (x) is unit stride.
 * - `stream` is a hipStream_t (NULL = the legacy default stream). Calls that
 *   only launch work (sc_apply_composed) are asynchronous on that stream;
 *   solver calls (sc_solve_biharmonic, sc_ch_step, sc_grid_diagnostics)
 *   return after their work on that stream has completed, because they
 *   test convergence on the host. A solver call made on the NULL stream runs
 *   on a per-thread library stream that first waits for the NULL stream's
 *   queued work (the NULL stream cannot be captured into a hipGraph).
 * - Weights are exact rationals: weight k is num[k] / (den * h^p) where p is
 *   the stencil's power of h (its derivative order). They are converted to
 *   the grid's floating type once, per call.
 */
#ifndef SCOMP_H
#define SCOMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hipStream_t without pulling in the HIP headers. */
typedef struct ihipStream_t* sc_stream_t;

typedef enum sc_status {
  SC_OK = 0,
  SC_EINVAL = 1,       /* bad argument: shapes, sizes, dtypes, aliasing, NULL */
  SC_EOVERFLOW = 2,    /* exact rational arithmetic would overflow int64 */
  SC_EDEVICE = 3,      /* a HIP runtime call failed */
  SC_ENOMEM = 4,       /* device workspace could not be allocated */
  SC_ENOTCONV = 5,     /* iteration limit reached; statistics are filled */
  SC_EBREAKDOWN = 6,   /* CG breakdown: p.Ap <= 0 or not finite */
  SC_EUNSUPPORTED = 7, /* valid request outside what the kernels implement */
  SC_ECANCELLED = 8    /* request cancelled before it finished */
} sc_status;

typedef enum sc_dtype { SC_F64 = 0, SC_F32 = 1 } sc_dtype;

/* How values outside the grid's interior are obtained when a stencil reads
 * them: SC_BC_PERIODIC wraps indices modulo n (true modulo, so stencils wider
 * than the grid alias correctly); SC_BC_HALO reads the ring of width
 * grid.halo stored around the interior (which must be >= the radius). */
typedef enum sc_bc { SC_BC_PERIODIC = 0, SC_BC_HALO = 1 } sc_bc;

/* Arithmetic of the Krylov solves.
 *   SC_PREC_F64     plain FP64 CG.
 *   SC_PREC_F32_IR  FP32 CG (FP32 vectors and applies, FP64 dot-product
 *                   accumulators) inside FP64 iterative refinement: each
 *                   outer step solves A d = r / ||r|| from scratch to a
 *                   relative reduction inner_tol, then x += ||r|| d in FP64
 *                   and r = b - A x is recomputed in FP64.
 *   SC_PREC_F32_RU  FP32 CG with reliable updates (Sleijpen and van der
 *                   Vorst, 1996): whenever the FP32 recursive residual has
 *                   dropped by inner_tol since the last update, the FP32
 *                   solution increment is folded into the FP64 solution, the
 *                   residual is replaced by the FP64 true residual, and the
 *                   FP32 recurrence continues with its search direction
 *                   instead of restarting. Same precisions as SC_PREC_F32_IR.
 * Both mixed modes stop on the FP64 true residual. */
typedef enum sc_precision { SC_PREC_F64 = 0, SC_PREC_F32_IR = 1, SC_PREC_F32_RU = 2 } sc_precision;

/* Preconditioner of the biharmonic BVP's CG.
 *   SC_PC_NONE          plain CG.
 *   SC_PC_FASTPOISSON   M = L_D^2, L_D the 5/7-point Laplacian on the unknowns
 *                       with a zero ring (the composition of Sec. 3.3 on the
 *                       interior). The BVP operator differs from L_D^2 by a
 *                       non-negative diagonal next to the boundary, so CG on
 *                       M^-1 A needs few iterations at any grid size (10..25
 *                       for 33..257 nodes per side). M^-1 is applied with the
 *                       orthonormal sine transform along every axis (dense
 *                       products on the device) and a pointwise division by
 *                       the squared eigenvalues. In the mixed precisions the
 *                       FP32 recurrence is preconditioned in FP32. Blocks of
 *                       preconditioned iterations are not graph-captured. */
typedef enum sc_precond { SC_PC_NONE = 0, SC_PC_FASTPOISSON = 1 } sc_precond;

typedef struct sc_stencil sc_stencil;

/*
 * A structured grid in device memory.
 *   dim      2 or 3.
 *   halo     width of the ring stored around the interior on every active
 *            axis (0 allowed).
 *   n[3]     interior points along x, y, z; n[2] must be 1 when dim == 2.
 *   pitch[2] elements between consecutive rows (y) and planes (z);
 *            pitch[0] >= n[0] + 2 halo, pitch[1] >= pitch[0] (n[1] + 2 halo).
 *            pitch[1] is ignored in 2D.
 *   dtype    sc_dtype of the elements.
 *   data     device pointer to the first stored element (the ring corner).
 * Interior element (i, j, k), with -halo <= i < n[0] + halo etc., sits at
 *   data[(i + halo) + (j + halo) pitch[0] + (k + halo) pitch[1]]   (3D)
 *   data[(i + halo) + (j + halo) pitch[0]]                           (2D).
 */
typedef struct sc_grid {
  int32_t dim;
  int32_t halo;
  int64_t n[3];
  int64_t pitch[2];
  int32_t dtype;
  void* data;
} sc_grid;

/* ---------------------------------------------------------------------------
 * Stencils (host-side exact algebra)
 * ------------------------------------------------------------------------- */

/*
 * Create a stencil from npts taps: offsets[3*t .. 3*t+2] is the integer
 * lattice offset u_t (unused components must be 0 when dim < 3), and the
 * weight of tap t is num[t] / (den * h^hpow) (Sec. 2.1: weights
 * proportional to h^-p). Repeated offsets are summed, zero weights dropped,
 * and the result is reduced to lowest terms with den > 0.
 * Errors: SC_EINVAL (dim not in 1..3, npts < 1, den == 0, NULL pointers,
 * |offset| > 64), SC_EOVERFLOW.
 */
sc_status sc_stencil_create(int32_t dim, int32_t npts, const int32_t* offsets,
                            const int64_t* num, int64_t den, int32_t hpow,
                            sc_stencil** out);

/*
 * Stencil composition C = B(A) (Sec. 2.2, eq. (C=B(A))): the inner stencil A
 * is applied first and the outer stencil B to its result, so
 * C[u_i + v_j] += a_i b_j, the denominators multiply and the powers of h
 * (derivative orders) add. Composition of translation-invariant stencils is
 * commutative (the lemma of Sec. 2.2.1). `a` and `b` are the inner and outer
 * stencils; both must have the same dim.
 * Errors: SC_EINVAL (NULL, dim mismatch), SC_EOVERFLOW.
 */
sc_status sc_compose_stencil(const sc_stencil* a, const sc_stencil* b, sc_stencil** out);

/*
 * Linear combination sum_k (cnum[k]/cden[k]) h^{chpow[k]} S_k (Sec. 2.1: the
 * Taylor sequences form a vector space). All terms must have the same dim
 * and the same S_k.hpow - chpow[k], which becomes the result's hpow. Used to
 * form operators such as I + dt eps^2 L o L - dt S L as one stencil.
 * Errors: SC_EINVAL, SC_EOVERFLOW.
 */
sc_status sc_stencil_lincomb(int32_t n, const sc_stencil* const* terms, const int64_t* cnum,
                             const int64_t* cden, const int32_t* chpow, sc_stencil** out);

/*
 * Read back a stencil. *npts is always written; offsets (3 * npts int32) and
 * num (npts int64) are written only if non-NULL and capacity >= npts. Taps
 * are in canonical order (z, then y, then x offset ascending).
 */
sc_status sc_stencil_get(const sc_stencil* s, int32_t* dim, int32_t* npts, int32_t capacity,
                         int32_t* offsets, int64_t* num, int64_t* den, int32_t* hpow);

/* Chebyshev radius max_t max_d |u_t,d|. */
int32_t sc_stencil_radius(const sc_stencil* s);

void sc_stencil_free(sc_stencil* s);

/* ---------------------------------------------------------------------------
 * Matrix-free application
 * ------------------------------------------------------------------------- */

/*
 * out = S in on the interior of `out`, with weights num/(den h^p) rounded
 * once to the grids' dtype: out(i) = sum_t w_t in(i + u_t) (the definition of
 * applying a stencil, Sec. 2.1; for a composed stencil the taps are those of
 * eq. (C=B(A)), so one pass replaces the two sequential passes of the
 * factors). `in` and `out` must share dim, n and dtype, and must not
 * overlap in memory. In SC_BC_HALO mode in->halo >= max(1, radius(s)). Only the
 * interior of `out` is written; its ring is left untouched.
 * Supported: dim 2 with radius <= 4, dim 3 with radius <= 2 (any pattern
 * inside those boxes). Asynchronous on `stream`.
 * Errors: SC_EINVAL, SC_EUNSUPPORTED, SC_EDEVICE.
 */
sc_status sc_apply_composed(const sc_stencil* s, double h, const sc_grid* in, sc_grid* out,
                            sc_bc bc, sc_stream_t stream);

/*
 * Composition with a varying coefficient between the factors (Sec. 2.2.3,
 * where a spatially varying mobility M sits between an outer first
 * derivative and the composed inner part, as in d_x(M d_x(d_xx f))):
 *     out = sum_{t < nterms} outer[t]( mob * inner[t](in) ),
 * with `*` the pointwise product. For div(M grad(L f)) the terms are
 * inner[a] = D1_a o L and outer[a] = D1_a, a over the axes.
 * `mob` (the coefficient), `in` and `out` share dim, n and dtype; out must
 * not overlap them. SC_BC_PERIODIC: indices wrap. SC_BC_HALO: in->halo >=
 * rA + rB and mob->halo >= rB (rA, rB the largest inner and outer radii),
 * since mob * inner(in) is needed on the grid plus the ring the outer
 * stencils read. 1 <= nterms <= 16. On 2D grids with nterms <= 4, inner
 * stencils of at most 40 and outer ones of at most 16 nonzero taps,
 * rB <= 2 and rA + rB <= 6, one fused kernel computes the sum and the call
 * is asynchronous on `stream`. Otherwise each term is two sweeps through a
 * library workspace, and the call returns after its work on `stream` has
 * completed. The two forms sum in different orders; results agree to
 * rounding. Errors: SC_EINVAL, SC_EUNSUPPORTED, SC_ENOMEM, SC_EDEVICE.
 */
sc_status sc_apply_varcoef(int32_t nterms, const sc_stencil* const* inner, const sc_stencil* const* outer,
                           double h, const sc_grid* mob, const sc_grid* in, sc_grid* out, sc_bc bc,
                           sc_stream_t stream);

/* ---------------------------------------------------------------------------
 * Krylov solves
 * ------------------------------------------------------------------------- */

typedef struct sc_solve_opts {
  double tol;           /* target true relative residual ||b - A x||_2 / ||b||_2 (FP64) */
  int64_t max_iter;     /* cap on CG iterations (FP32 iterations in the mixed modes) */
  int32_t precision;    /* sc_precision */
  double inner_tol;     /* mixed modes: FP32 residual reduction per stretch (per
                           refinement solve, or between reliable updates);
                           <= 0 selects 1e-4 (F32_IR) or 0.1 (F32_RU) */
  int32_t check_every;  /* CG iterations launched between host convergence checks */
  int32_t use_graph;    /* 1: replay each block of check_every iterations from a
                           captured hipGraph; 0: plain launches */
  int32_t precond;      /* sc_precond (biharmonic BVP only; ignored for CH) */
  int32_t onchip;       /* 1: a 2D FP64 unpreconditioned BVP that fits one
                           workgroup (see sc_solve_biharmonic_batch) is solved on
                           chip by one kernel; 0: always the grid solver */
} sc_solve_opts;

typedef struct sc_solve_stats {
  int64_t iterations;   /* CG iterations performed (FP32 inner iterations under IR) */
  int32_t outer;        /* true-residual evaluations / refinement steps */
  double rel_residual;  /* true ||b - A x||_2 / ||b||_2 at return, FP64 on the device */
  double bnorm;         /* ||b||_2 */
  double seconds;       /* wall time of the call */
} sc_solve_stats;

/* Fill opts with defaults: tol 1e-10, max_iter 10^7, SC_PREC_F64,
 * inner_tol 0 (the precision's default), check_every 64, use_graph 1,
 * precond SC_PC_NONE, onchip 1. */
void sc_solve_opts_default(sc_solve_opts* opts);

/*
 * Biharmonic boundary-value problem (Sec. 3.3): A u = f at the unknowns,
 * where A is the composed operator `op` scaled by h^-p (for example the
 * 5/7-point Laplacian composed with itself) and the values on the ring of
 * width radius(op) around the unknowns are prescribed by `g`. Writing
 * u = x + g with x zero on the ring, the solve is textbook CG from the
 * initial guess in `u` on
 *     A0 x = f - A g_ring,
 * A0 being `op` with a zero ring (symmetric positive definite for the
 * composed Laplacian), to ||b - A0 x|| <= tol ||b|| checked on the true
 * residual.
 *   f  FP64 grid, the forcing at the unknowns (ring ignored).
 *   g  FP64 grid with halo >= max(1, radius(op)) holding the ring values (interior
 *      ignored), or NULL for a zero ring.
 *   u  FP64 grid: initial guess at the unknowns on entry, solution on
 *      return; its ring is not touched.
 * All three share dim and n. Supported: dim 2 radius <= 4, dim 3 radius <= 2.
 * Workspace is allocated from a per-device pool owned by the library.
 * Errors: SC_EINVAL, SC_EUNSUPPORTED, SC_ENOMEM, SC_EDEVICE,
 * SC_ENOTCONV (stats filled, u holds the last iterate),
 * SC_EBREAKDOWN (operator not positive definite on the iterates).
 */
sc_status sc_solve_biharmonic(const sc_stencil* op, double h, const sc_grid* f, const sc_grid* g,
                              const sc_solve_opts* opts, sc_grid* u, sc_solve_stats* stats,
                              sc_stream_t stream);

/*
 * A batch of small 2D biharmonic BVPs, each the problem of
 * sc_solve_biharmonic (Sec. 3.3: plain CG in FP64 from the initial guess in
 * u[i] on A0 x = f - A g_ring, stopped on the recurrence residual and
 * confirmed on the true residual), solved concurrently with one workgroup
 * per problem and all of its vectors on chip: the form for latency-bound
 * sizes. One operator `op` (2D) for all problems; per problem i the spacing
 * h[i], the FP64 grids f[i], u[i] and optionally g[i] (g NULL, or
 * g[i].data NULL, for a zero ring; else halo >= radius), of one shape per
 * problem with ceil(n0 / 8) n1 <= 512 and (8 ceil(n0 / 8) + 2R)(n1 + 2R) <= 7936
 * (R the operator's pattern radius; 64 x 64 unknowns for the 13-point
 * L o L).
 * From opts: tol and max_iter; precision must be SC_PREC_F64 and precond
 * SC_PC_NONE; check_every and use_graph do not apply. A problem's result
 * does not depend on the rest of the batch. stats (count entries, may be
 * NULL) receive every problem's statistics, `seconds` being the whole
 * call's. Blocking. Returns SC_OK when every problem converged, else the
 * status of the first problem that did not (SC_ENOTCONV, SC_EBREAKDOWN).
 * Errors: SC_EINVAL, SC_EUNSUPPORTED (sizes, dimension, options),
 * SC_ENOMEM, SC_EDEVICE.
 */
sc_status sc_solve_biharmonic_batch(const sc_stencil* op, const double* h, int32_t count, const sc_grid* f,
                                    const sc_grid* g, const sc_solve_opts* opts, sc_grid* u,
                                    sc_solve_stats* stats, sc_stream_t stream);

/* Cahn-Hilliard step parameters (normalised form u_t = Lap(u^3 - u - eps^2 Lap u)). */
typedef struct sc_ch_params {
  double h;    /* grid spacing (periodic unit domain: h = 1/n) */
  double eps;  /* interface width */
  double dt;   /* time step */
  double S;    /* linear stabilisation constant */
} sc_ch_params;

/*
 * One Cahn-Hilliard step with the linear fourth-order part implicit and the
 * non-linear part explicit (Sec. 4.1, eq. (cahn) and the IMEX treatment
 * stated there), with linear stabilisation S:
 *   (I + dt eps^2 L o L - dt S L) u^{n+1} = u^n + dt L((u^n)^3 - (1+S) u^n),
 * on a periodic grid. `lap` is the Laplacian stencil L (p = 2); the library
 * composes L o L with sc_compose_stencil's algebra and forms the operator as
 * one stencil. The solve starts from x0 = u^n, which keeps the mean of u
 * unchanged in exact arithmetic.
 *   u  FP64 grid (periodic; halo ignored), advanced in place.
 * Errors: as sc_solve_biharmonic.
 */
sc_status sc_ch_step(const sc_stencil* lap, const sc_ch_params* prm, const sc_solve_opts* opts,
                     sc_grid* u, sc_solve_stats* stats, sc_stream_t stream);

/*
 * Diagnostics of a periodic FP64 grid: mass = h^d sum u and the discrete
 * free energy E = h^d sum[(u^2-1)^2/4 + eps^2/2 sum_axes ((u_{i+e}-u_i)/h)^2]
 * (Sec. 4.1, free energy with a double well and gradient term). Either
 * output pointer may be NULL. Reductions are deterministic (fixed order).
 */
sc_status sc_grid_diagnostics(const sc_grid* u, double h, double eps, double* mass,
                              double* energy, sc_stream_t stream);

/* ---------------------------------------------------------------------------
 * Request server: continuous batching of solves
 *
 * A server owns a worker thread, `max_slots` HIP streams and a device-memory
 * budget. Submitted requests are copied and queued; the worker admits them
 * in arrival order whenever a slot is free and their device footprint fits
 * the budget, keeps their whole solver state resident on the device, and
 * advances every admitted request by blocks of check_every CG iterations
 * (each block one hipGraph replay on the request's own stream), so requests
 * that arrive while others run join at the next block boundary and their
 * kernels overlap on the GPU. Finished requests are copied back and retired,
 * which frees their slot and budget for the next ones. Each request computes
 * exactly what the blocking entry point would: results are bit-identical
 * whether a request runs alone or in a mix.
 * ------------------------------------------------------------------------- */

typedef struct sc_server sc_server;

typedef enum sc_request_kind { SC_REQ_BVP = 0, SC_REQ_CH_STEP = 1 } sc_request_kind;

typedef struct sc_server_opts {
  uint64_t hbm_budget;   /* device bytes for request state; 0 = 80% of the free memory */
  int32_t max_slots;     /* requests resident on the device at once (1..256) */
  sc_solve_opts solve;   /* solver options for every request */
  int32_t fake_device;   /* 1: run the scheduler with no device work (testing) */
} sc_server_opts;

/*
 * One request. Host arrays are contiguous FP64 with x fastest and are copied
 * at submit (the caller may reuse them at once); u_out must stay valid until
 * the request's result has been polled.
 *   SC_REQ_BVP:     op = composed operator; f = forcing on the n unknowns;
 *                   g = ring values on the (n + 2 r) box, r = max(1,
 *                   radius(op)), or NULL (zero ring); u0 = initial guess
 *                   or NULL (zero).
 *   SC_REQ_CH_STEP: op = the Laplacian; u0 = u^n (periodic); ch = step
 *                   parameters; f, g unused.
 *   precision       sc_precision for this request, or -1 for the server's.
 */
typedef struct sc_request {
  int32_t kind;
  int32_t dim;
  int64_t n[3];
  double h;
  const sc_stencil* op;
  const double* f;
  const double* g;
  const double* u0;
  double* u_out;
  sc_ch_params ch;
  int32_t precision;
} sc_request;

typedef struct sc_result {
  uint64_t id;
  int32_t status;        /* the solve's sc_status; SC_ECANCELLED; SC_ENOMEM if the
                            request can never fit the budget */
  int64_t iterations;
  int32_t outer;
  double rel_residual;
  double t_submit;       /* seconds since server creation */
  double t_admit;
  double t_done;
  uint64_t device_bytes; /* footprint charged to the budget */
} sc_result;

/* Create a server and start its worker. Errors: SC_EINVAL, SC_EDEVICE. */
sc_status sc_server_create(const sc_server_opts* opts, sc_server** out);
/* Queue a request; *id identifies its result. Errors: SC_EINVAL (shape,
 * stencil, missing arrays), SC_EUNSUPPORTED. */
sc_status sc_server_submit(sc_server* s, const sc_request* r, uint64_t* id);
/* Move up to `max` finished results into out[0..*n); waits up to wait_ms
 * for the first one when none is ready. */
sc_status sc_server_poll(sc_server* s, sc_result* out, int32_t max, int32_t* n, int32_t wait_ms);
/* Cancel a queued or running request (its result reports SC_ECANCELLED);
 * SC_EINVAL if the id is unknown or already finished. */
sc_status sc_server_cancel(sc_server* s, uint64_t id);
/* Requests queued, resident on the device, and finished-but-unpolled. */
sc_status sc_server_load(sc_server* s, int32_t* queued, int32_t* active, int32_t* finished,
                         uint64_t* device_bytes);
/* Stop the worker after the resident requests finish; queued ones are
 * cancelled; unpolled results are discarded. */
void sc_server_destroy(sc_server* s);

/* ---------------------------------------------------------------------------
 * The spinodal-decomposition benchmark (Sec. 4) with IMEX time stepping
 * ------------------------------------------------------------------------- */

/* c_t = div(M grad(f'(c) - kappa Lap c)), f(c) = rho (c - c_alpha)^2 (c - c_beta)^2
 * (Sec. 4.1, eq. (cahn); the benchmark uses M = 5, kappa = 2, rho = 5,
 * c_alpha = 0.3, c_beta = 0.7, h = 1). */
typedef struct sc_spinodal_params {
  double h;         /* grid spacing */
  double dt;        /* time step */
  double mobility;  /* M (constant) */
  double kappa;     /* gradient energy coefficient */
  double rho;       /* height of the double well */
  double c_alpha;   /* the double well's minima */
  double c_beta;
  int32_t order;    /* IMEX order: 1, 2 or 3 */
} sc_spinodal_params;

typedef struct sc_spinodal_stats {
  int64_t steps;
  int64_t solves;           /* implicit stage solves */
  int64_t iterations;       /* CG iterations over all stage solves */
  double max_rel_residual;  /* largest true relative residual a stage solve ended with */
  double seconds;
} sc_spinodal_stats;

/*
 * Advance c by `nsteps` IMEX Runge-Kutta steps on a periodic grid. The
 * linear fourth-order part K(c) = -M kappa (L o L) c is implicit and the
 * non-linear part N(c) = M L f'(c) explicit, as in Sec. 4.1; L is `lap`
 * (the second-order 5- or 7-point Laplacian, p = 2, or in 2D a radius-2
 * cross Laplacian) and L o L its exact composition. Orders 1, 2 and 3 are
 * the L-stable, stiffly accurate pairs of Ascher, Ruuth and Spiteri (1997):
 * forward/backward Euler, ARS(2,2,2) and ARS(4,4,3); each implicit stage is
 * a CG solve of (I + dt a_ii M kappa L o L) Y_i = (explicit terms), started
 * from the previous stage, to opts->tol (true relative residual) in the
 * precision opts->precision (fast-Poisson preconditioning does not apply;
 * opts->precond must be SC_PC_NONE). c is FP64, any halo (the ring is not
 * touched), updated in place. Blocking: returns after the last step.
 * Errors: SC_EINVAL, SC_EUNSUPPORTED, SC_ENOMEM, SC_EDEVICE, SC_ENOTCONV /
 * SC_EBREAKDOWN from a stage (c then holds the last completed step).
 */
sc_status sc_spinodal_steps(const sc_stencil* lap, const sc_spinodal_params* p, int32_t nsteps,
                            const sc_solve_opts* opts, sc_grid* c, sc_spinodal_stats* stats,
                            sc_stream_t stream);
/*
 * Mass h^d sum c and the free energy of Sec. 4.1,
 * F = h^d sum [rho (c - c_alpha)^2 (c - c_beta)^2 + (kappa / 2) |grad c|^2]
 * with forward differences on the periodic grid (c FP64). Blocking.
 */
sc_status sc_spinodal_energy(const sc_grid* c, const sc_spinodal_params* p, double* mass, double* energy,
                             sc_stream_t stream);

/* ---------------------------------------------------------------------------
 * Assembled operator (the baseline the matrix-free apply is measured against)
 * ------------------------------------------------------------------------- */

typedef struct sc_csr sc_csr;

/* Which values the assembled rows reach: SC_CSR_PERIODIC wraps indices
 * modulo n (taps that alias to one column on grids narrower than the stencil
 * are summed into one entry); SC_CSR_ZERO_RING drops taps that leave the
 * grid, which is the operator of Krylov vectors with a zero ring (the BVP
 * matrix A of Sec. 3.3). */
typedef enum sc_csr_bc { SC_CSR_PERIODIC = 0, SC_CSR_ZERO_RING = 1 } sc_csr_bc;
/* rocSPARSE's CSR SpMV algorithm: row-split (no analysis, deterministic) or
 * adaptive (an analysis pass at the first product). */
typedef enum sc_csr_alg { SC_CSR_ROWSPLIT = 0, SC_CSR_ADAPTIVE = 1 } sc_csr_alg;

/*
 * Assemble stencil `s` on an n[0] x n[1] (x n[2]) grid of unknowns as a CSR
 * matrix in device memory, the assembled form in which the paper builds its
 * composed operators (Sec. 4.5-4.6; Table 3 counts its non-zeros, e.g. 13 per
 * row for the 13-point bi-Laplacian on a periodic grid). Row i = x + n0 (y +
 * n1 z) holds, for every tap t, the weight num_t/(den h^p) (rounded once, to
 * double and then to `dtype`, as in sc_apply_composed) in the column of grid
 * point (x, y, z) + u_t. Columns ascend within each row. Row pointers are
 * int64 (rows + 1 of them), column indices int32, so the grid must hold fewer
 * than 2^31 points; at most 128 taps. dim is 2 or 3 and equals the
 * stencil's; n[2] must be 1 in 2D. bc is an sc_csr_bc, dtype an sc_dtype,
 * alg an sc_csr_alg. Assembly runs on the current device on `stream` and the
 * call returns once it has completed. The library owns the matrix: release
 * it with sc_csr_free. Errors: SC_EINVAL, SC_EUNSUPPORTED (taps),
 * SC_ENOMEM, SC_EDEVICE.
 */
sc_status sc_csr_assemble(const sc_stencil* s, double h, int32_t dim, const int64_t* n, int32_t bc,
                          int32_t dtype, int32_t alg, sc_stream_t stream, sc_csr** out);
/* Rows, stored entries and device bytes of the three CSR arrays; NULL
 * outputs are skipped. */
sc_status sc_csr_info(const sc_csr* m, int64_t* rows, int64_t* nnz, uint64_t* bytes);
/*
 * y = A x by rocSPARSE on `stream`. x and y match the matrix's grid and
 * dtype, with halo 0 and contiguous storage (pitch[0] == n[0], and in 3D
 * pitch[1] == n[0] n[1]); y must not overlap x; the current device must be
 * the matrix's. The first product on a matrix also sizes and allocates the
 * library's SpMV workspace and runs its analysis (blocking); later products
 * are asynchronous. Calls on one matrix must not run concurrently from
 * several threads. Errors: SC_EINVAL, SC_ENOMEM, SC_EDEVICE.
 */
sc_status sc_csr_spmv(sc_csr* m, const sc_grid* x, sc_grid* y, sc_stream_t stream);
/* Copy the CSR arrays to caller-owned host buffers (rows + 1 int64 row
 * pointers, nnz int32 columns, nnz values of the matrix's dtype); NULL
 * buffers are skipped. Synchronous. */
sc_status sc_csr_export(const sc_csr* m, int64_t* row_ptr, int32_t* col, void* val);
/* Wait for the device, then release the matrix (NULL is ignored). */
void sc_csr_free(sc_csr* m);

/* ---------------------------------------------------------------------------
 * Errors and version
 * ------------------------------------------------------------------------- */

const char* sc_status_str(sc_status s);
/* Message of the last failing call on this thread ("" if none). */
const char* sc_last_error(void);
/* Library version string. */
const char* sc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SCOMP_H */
