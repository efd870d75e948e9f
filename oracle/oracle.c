/*
 * Naive FP64 reference loops for the stencil-composition oracle.
 *
 * TEST INFRASTRUCTURE ONLY: this file is part of the independent CPU oracle.
 * It shares no code with the GPU library and is only loaded by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark.
 *
 * Built with -O2 -ffp-contract=off so that every product and sum is rounded
 * separately (no fused multiply-add), and OpenMP over the slowest output
 * axis only: each output point is computed by one thread in a fixed tap
 * order, so results do not depend on the thread count. Dot products are
 * serial sums in index order.
 *
 * Conventions
 *   Arrays are contiguous with x fastest: element (i, j, k) of an n0 x n1 x n2
 *   grid sits at i + n0 * (j + n1 * k). A 2D grid has n2 = 1.
 *   A stencil is npts taps, offsets (ox, oy, oz) int32 triples and weights
 *   double; the weight already contains the h^-p scale.
 *   Output point (i, j, k) = sum_t w_t * in(i + ox_t, j + oy_t, k + oz_t)
 *   (the definition of applying a stencil, Sec. 2.1; for a composed stencil
 *   the taps come from eq. (C=B(A))).
 *
 * Boundary modes for reading in(.) outside the grid:
 *   OR_PERIODIC  : indices taken modulo n (true modulo, so offsets larger
 *                  than the grid alias correctly);
 *   OR_ZERO_RING : values outside the grid are zero (the operator restricted
 *                  to the unknowns, as used for Krylov vectors of a BVP);
 *   OR_HALO      : the input array carries a ring of width `halo` on every
 *                  active axis and values are read from it;
 *   OR_ODD_REFLECT: the boundary nodes just outside the grid hold zero and
 *                  values further out are the negated mirror images of the
 *                  interior (the simply supported plate of Sec. 3.3: f = 0
 *                  and a vanishing second normal derivative).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PERIODIC 0
#define OR_ZERO_RING 1
#define OR_HALO 2
#define OR_ODD_REFLECT 3

static int64_t pmod(int64_t a, int64_t n) {
  int64_t r = a % n;
  return r < 0 ? r + n : r;
}

/*
 * Odd reflection about the boundary nodes at index -1 and n (whose value is
 * zero): index -2 - a mirrors a < -1 and 2n - a mirrors a > n, each mirror
 * flipping the sign. Returns -1 when the index lands on a boundary node.
 */
static int64_t reflect(int64_t a, int64_t n, double* sign) {
  for (;;) {
    if (a == -1 || a == n) return -1;
    if (a < -1) { a = -2 - a; *sign = -*sign; continue; }
    if (a > n) { a = 2 * n - a; *sign = -*sign; continue; }
    return a;
  }
}

/* y = W in, for one of the boundary modes above. */
int or_apply(int dim, const int64_t* n, int mode, int halo, const double* in,
             int npts, const int32_t* off, const double* w, double* y) {
  if (dim < 1 || dim > 3 || npts < 0) return 1;
  int64_t n0 = n[0], n1 = dim > 1 ? n[1] : 1, n2 = dim > 2 ? n[2] : 1;
  int64_t H = (mode == OR_HALO) ? halo : 0;
  int64_t m0 = n0 + 2 * H, m1 = dim > 1 ? n1 + 2 * H : 1;
  int64_t H1 = dim > 1 ? H : 0, H2 = dim > 2 ? H : 0;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n2; ++k) {
    for (int64_t j = 0; j < n1; ++j) {
      for (int64_t i = 0; i < n0; ++i) {
        double acc = 0.0;
        for (int t = 0; t < npts; ++t) {
          int64_t a = i + off[3 * t + 0];
          int64_t b = j + off[3 * t + 1];
          int64_t c = k + off[3 * t + 2];
          double v;
          if (mode == OR_PERIODIC) {
            v = in[pmod(a, n0) + n0 * (pmod(b, n1) + n1 * pmod(c, n2))];
          } else if (mode == OR_ZERO_RING) {
            if (a < 0 || a >= n0 || b < 0 || b >= n1 || c < 0 || c >= n2)
              v = 0.0;
            else
              v = in[a + n0 * (b + n1 * c)];
          } else if (mode == OR_ODD_REFLECT) {
            double s = 1.0;
            int64_t ra = reflect(a, n0, &s);
            int64_t rb = dim > 1 ? reflect(b, n1, &s) : b;
            int64_t rc = dim > 2 ? reflect(c, n2, &s) : c;
            if (ra < 0 || rb < 0 || rc < 0)
              v = 0.0;
            else
              v = s * in[ra + n0 * (rb + n1 * rc)];
          } else {
            v = in[(a + H) + m0 * ((b + H1) + m1 * (c + H2))];
          }
          acc = acc + w[t] * v;
        }
        y[i + n0 * (j + n1 * k)] = acc;
      }
    }
  }
  return 0;
}

static double dot(int64_t N, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t i = 0; i < N; ++i) s = s + a[i] * b[i];
  return s;
}

/*
 * Textbook conjugate gradients (Hestenes-Stiefel, no preconditioner) on
 * W x = b, with W the stencil in OR_PERIODIC, OR_ZERO_RING or
 * OR_ODD_REFLECT mode. The
 * operator must be symmetric positive definite on the vectors it acts on.
 *
 * Stops when the recurrence residual satisfies ||r|| <= tol ||b||, then
 * recomputes the true residual b - W x; if that fails the test the
 * recurrence is restarted from the true residual (at most max_iter
 * iterations in total).
 *
 * Returns 0 on convergence, 2 on breakdown (p.Wp <= 0 or not finite),
 * 3 if max_iter was reached. iters and relres (true ||b-Wx||/||b||) are
 * always written.
 */
int or_cg(int dim, const int64_t* n, int mode, int npts, const int32_t* off,
          const double* w, const double* b, double* x, double tol,
          int64_t max_iter, int64_t* iters, double* relres) {
  int64_t N = n[0] * (dim > 1 ? n[1] : 1) * (dim > 2 ? n[2] : 1);
  double* r = (double*)malloc(sizeof(double) * N);
  double* p = (double*)malloc(sizeof(double) * N);
  double* q = (double*)malloc(sizeof(double) * N);
  if (!r || !p || !q) {
    free(r); free(p); free(q);
    return 4;
  }
  double bnorm = sqrt(dot(N, b, b));
  int status = 3;
  int64_t it = 0;
  if (bnorm == 0.0) {
    memset(x, 0, sizeof(double) * N);
    *iters = 0;
    *relres = 0.0;
    free(r); free(p); free(q);
    return 0;
  }
  for (;;) {
    /* (re)start from the true residual */
    or_apply(dim, n, mode, 0, x, npts, off, w, q);
    for (int64_t i = 0; i < N; ++i) r[i] = b[i] - q[i];
    double rr = dot(N, r, r);
    if (sqrt(rr) <= tol * bnorm) { status = 0; break; }
    memcpy(p, r, sizeof(double) * N);
    int restart = 0;
    while (it < max_iter) {
      or_apply(dim, n, mode, 0, p, npts, off, w, q);
      double pq = dot(N, p, q);
      if (!(pq > 0.0) || !isfinite(pq)) { status = 2; goto done; }
      double alpha = rr / pq;
      for (int64_t i = 0; i < N; ++i) x[i] = x[i] + alpha * p[i];
      for (int64_t i = 0; i < N; ++i) r[i] = r[i] - alpha * q[i];
      double rr_new = dot(N, r, r);
      ++it;
      if (sqrt(rr_new) <= tol * bnorm) { restart = 1; break; }
      double beta = rr_new / rr;
      for (int64_t i = 0; i < N; ++i) p[i] = r[i] + beta * p[i];
      rr = rr_new;
    }
    if (!restart) { status = 3; break; }
    /* recurrence converged: verify the true residual at the top of the loop */
  }
done:
  or_apply(dim, n, mode, 0, x, npts, off, w, q);
  for (int64_t i = 0; i < N; ++i) r[i] = b[i] - q[i];
  *relres = sqrt(dot(N, r, r)) / bnorm;
  *iters = it;
  free(r); free(p); free(q);
  return status;
}

/* Number of OpenMP threads the apply loop uses. */
int or_threads(void) { return omp_get_max_threads(); }
