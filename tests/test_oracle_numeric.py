"""Pins of the oracle's naive apply, CG, BVP and Cahn-Hilliard step.

Each check ties the oracle to something other than itself: a dense
matrix-vector product, a trigonometric closed form, a library linear solve,
the paper's stated convergence order, or conservation laws.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import synthetic as S
from oracle import capi
from oracle import problems as P
from oracle import rational as R


def test_apply_periodic_equals_dense_matvec():
    for st in [R.biharmonic(2), R.compose(R.embed(R.forward_first(), 0, 2), R.laplacian(2, True))]:
        for n in (3, 5, 8):
            x = S.uniform_field((n + 1, n), seed=n)
            M = R.assemble_dense(st, (n, n + 1), True)
            y = capi.apply(st, x, capi.PERIODIC)
            np.testing.assert_allclose(y.ravel(), M @ x.ravel(), rtol=1e-13, atol=1e-12)
            y0 = capi.apply(st, x, capi.ZERO_RING)
            M0 = R.assemble_dense(st, (n, n + 1), False)
            np.testing.assert_allclose(y0.ravel(), M0 @ x.ravel(), rtol=1e-13, atol=1e-12)


def test_apply_fourier_mode_nonsymmetric():
    # A periodic mode exp(i theta . x) is an eigenvector with eigenvalue
    # sigma(theta) = sum w exp(i theta . u); a transposed offset or a sign
    # error turns sigma into its conjugate, which the sine part detects.
    st = R.compose(R.embed(R.forward_first(), 0, 2), R.embed(R.central_second_4th(), 1, 2))
    n0, n1 = 24, 20
    k0, k1 = 5, 3
    j, i = np.meshgrid(np.arange(n1), np.arange(n0), indexing="ij")
    ph = 2 * math.pi * (k0 * i / n0 + k1 * j / n1)
    sig = R.symbol(st, np.array([2 * math.pi * k0 / n0, 2 * math.pi * k1 / n1]))
    yc = capi.apply(st, np.cos(ph), capi.PERIODIC)
    ys = capi.apply(st, np.sin(ph), capi.PERIODIC)
    z = sig * np.exp(1j * ph)
    np.testing.assert_allclose(yc, z.real, atol=1e-12)
    np.testing.assert_allclose(ys, z.imag, atol=1e-12)


def test_apply_3d_fourier_mode():
    st = R.biharmonic(3)
    n = (6, 7, 8)  # (n2, n1, n0) in numpy order
    kv = (1, 2, 3)
    x = S.periodic_cos_mode(n, kv)
    th = np.array([2 * math.pi * kv[0] / n[2], 2 * math.pi * kv[1] / n[1], 2 * math.pi * kv[2] / n[0]])
    np.testing.assert_allclose(capi.apply(st, x, capi.PERIODIC), R.symbol(st, th).real * x, atol=1e-11)


@pytest.mark.parametrize("fourth", [False, True])
def test_composed_equals_sequential_integer_exact(fourth):
    # Composed apply on the unknowns with a prescribed ring equals applying the
    # inner factor on unknowns + ring and then the outer factor, bit-exact for
    # integer data (all partial sums are exact in FP64).
    L = R.laplacian(2, fourth)
    C = R.compose(L, L)
    r = L.radius()
    n = 13
    x = S.integer_field((n + 4 * r, n + 4 * r), seed=3)
    # unscaled integer weights keep every product and partial sum exact
    nums, den = L.integer_form()
    Li = R.RStencil(2, 0, {o: v for o, v in nums.items()})
    numsc, denc = C.integer_form()
    Ci = R.RStencil(2, 0, {o: v for o, v in numsc.items()})
    inner = capi.apply(Li, x, capi.HALO, r)          # on unknowns + ring r
    seq = capi.apply(Li, inner, capi.HALO, r)
    comp = capi.apply(Ci, x, capi.HALO, 2 * r)
    assert den * den == denc
    assert np.array_equal(seq, comp)


def test_manufactured_order_33pt_and_13pt():
    # Periodic sin(2 pi x) sin(2 pi y): Delta^2 u = 64 pi^4 u. The composed
    # fourth-order operator converges at order 4 and the composed
    # second-order one at order 2 (Lemma (Accuracy)); grids stay at N <= 128
    # where truncation error dominates rounding.
    for st, order in [(R.biharmonic(2, True), 4), (R.biharmonic(2, False), 2)]:
        errs, hs = [], []
        for N in (16, 32, 64, 128):
            u, h = S.periodic_sin_mode(2, N)
            y = capi.apply(st, u, capi.PERIODIC, 0, h)
            errs.append(np.abs(y - 64 * math.pi ** 4 * u).max())
            hs.append(h)
        rates = [math.log(errs[i] / errs[i + 1]) / math.log(hs[i] / hs[i + 1]) for i in range(3)]
        assert abs(rates[-1] - order) < 0.1, rates


def test_cg_matches_dense_solve():
    st = R.biharmonic(2)
    n = 7
    b = S.uniform_field((n, n), seed=11)
    x, it, rel, rc = capi.cg(st, b, None, capi.ZERO_RING, 1e-13)
    M = R.assemble_dense(st, (n, n), False)
    ref = np.linalg.solve(M, b.ravel())
    assert rc == 0 and rel <= 1e-13
    np.testing.assert_allclose(x.ravel(), ref, rtol=1e-10, atol=1e-12)


def test_bvp_matches_dense_solve_17():
    bvp = S.biharmonic_bvp(2, 17)
    op = R.biharmonic(2)
    x, it, rel, rc = P.bvp_solve(op, bvp.f, bvp.g, bvp.halo, bvp.h, tol=1e-12)
    b = P.bvp_rhs(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    M = R.assemble_dense(op, (bvp.n, bvp.n), False, bvp.h)
    ref = np.linalg.solve(M, b.ravel())
    np.testing.assert_allclose(x.ravel(), ref, rtol=1e-9)


def _exact_zero_ring_apply(op, x):
    # brute force in rational arithmetic: y_i = sum_k w_k x_{i+o_k}, zero outside
    dim = op.dim
    y = np.empty(x.shape, dtype=object)
    for idx in np.ndindex(*x.shape):
        acc = Fraction(0)
        for off, w in op.weights.items():
            j = tuple(idx[ax] + off[dim - 1 - ax] for ax in range(dim))
            if all(0 <= j[ax] < x.shape[ax] for ax in range(dim)):
                acc += w * Fraction(float(x[j]))
        y[idx] = acc
    return y


@pytest.mark.parametrize("dim,fourth", [(2, False), (2, True), (3, False)])
def test_extended_apply_pins(dim, fourth):
    op = R.biharmonic(dim, fourth) if dim == 2 else R.biharmonic(3)
    rad = op.radius()
    nums, den = op.integer_form()
    wsum = sum(abs(v) for v in nums.values())
    shape = (7, 6, 5)[:dim]
    # brute force: exact rational sums on a tiny grid
    xr = S.uniform_field(shape, seed=43)
    ex = _exact_zero_ring_apply(op, xr)
    got = P.apply_extended(op, xr, capi.ZERO_RING)
    err = max(abs(Fraction(float(g)) - e) for g, e in zip(got.ravel(), ex.ravel()))
    assert err <= Fraction(1, 2 ** 50) * wsum / den
    # integer inputs: the numerator sums are exact in both precisions
    xi = S.integer_field(shape, seed=41)
    ext = P.apply_extended(op, xi, capi.ZERO_RING)
    assert np.array_equal(np.rint(ext * den), np.vectorize(lambda v: float(v * den))(_exact_zero_ring_apply(op, xi)))
    if den == 1:
        assert np.array_equal(ext.astype(np.float64), capi.apply(op, xi, capi.ZERO_RING))
    # halo mode is the zero-ring apply of the unknowns plus the ring's part
    xh = S.uniform_field(tuple(s + 2 * rad for s in shape), seed=44)
    inner = tuple(slice(rad, s - rad) for s in xh.shape)
    ring = xh.copy()
    ring[inner] = 0.0
    lhs = P.apply_extended(op, xh, capi.HALO, rad)
    rhs = P.apply_extended(op, xh[inner], capi.ZERO_RING) + P.apply_extended(op, ring, capi.HALO, rad)
    assert float(np.max(np.abs(lhs - rhs))) <= 2.0 ** -58 * wsum / den
    # an exactly linear field with full 53-bit values (1 + c (2^-30 + 2^-52),
    # c < 64) is annihilated; its products and partial sums need up to 66 bits
    c = np.indices(tuple(s + 2 * rad for s in shape)).sum(axis=0).astype(np.float64)
    lin = 1.0 + c * (2.0 ** -30 + 2.0 ** -52)
    e_ext = float(np.max(np.abs(P.apply_extended(op, lin, capi.HALO, rad)))) * den
    e_64 = float(np.max(np.abs(capi.apply(op, lin, capi.HALO, rad)))) * den
    assert e_ext <= 2.0 ** -60 * wsum * 2
    if max(abs(v) for v in nums.values()) <= 64:
        assert e_ext == 0.0 and e_64 > 0.0


def test_extended_residual_matches_fp64_where_fp64_is_accurate():
    bvp = S.biharmonic_bvp(2, 33)
    op = R.biharmonic(2)
    x, it, rel, rc = P.bvp_solve(op, bvp.f, bvp.g, bvp.halo, bvp.h, tol=1e-8)
    b = P.bvp_rhs(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    r64 = P.true_relres(op, x, b, capi.ZERO_RING, bvp.h)
    rext = P.bvp_relres_extended(op, x, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert abs(rext - r64) <= 1e-6 * r64


@pytest.mark.parametrize("N", [17, 33, 65])
def test_bvp_odd_reflection_closed_form(N):
    # Simply supported plate (Sec. 3.3): with u = 0 on the boundary and odd
    # reflection beyond it, L o L reduces to L_II^2 and sin(pi x) sin(pi y) is
    # an eigenvector with eigenvalue mu^2, mu = -(8/h^2) sin^2(pi h / 2):
    # the discrete solution is (4 pi^4 / mu^2) phi and CG needs one step (up
    # to the FP64 rounding floor of an h^-4 operator, ~ 1e-16 sum|w| / mu^2,
    # which reaches 1e-10 at N = 65, hence the tolerance).
    bvp = S.biharmonic_bvp(2, N)
    op = R.biharmonic(2)
    h = bvp.h
    mu = -(8.0 / h ** 2) * math.sin(math.pi * h / 2) ** 2
    exact_discrete = 4 * math.pi ** 4 / mu ** 2 * bvp.u
    x, it, rel, rc = capi.cg(op, bvp.f, None, capi.ODD_REFLECT, 1e-9, 100, h)
    assert rc == 0 and it <= 3
    np.testing.assert_allclose(x, exact_discrete, rtol=1e-9, atol=1e-12)


def test_bvp_second_order_convergence():
    # Sec. 3.3: the composed second-order Laplacian keeps second order; the
    # observed order between the two finest grids is within 0.1 of 2.
    op = R.biharmonic(2)
    errs, hs = [], []
    for N in (17, 33, 65):
        bvp = S.biharmonic_bvp(2, N)
        x, it, rel, rc = P.bvp_solve(op, bvp.f, bvp.g, bvp.halo, bvp.h, tol=1e-10)
        assert rc == 0 and rel <= 1e-10
        errs.append(np.abs(x - bvp.u).max())
        hs.append(bvp.h)
    rate = math.log(errs[1] / errs[2]) / math.log(hs[1] / hs[2])
    assert abs(rate - 2) < 0.1


def test_bvp3d_second_order_convergence():
    op = R.biharmonic(3)
    errs, hs = [], []
    for n in (7, 15, 31):
        bvp = S.biharmonic_bvp(3, n)
        x, it, rel, rc = P.bvp_solve(op, bvp.f, bvp.g, bvp.halo, bvp.h, tol=1e-10)
        assert rc == 0 and rel <= 1e-10
        errs.append(np.abs(x - bvp.u).max())
        hs.append(bvp.h)
    rate = math.log(errs[1] / errs[2]) / math.log(hs[1] / hs[2])
    assert abs(rate - 2) < 0.15


def _ch_mode_closed_form(a, N, k, eps, dt, Sst):
    # u = a cos(phi), phi = 2 pi (k0 i + k1 j)/N. cos^3 = (3 cos + cos 3.)/4.
    h = 1.0 / N
    th = 2 * math.pi * np.array(k) / N

    def sig(t):  # symbol of the 5-point Laplacian / h^2
        return (2 * math.cos(t[0]) - 2 + 2 * math.cos(t[1]) - 2) / h ** 2

    s1, s3 = sig(th), sig(3 * th)
    r1 = a + dt * s1 * (0.75 * a ** 3 - (1 + Sst) * a)
    r3 = dt * s3 * 0.25 * a ** 3
    c1 = r1 / (1 + dt * eps ** 2 * s1 ** 2 - dt * Sst * s1)
    c3 = r3 / (1 + dt * eps ** 2 * s3 ** 2 - dt * Sst * s3)
    j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ph = 2 * math.pi * (k[0] * i + k[1] * j) / N
    return a * np.cos(ph), c1 * np.cos(ph) + c3 * np.cos(3 * ph)


def test_ch_step_single_mode_closed_form():
    N = 32
    h = 1.0 / N
    eps, dt, Sst = 4 * h, 0.1 * h * h, 2.0
    u0, expect = _ch_mode_closed_form(0.3, N, (2, 1), eps, dt, Sst)
    u1, it, rel, rc = P.ch_step(u0, h, eps, dt, Sst, tol=1e-14)
    assert rc == 0
    np.testing.assert_allclose(u1, expect, atol=1e-13)


def test_ch_constant_state_is_fixed_point():
    N = 16
    h = 1.0 / N
    u = np.full((N, N), 0.37)
    u1, it, rel, rc = P.ch_step(u, h, 4 * h, 0.1 * h * h, 2.0)
    np.testing.assert_allclose(u1, u, atol=1e-15)


def test_ch_energy_closed_form_and_summation_by_parts():
    N, k, a = 32, 3, 0.4
    h = 1.0 / N
    eps = 4 * h
    u = a * S.periodic_cos_mode((N, N), (k, 0))
    E = P.ch_energy(u, h, eps)
    expect = (3 * a ** 4 / 8 - a ** 2 + 1) / 4 + eps ** 2 * a ** 2 * N ** 2 * math.sin(math.pi * k / N) ** 2
    assert abs(E - expect) < 1e-13
    grad = -0.5 * eps ** 2 * h ** 2 * float(np.sum(u * capi.apply(R.laplacian(2), u, capi.PERIODIC, 0, h)))
    bulk = h ** 2 * float(np.sum(0.25 * (u * u - 1) ** 2))
    assert abs(E - (bulk + grad)) < 1e-13


@pytest.mark.parametrize("dim,N,steps", [(2, 64, 12), (3, 16, 6)])
def test_ch_mass_and_energy(dim, N, steps):
    h = 1.0 / N
    eps, dt, Sst = 4 * h, 0.1 * h * h, 2.0
    u = S.zero_mean_uniform((N,) * dim, seed=7)
    m0 = u.mean()
    E = [P.ch_energy(u, h, eps)]
    for _ in range(steps):
        u, it, rel, rc = P.ch_step(u, h, eps, dt, Sst)
        assert rc == 0 and rel <= 1e-10
        assert abs(u.mean() - m0) <= 1e-12
        E.append(P.ch_energy(u, h, eps))
    assert all(E[i + 1] <= E[i] + 1e-14 * abs(E[i]) for i in range(steps))
    assert E[-1] < E[0]
