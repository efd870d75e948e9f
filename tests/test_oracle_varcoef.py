"""Pins of the variable-coefficient oracle y = sum_a B_a(M * A_a(x)).

The operator is div(M grad(L f)) discretised by composition (Sec. 2.2.3):
the inner part D1_a o L is composed first, scaled pointwise by the mobility
M, then composed with the outer central first derivative D1_a. Pins:
* M = 1 reduces it to the constant composed stencil sum_a D1_a o D1_a o L,
  built by exact rational composition (bit-exact on integer inputs);
* a constant M = c scales the M = 1 result by c;
* the dense product sum_a B_a diag(M) A_a on small periodic grids;
* a manufactured solution with a smooth varying mobility converges at second
  order to the analytic div(M grad(Lap f)).
"""

import math

import numpy as np
import pytest

import synthetic as S
from oracle import capi
from oracle import problems as OP
from oracle import rational as R


def _constant_operator(dim, inner):
    total = None
    for a in range(dim):
        d1 = R.embed(R.central_first(), a, dim)
        t = R.compose(d1, R.compose(d1, inner))
        total = t if total is None else R.add(total, t)
    return total


@pytest.mark.parametrize("dim", [2, 3])
def test_unit_mobility_is_the_composed_stencil(dim):
    L = R.laplacian(dim)
    terms = OP.flux_terms(dim, L)
    C = _constant_operator(dim, L)
    assert C.radius() == 3
    shape = (9, 11, 13)[:dim]
    x = S.integer_field(shape, seed=11, lo=-64, hi=64)
    M = np.ones(shape)
    y = OP.varcoef_apply(terms, M, x, capi.PERIODIC)
    assert np.array_equal(y, capi.apply(C, x, capi.PERIODIC))
    # halo mode: ring 3 = inner radius 2 + outer radius 1; M on the grid + 1
    xh = S.integer_field(tuple(s + 6 for s in shape), seed=12, lo=-64, hi=64)
    Mh = np.ones(tuple(s + 2 for s in shape))
    yh = OP.varcoef_apply(terms, Mh, xh, capi.HALO, 3)
    assert np.array_equal(yh, capi.apply(C, xh, capi.HALO, 3))


def test_constant_mobility_scales():
    L = R.laplacian(2)
    terms = OP.flux_terms(2, L)
    x = S.uniform_field((12, 10), seed=3)
    y1 = OP.varcoef_apply(terms, np.ones((12, 10)), x, capi.PERIODIC)
    y4 = OP.varcoef_apply(terms, np.full((12, 10), 4.0), x, capi.PERIODIC)
    assert np.array_equal(y4, 4.0 * y1)


@pytest.mark.parametrize("fourth", [False, True])
def test_dense_product_on_small_periodic_grid(fourth):
    dim = 2
    L = R.laplacian(dim, fourth)
    terms = OP.flux_terms(dim, L)
    n = (7, 6)  # (n0, n1); numpy arrays are (n1, n0)
    x = S.uniform_field((n[1], n[0]), seed=5)
    M = 1.0 + 0.5 * S.uniform_field((n[1], n[0]), seed=6)
    y = OP.varcoef_apply(terms, M, x, capi.PERIODIC)
    dense = np.zeros((n[0] * n[1], n[0] * n[1]))
    for A, B in terms:
        dense += R.assemble_dense(B, n, True) @ np.diag(M.reshape(-1)) @ R.assemble_dense(A, n, True)
    ref = (dense @ x.reshape(-1)).reshape(x.shape)
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


def _manufactured(N):
    h = 1.0 / N
    c = np.arange(N) * h
    X, Y = np.meshgrid(c, c, indexing="xy")  # arrays (n1, n0): x along the last axis
    k = 2 * math.pi
    f = np.sin(k * X) * np.sin(k * Y)
    M = 1.0 + 0.5 * np.cos(k * X)
    # Lap f = -2 k^2 f; div(M grad(Lap f)) = -2 k^2 (dM/dx df/dx + M Lap f)
    dM = -0.5 * k * np.sin(k * X)
    fx = k * np.cos(k * X) * np.sin(k * Y)
    exact = -2 * k * k * (dM * fx + M * (-2 * k * k) * f)
    return f, M, exact, h


def test_manufactured_variable_mobility_second_order():
    terms = OP.flux_terms(2, R.laplacian(2))
    errs, hs = [], []
    for N in (32, 64, 128):
        f, M, exact, h = _manufactured(N)
        y = OP.varcoef_apply(terms, M, f, capi.PERIODIC, h=h)
        errs.append(np.max(np.abs(y - exact)) / np.max(np.abs(exact)))
        hs.append(h)
    rate = math.log(errs[1] / errs[2]) / math.log(hs[1] / hs[2])
    assert abs(rate - 2.0) < 0.1, (errs, rate)


def test_halo_mode_matches_periodic_embedding():
    # A periodic field, padded with its own periodic images, gives the same
    # result in halo mode (ring 3 for x, ring 1 for M).
    terms = OP.flux_terms(2, R.laplacian(2))
    x = S.uniform_field((10, 14), seed=8)
    M = 1.0 + 0.25 * S.uniform_field((10, 14), seed=9)
    y = OP.varcoef_apply(terms, M, x, capi.PERIODIC)
    xh = np.pad(x, 3, mode="wrap")
    Mh = np.pad(M, 1, mode="wrap")
    yh = OP.varcoef_apply(terms, Mh, xh, capi.HALO, 3)
    assert np.max(np.abs(yh - y)) <= 1e-13 * np.max(np.abs(y))
