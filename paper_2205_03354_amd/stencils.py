"""Named factor stencils of the paper, built with the library's exact algebra.

Only the one-dimensional factor weights are written out here (they are the
standard central differences the paper starts from); every multi-dimensional
or composed stencil is formed by ``stencil_lincomb`` / ``compose_stencil``.
"""

from __future__ import annotations

from ._native import Stencil, compose_stencil, stencil_lincomb


def _axis(dim: int, axis: int, offs, num, den: int, hpow: int) -> Stencil:
    taps = []
    for o in offs:
        t = [0, 0, 0]
        t[axis] = o
        taps.append(t)
    return Stencil.create(dim, taps, num, den, hpow)


def second_derivative(dim: int, axis: int, fourth_order: bool = False) -> Stencil:
    """(f_1 - 2 f_0 + f_-1)/h^2 (Sec. 2.1.2), or the fourth-order
    (-1, 16, -30, 16, -1)/(12 h^2), along one axis."""
    if fourth_order:
        return _axis(dim, axis, [-2, -1, 0, 1, 2], [-1, 16, -30, 16, -1], 12, 2)
    return _axis(dim, axis, [-1, 0, 1], [1, -2, 1], 1, 2)


def first_derivative(dim: int, axis: int) -> Stencil:
    """(f_1 - f_-1)/(2h) (Sec. 2.1.1)."""
    return _axis(dim, axis, [-1, 1], [-1, 1], 2, 1)


def laplacian(dim: int, fourth_order: bool = False) -> Stencil:
    """Sum of the second derivatives over the axes (5/7-point, or the
    9/13-point fourth-order cross)."""
    parts = [second_derivative(dim, a, fourth_order) for a in range(dim)]
    return stencil_lincomb([(1, 1, 0, p) for p in parts])


def biharmonic(dim: int, fourth_order: bool = False) -> Stencil:
    """The Laplacian composed with itself (Sec. 3.3): 13-point (2D),
    25-point (3D), or 33-point for the fourth-order factor in 2D."""
    L = laplacian(dim, fourth_order)
    return compose_stencil(L, L)


def flux_terms(dim: int, inner: Stencil):
    """Terms (D1_a o inner, D1_a) of div(M grad(inner f)) for apply_varcoef,
    with the central first derivative D1 (Sec. 2.2.3)."""
    terms = []
    for a in range(dim):
        d1 = first_derivative(dim, a)
        terms.append((compose_stencil(d1, inner), d1))
    return terms
