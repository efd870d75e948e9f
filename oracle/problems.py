"""Problem-level oracle: biharmonic BVP, Cahn-Hilliard step, diagnostics.

Test infrastructure only. Built from the naive loops in ``oracle.c`` and
plain numpy element-wise operations; every function follows the paper's
statement of the problem:

* ``bvp_rhs`` / ``bvp_solve``: the biharmonic boundary-value problem of
  Sec. 3.3 discretised with the Laplacian composed with itself. The unknowns
  are the nodes inside the prescribed ring; the ring values enter the right
  hand side: A u_I = f - A_ring(g), where A_ring(g) is the composed stencil
  applied to a field that holds g on the ring and zero at the unknowns.
* ``ch_rhs`` / ``ch_step``: one step of Cahn-Hilliard (Sec. 4.1,
  eq. (cahn)) with the linear fourth-order part implicit and the non-linear
  part explicit. The normalised form used here is
  u_t = Lap(u^3 - u - eps^2 Lap u) with a linear stabilisation S:
  (I + dt eps^2 L o L - dt S L) u^{n+1} = u^n + dt L((u^n)^3 - (1+S) u^n).
* ``ch_energy`` / ``mass``: the discrete free energy of Sec. 4.1 for the
  double well (u^2-1)^2/4 with gradient coefficient eps^2 (forward
  differences), and h^d sum u.
* ``apply_extended`` / ``bvp_relres_extended``: the same apply and BVP
  residual summed in x87 extended precision, for residual checks at grid
  sizes where an FP64 sum rounds near the 1e-10 stopping tolerance.
* ``flux_terms`` / ``varcoef_apply``: a composition with a varying
  coefficient between its factors (Sec. 2.2.3): y = sum_t B_t(M * A_t(x)),
  e.g. div(M grad(Lap f)) with A_a = D1_a o Lap and B_a = D1_a.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import capi
from . import rational as R


def bvp_rhs(op: R.RStencil, f: np.ndarray, g: np.ndarray, halo: int, h: float) -> np.ndarray:
    """b = f - A_ring(g) at the unknowns (A scaled by h^-p)."""
    ring = np.array(g, dtype=np.float64, copy=True)
    inner = tuple(slice(halo, s - halo) for s in ring.shape)
    ring[inner] = 0.0
    return f - capi.apply(op, ring, capi.HALO, halo, h)


def bvp_solve(op: R.RStencil, f: np.ndarray, g: np.ndarray, halo: int, h: float,
              tol: float = 1e-10, max_iter: int = 10**7):
    """Textbook CG from x0 = 0 on A x = b, A with a zero ring (Krylov vectors)."""
    b = bvp_rhs(op, f, g, halo, h)
    return capi.cg(op, b, None, capi.ZERO_RING, tol, max_iter, h)


def true_relres(op: R.RStencil, x: np.ndarray, b: np.ndarray, mode: int, h: float) -> float:
    """||b - A x||_2 / ||b||_2, FP64, by the oracle's own apply."""
    r = b - capi.apply(op, x, mode, 0, h)
    return float(np.linalg.norm(r.ravel()) / np.linalg.norm(b.ravel()))


def apply_extended(op: R.RStencil, x: np.ndarray, mode: int, halo: int = 0, h: float = 1.0) -> np.ndarray:
    """y = (1/h^p) W x at the unknowns, summed in x87 extended precision.

    The integer numerators multiply x in a 64-bit significand and the common
    denominator and h^p divide once at the end, so a sum whose FP64 rounding
    is large next to its value (a nearly converged residual of the
    bi-Laplacian at fine h, where |W||x| ~ 1e15 |W x|) keeps about three
    more digits. ``mode`` is ZERO_RING (x holds the unknowns) or HALO (x
    carries a ring of width ``halo``)."""
    if np.finfo(np.longdouble).nmant < 63:
        raise RuntimeError("extended precision is not available on this host")
    nums, den = op.integer_form()
    dim = op.dim
    xe = np.asarray(x, dtype=np.longdouble)
    if mode == capi.ZERO_RING:
        halo = op.radius()
        xe = np.pad(xe, halo)
    elif mode != capi.HALO:
        raise ValueError("mode must be ZERO_RING or HALO")
    shape = tuple(s - 2 * halo for s in xe.shape)
    acc = np.zeros(shape, dtype=np.longdouble)
    for off, num in sorted(nums.items()):
        # offset component a runs along numpy axis dim-1-a (x is the last axis)
        sl = tuple(slice(halo + off[dim - 1 - ax], halo + off[dim - 1 - ax] + shape[ax]) for ax in range(dim))
        acc += np.longdouble(num) * xe[sl]
    return acc / (np.longdouble(den) * np.longdouble(h) ** op.p)


def bvp_relres_extended(op: R.RStencil, x: np.ndarray, f: np.ndarray, g: np.ndarray, halo: int,
                        h: float) -> float:
    """||b - A x||_2 / ||b||_2 with b = f - A_ring(g), all in extended precision."""
    ring = np.array(g, dtype=np.longdouble, copy=True)
    ring[tuple(slice(halo, s - halo) for s in ring.shape)] = 0
    b = np.asarray(f, dtype=np.longdouble) - apply_extended(op, ring, capi.HALO, halo, h)
    r = b - apply_extended(op, x, capi.ZERO_RING, 0, h)
    return float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(b * b)))


def ch_operator(dim: int, h: float, eps: float, dt: float, S: float) -> R.RStencil:
    """I + dt eps^2 L o L - dt S L as an exact stencil when eps/h, dt/h^2 and
    S are exactly representable rationals (they are for the configurations
    used here: eps = 4h, dt = h^2/10, S = 2)."""
    e = Fraction(eps / h).limit_denominator(10**6)
    k = Fraction(dt / (h * h)).limit_denominator(10**6)
    s = Fraction(S).limit_denominator(10**6)
    return R.ch_operator(dim, e, k, s)


def ch_rhs(u: np.ndarray, h: float, dt: float, S: float) -> np.ndarray:
    """u + dt L(u^3 - (1+S) u), L the 5/7-point Laplacian (periodic)."""
    dim = u.ndim
    L = R.laplacian(dim)
    g = u * u * u - (1.0 + S) * u
    return u + dt * capi.apply(L, g, capi.PERIODIC, 0, h)


def ch_step(u: np.ndarray, h: float, eps: float, dt: float, S: float,
            tol: float = 1e-10, max_iter: int = 10**6):
    """One linearly stabilised semi-implicit step; CG from x0 = u^n.

    Returns (u^{n+1}, iterations, true relative residual, status).
    """
    A = ch_operator(u.ndim, h, eps, dt, S)
    rhs = ch_rhs(u, h, dt, S)
    return capi.cg(A, rhs, u, capi.PERIODIC, tol, max_iter, 1.0)


def mass(u: np.ndarray, h: float) -> float:
    return float(h ** u.ndim * np.sum(u))


def ch_energy(u: np.ndarray, h: float, eps: float) -> float:
    """h^d sum[(u^2-1)^2/4 + eps^2/2 sum_axes ((u_{i+e} - u_i)/h)^2] (periodic)."""
    bulk = 0.25 * (u * u - 1.0) ** 2
    grad = np.zeros_like(u)
    for ax in range(u.ndim):
        d = (np.roll(u, -1, axis=ax) - u) / h
        grad = grad + d * d
    return float(h ** u.ndim * np.sum(bulk + 0.5 * eps * eps * grad))


# -- variable-coefficient composition ----------------------------------------

def flux_terms(dim: int, inner: R.RStencil):
    """The terms (A_a, B_a) of div(M grad(inner f)) with central first
    derivatives: A_a = D1_a o inner, B_a = D1_a (Sec. 2.2.3: the inner part is
    composed first, scaled pointwise by the mobility M, and the result is
    composed with the outer first derivative)."""
    terms = []
    for a in range(dim):
        d1 = R.embed(R.central_first(), a, dim)
        terms.append((R.compose(d1, inner), d1))
    return terms


def varcoef_apply(terms, M: np.ndarray, x: np.ndarray, mode: int, halo: int = 0, h: float = 1.0) -> np.ndarray:
    """y = sum_t B_t(M * A_t(x)), by definition: each inner stencil applied to
    x, the result multiplied pointwise by M, the outer stencil applied to that.

    PERIODIC: x and M have the grid's shape. HALO: x carries a ring of width
    halo >= rA + rB (rA, rB the largest inner and outer radii) and M a ring of
    width halo - rA around the grid, so that M * A_t(x) is defined on the
    grid plus the ring the outer stencils read."""
    y = None
    if mode == capi.PERIODIC:
        for A, B in terms:
            w = M * capi.apply(A, x, capi.PERIODIC, 0, h)
            t = capi.apply(B, w, capi.PERIODIC, 0, h)
            y = t if y is None else y + t
        return y
    rA = max(A.radius() for A, _ in terms)
    rB = halo - rA
    if rB < max(B.radius() for _, B in terms):
        raise ValueError("halo must cover the inner plus the outer radius")
    for A, B in terms:
        w = M * capi.apply(A, x, capi.HALO, rA, h)  # on the grid plus a ring of width rB
        t = capi.apply(B, w, capi.HALO, rB, h)
        y = t if y is None else y + t
    return y
