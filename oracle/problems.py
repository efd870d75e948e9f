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
