"""Oracle for the spinodal-decomposition benchmark of Sec. 4 with IMEX time
stepping of orders 1-3 (test infrastructure only).

The model (Sec. 4.1, eq. (cahn)): the concentration c evolves by
    c_t = div(M grad(f_chem'(c) - kappa Lap c)),
    f_chem(c) = rho (c - c_alpha)^2 (c - c_beta)^2,
with constant mobility M, so c_t = M Lap f_chem'(c) - M kappa Lap^2 c. On a
periodic grid with the composed stencils this is the ODE system
    c' = N(c) + K(c),   N(c) = M L f'(c)   (explicit, non-linear),
                        K(c) = -M kappa (L o L) c   (implicit, linear),
L the 5/7-point Laplacian (Sec. 4.1 treats the fourth-order linear part
implicitly and the non-linear part explicitly).

Time stepping: implicit-explicit Runge-Kutta methods written as a pair of
Butcher tableaux (explicit Ahat, bhat; implicit A, b) over stages
0 .. s, stage 0 explicit:
    Y_i = c^n + dt sum_{j<i} Ahat_ij N(Y_j) + dt sum_{j<=i} A_ij K(Y_j),
    c^{n+1} = c^n + dt sum_j bhat_j N(Y_j) + dt sum_j b_j K(Y_j),
each stage an SPD solve (I + dt A_ii M kappa L o L) Y_i = (known terms).
The paper names only the orders (1, 2, 3); the schemes used are the
L-stable ones of Ascher, Ruuth and Spiteri (Appl. Numer. Math. 25, 1997):
order 1 forward/backward Euler, ARS(2,2,2), ARS(4,4,3).

Every solve is the oracle's textbook CG (oracle.c) to a true relative
residual ``tol``; every stencil application the oracle's naive FP64 apply.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction
from typing import List

import numpy as np

from . import capi
from . import rational as R


@dataclass
class Tableau:
    order: int
    Ahat: List[List[float]]  # explicit, strictly lower triangular
    bhat: List[float]
    A: List[List[float]]     # implicit, lower triangular, A[0][0] = 0
    b: List[float]


def _exact(rows):
    return [[Fraction(v) for v in r] for r in rows]


def tableau_exact(order: int):
    """The order-1 and order-3 pairs in exact rationals (order 2 has an
    irrational diagonal and is returned by ``tableau`` only)."""
    if order == 1:
        Ahat = _exact([[0, 0], [1, 0]])
        A = _exact([[0, 0], [0, 1]])
        return Ahat, [Fraction(1), Fraction(0)], A, [Fraction(0), Fraction(1)]
    if order == 3:
        F = Fraction
        Ahat = [[F(0)] * 5,
                [F(1, 2), F(0), F(0), F(0), F(0)],
                [F(11, 18), F(1, 18), F(0), F(0), F(0)],
                [F(5, 6), F(-5, 6), F(1, 2), F(0), F(0)],
                [F(1, 4), F(7, 4), F(3, 4), F(-7, 4), F(0)]]
        A = [[F(0)] * 5,
             [F(0), F(1, 2), F(0), F(0), F(0)],
             [F(0), F(1, 6), F(1, 2), F(0), F(0)],
             [F(0), F(-1, 2), F(1, 2), F(1, 2), F(0)],
             [F(0), F(3, 2), F(-3, 2), F(1, 2), F(1, 2)]]
        return Ahat, list(Ahat[4]), A, list(A[4])
    raise ValueError("exact tableaux exist for orders 1 and 3")


def tableau(order: int) -> Tableau:
    if order in (1, 3):
        Ahat, bhat, A, b = tableau_exact(order)
        f = lambda m: [[float(v) for v in r] for r in m]  # noqa: E731
        return Tableau(order, f(Ahat), [float(v) for v in bhat], f(A), [float(v) for v in b])
    if order == 2:
        g = 1.0 - 1.0 / math.sqrt(2.0)
        d = 1.0 - 1.0 / (2.0 * g)
        Ahat = [[0.0, 0.0, 0.0], [g, 0.0, 0.0], [d, 1.0 - d, 0.0]]
        A = [[0.0, 0.0, 0.0], [0.0, g, 0.0], [0.0, 1.0 - g, g]]
        return Tableau(2, Ahat, [d, 1.0 - d, 0.0], A, [0.0, 1.0 - g, g])
    raise ValueError("order must be 1, 2 or 3")


@dataclass
class Params:
    h: float = 1.0
    M: float = 5.0
    kappa: float = 2.0
    rho: float = 5.0
    ca: float = 0.3
    cb: float = 0.7


def fprime(c: np.ndarray, p: Params) -> np.ndarray:
    """d f_chem / dc = 2 rho (c - ca)(c - cb)(2c - ca - cb)."""
    return 2.0 * p.rho * (c - p.ca) * (c - p.cb) * (2.0 * c - p.ca - p.cb)


def explicit_part(c: np.ndarray, p: Params) -> np.ndarray:
    """N(c) = M L f'(c) (periodic)."""
    L = R.laplacian(c.ndim)
    return p.M * capi.apply(L, fprime(c, p), capi.PERIODIC, 0, p.h)


def implicit_part(c: np.ndarray, p: Params) -> np.ndarray:
    """K(c) = -M kappa (L o L) c (periodic)."""
    B = R.biharmonic(c.ndim)
    return -p.M * p.kappa * capi.apply(B, c, capi.PERIODIC, 0, p.h)


def stage_operator(dim: int, gamma: float, h: float) -> R.RStencil:
    """I + gamma L o L with L o L scaled by h^-4, as an exact stencil of
    grid-unit weights (gamma / h^4 taken exactly as a double)."""
    B = R.biharmonic(dim)
    s = Fraction(gamma / h ** 4)
    return R.add(R.identity(dim), R.RStencil(dim, 0, {k: s * v for k, v in B.weights.items()}))


def imex_step(c: np.ndarray, dt: float, order: int, p: Params, tol: float = 1e-12):
    """One step of the IMEX RK pair; returns (c^{n+1}, CG iterations)."""
    T = tableau(order)
    s = len(T.b)
    N, K, its = [], [], 0
    for i in range(s):
        known = c.copy()
        for j in range(i):
            if T.Ahat[i][j] != 0.0:
                known += dt * T.Ahat[i][j] * N[j]
            if T.A[i][j] != 0.0:
                known += dt * T.A[i][j] * K[j]
        if T.A[i][i] == 0.0:
            Y = known
        else:
            op = stage_operator(c.ndim, dt * T.A[i][i] * p.M * p.kappa, p.h)
            x0 = c if i == 0 else Y
            Y, it, rel, rc = capi.cg(op, known, x0, capi.PERIODIC, tol)
            if rc != 0:
                raise RuntimeError(f"stage solve failed (status {rc}, residual {rel})")
            its += it
        N.append(explicit_part(Y, p))
        K.append(implicit_part(Y, p))
    out = c.copy()
    for j in range(s):
        if T.bhat[j] != 0.0:
            out += dt * T.bhat[j] * N[j]
        if T.b[j] != 0.0:
            out += dt * T.b[j] * K[j]
    return out, its


def integrate(c0: np.ndarray, dt: float, steps: int, order: int, p: Params, tol: float = 1e-12):
    c, its = c0.copy(), 0
    for _ in range(steps):
        c, it = imex_step(c, dt, order, p, tol)
        its += it
    return c, its


def free_energy(c: np.ndarray, p: Params):
    """(mass, F): mass = h^d sum c, and the free energy of Sec. 4.1,
    F = h^d sum [f_chem(c) + (kappa/2) |grad c|^2] with forward differences
    on the periodic grid."""
    hd = p.h ** c.ndim
    bulk = p.rho * (c - p.ca) ** 2 * (c - p.cb) ** 2
    grad = np.zeros_like(c)
    for ax in range(c.ndim):
        d = (np.roll(c, -1, axis=ax) - c) / p.h
        grad += d * d
    return hd * float(np.sum(c)), hd * float(np.sum(bulk + 0.5 * p.kappa * grad))
