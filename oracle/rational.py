"""Exact rational stencil algebra (oracle; test infrastructure only).

A stencil is a finite set of integer lattice offsets u_i in Z^d with weights
a_i proportional to h^-p (Sec. 2.1, the definition preceding
eq. (CompactNotation)). Here a stencil stores the weights as exact
``Fraction`` values of the coefficient of h^-p, so the weight applied to
f(x_0 + h u_i) is ``w[u_i] / h**p``.

Everything in this module is written from the definitions in the paper, with
no blocking or reordering:

* ``compose(b, a)``: eq. (C=B(A)) of Sec. 2.2. The outer stencil B is applied
  to the result of the inner stencil A, so C collects a_i b_j at offset
  u_i + v_j, and the h-powers (derivative orders) add.
* ``lincomb``: the Taylor sequences form a vector space (Sec. 2.1), so a
  weighted sum of stencils is a stencil.
* ``taylor``: t_alpha = sum_i a_i u_i^alpha / alpha!, eq. (CompactNotation),
  with multi-index powers for d > 1 (eq. (taylor2)).
* ``derivative_and_accuracy``: Definition (StencilRules), 1D.
* ``retarget_correction``: eq. (Retarget).
* ``symbol``: the Fourier symbol sum_i a_i exp(i theta . u_i), used for the
  von Neumann analysis of Sec. 2.2.3 / App. B and the spectra of Sec. 4.6.
* ``assemble_dense``: the matrix of a stencil on a small grid (periodic or
  with a zero Dirichlet ring), used for brute-force products (Sec. 1 notes
  that composition replaces sparse matrix-matrix products).
"""

from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from fractions import Fraction
from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np

Offset = Tuple[int, ...]


@dataclass
class RStencil:
    """Exact stencil: weights[u] is the coefficient of h^-p at offset u."""

    dim: int
    p: int
    weights: Dict[Offset, Fraction] = field(default_factory=dict)

    def __post_init__(self):
        clean = {}
        for off, w in self.weights.items():
            off = tuple(int(o) for o in off)
            if len(off) != self.dim:
                raise ValueError("offset dimension mismatch")
            w = Fraction(w)
            if w != 0:
                clean[off] = clean.get(off, Fraction(0)) + w
        self.weights = {k: v for k, v in clean.items() if v != 0}

    # -- views --------------------------------------------------------------
    def offsets(self) -> List[Offset]:
        return sorted(self.weights)

    def npts(self) -> int:
        return len(self.weights)

    def radius(self) -> int:
        """Largest |component| of any offset (Chebyshev radius)."""
        return max((max(abs(c) for c in off) for off in self.weights), default=0)

    def integer_form(self) -> Tuple[Dict[Offset, int], int]:
        """Weights as integers over one common positive denominator."""
        den = 1
        for w in self.weights.values():
            den = den * w.denominator // math.gcd(den, w.denominator)
        nums = {off: int(w * den) for off, w in self.weights.items()}
        return nums, den

    def float_weights(self, h: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
        """(offsets int array [n, dim], float64 weights scaled by h^-p)."""
        offs = self.offsets()
        o = np.array(offs, dtype=np.int64).reshape(len(offs), self.dim)
        w = np.array([float(self.weights[k]) for k in offs], dtype=np.float64)
        return o, w / (h ** self.p)

    def __eq__(self, other):
        return (isinstance(other, RStencil) and self.dim == other.dim
                and self.p == other.p and self.weights == other.weights)


# -- constructors ------------------------------------------------------------

def stencil1d(offsets: Sequence[int], weights: Sequence, p: int) -> RStencil:
    return RStencil(1, p, {(int(o),): Fraction(w) for o, w in zip(offsets, weights)})


def embed(s: RStencil, axis: int, dim: int) -> RStencil:
    """Place a 1D stencil along ``axis`` of a d-dimensional lattice."""
    assert s.dim == 1
    out = {}
    for (o,), w in s.weights.items():
        off = [0] * dim
        off[axis] = o
        out[tuple(off)] = w
    return RStencil(dim, s.p, out)


def identity(dim: int) -> RStencil:
    return RStencil(dim, 0, {(0,) * dim: Fraction(1)})


# -- the algebra ---------------------------------------------------------------

def compose(b: RStencil, a: RStencil) -> RStencil:
    """C = B(A), eq. (C=B(A)): C[u_i + v_j] = sum a_i b_j; p_c = p_a + p_b."""
    if a.dim != b.dim:
        raise ValueError("dimension mismatch")
    out: Dict[Offset, Fraction] = {}
    for ui, ai in a.weights.items():
        for vj, bj in b.weights.items():
            key = tuple(x + y for x, y in zip(ui, vj))
            out[key] = out.get(key, Fraction(0)) + ai * bj
    return RStencil(a.dim, a.p + b.p, out)


def lincomb(terms: Iterable[Tuple[Fraction, int, RStencil]]) -> RStencil:
    """sum_k c_k h^{q_k} S_k for stencils S_k; all p_k - q_k must agree.

    The h-power of each coefficient is carried explicitly so that a sum of
    operators with different derivative orders (for example I + c L o L)
    remains an exact rational object.
    """
    terms = list(terms)
    if not terms:
        raise ValueError("empty combination")
    dim = terms[0][2].dim
    p_out = terms[0][2].p - terms[0][1]
    out: Dict[Offset, Fraction] = {}
    for c, q, s in terms:
        if s.dim != dim or s.p - q != p_out:
            raise ValueError("incompatible terms")
        for off, w in s.weights.items():
            out[off] = out.get(off, Fraction(0)) + Fraction(c) * w
    return RStencil(dim, p_out, out)


def add(a: RStencil, b: RStencil) -> RStencil:
    return lincomb([(1, 0, a), (1, 0, b)])


# -- Taylor series (Sec. 2.1) -------------------------------------------------

def taylor(s: RStencil, max_order: int) -> Dict[Tuple[int, ...], Fraction]:
    """Raw t_alpha = sum_i w_i u_i^alpha / alpha! for |alpha| <= max_order.

    This is eq. (CompactNotation) before the shift by the derivative order:
    t_alpha multiplies h^{|alpha| - p} f^{(alpha)}(x_0).
    """
    out = {}
    for total in range(max_order + 1):
        for alpha in _multi_indices(s.dim, total):
            acc = Fraction(0)
            fact = 1
            for a in alpha:
                fact *= math.factorial(a)
            for off, w in s.weights.items():
                term = Fraction(1)
                for u, a in zip(off, alpha):
                    term *= Fraction(u) ** a
                acc += w * term
            out[alpha] = acc / fact
    return out


def taylor1d(s: RStencil, max_order: int) -> List[Fraction]:
    """1D raw Taylor list [t_0 .. t_max] (coefficient of h^{k-p} f^(k))."""
    assert s.dim == 1
    t = taylor(s, max_order)
    return [t[(k,)] for k in range(max_order + 1)]


def normalized_series1d(s: RStencil, length: int) -> Tuple[List[Fraction], int]:
    """(T, beta_bar) as printed in the paper: drop the leading zeros.

    The first non-zero raw coefficient sits at index beta_bar (the derivative
    order approximated); T lists the coefficients from there on, T[k]
    multiplying h^k f^(beta_bar + k).
    """
    raw = taylor1d(s, length + 16)
    beta = next(k for k, v in enumerate(raw) if v != 0)
    return raw[beta:beta + length], beta


def derivative_and_accuracy(s: RStencil, search: int = 24) -> Tuple[int, int, Fraction]:
    """Definition (StencilRules), 1D: (derivative order, accuracy q, t_q).

    The stencil approximates the beta-th derivative where beta is the first
    non-zero raw coefficient (which must equal 1 after the h^-p scaling, i.e.
    beta == p); q is the distance to the next non-zero coefficient.
    """
    raw = taylor1d(s, search)
    beta = next(k for k, v in enumerate(raw) if v != 0)
    if beta != s.p or raw[beta] != 1:
        raise ValueError("not a consistent derivative stencil")
    for q in range(1, search - beta + 1):
        if raw[beta + q] != 0:
            return beta, q, raw[beta + q]
    raise ValueError("accuracy beyond search window")


def retarget_correction(T: Sequence[Fraction], shift: int, length: int) -> List[Fraction]:
    """Correction series C_{y0->x0} of eq. (Retarget), 1D, y0 - x0 = shift*h.

    A series sum_a t_a h^a f^(a+beta)(y_0) read at x_0 gains, for every
    delta >= 1, the terms t_a h^a (shift h)^delta / delta! f^(a+beta+delta):
    coefficient index a + delta.
    """
    out = [Fraction(0)] * length
    for a, ta in enumerate(T):
        for d in range(1, length):
            if a + d < length:
                out[a + d] += Fraction(ta) * Fraction(shift) ** d / math.factorial(d)
    return out


def cauchy_product(TA: Sequence[Fraction], TB: Sequence[Fraction], length: int) -> List[Fraction]:
    """Product of two truncation series, eq. (AccuracyComposition)."""
    out = [Fraction(0)] * length
    for i, a in enumerate(TA):
        for j, b in enumerate(TB):
            if i + j < length:
                out[i + j] += Fraction(a) * Fraction(b)
    return out


# -- Fourier symbol and matrices ------------------------------------------------

def symbol(s: RStencil, theta: np.ndarray, h: float = 1.0) -> np.ndarray:
    """sigma(theta) = h^-p sum_i w_i exp(i theta . u_i); theta shape [..., dim]."""
    theta = np.asarray(theta, dtype=np.float64)
    out = np.zeros(theta.shape[:-1], dtype=np.complex128)
    for off, w in s.weights.items():
        phase = np.zeros(theta.shape[:-1])
        for k, u in enumerate(off):
            phase = phase + theta[..., k] * u
        out = out + float(w) * np.exp(1j * phase)
    return out / (h ** s.p)


def assemble_dense(s: RStencil, n: Sequence[int], periodic: bool, h: float = 1.0) -> np.ndarray:
    """Dense matrix M with (M x)_i = sum_k w_k x_{i+o_k} on an n[0] x n[1] ... grid.

    Index order: the first axis is fastest (x), matching the row-major grids
    used everywhere (x unit stride). With ``periodic`` the neighbour index is
    taken modulo n; otherwise neighbours outside the grid read zero (a zero
    Dirichlet ring).
    """
    n = list(n)
    N = int(np.prod(n))
    M = np.zeros((N, N))
    offs, w = s.float_weights(h)
    strides = [int(np.prod(n[:k])) for k in range(len(n))]
    for idx in itertools.product(*[range(m) for m in n]):
        row = sum(i * st for i, st in zip(idx, strides))
        for o, wk in zip(offs, w):
            nb = [i + int(d) for i, d in zip(idx, o)]
            if periodic:
                nb = [v % m for v, m in zip(nb, n)]
            elif any(v < 0 or v >= m for v, m in zip(nb, n)):
                continue
            col = sum(v * st for v, st in zip(nb, strides))
            M[row, col] += wk
    return M


def nnz_of_assembled(s: RStencil, n: Sequence[int], periodic: bool = True) -> int:
    """Number of structurally non-zero entries of the assembled matrix."""
    n = list(n)
    strides = [int(np.prod(n[:k])) for k in range(len(n))]
    total = 0
    for idx in itertools.product(*[range(m) for m in n]):
        cols = set()
        for off in s.weights:
            nb = [i + d for i, d in zip(idx, off)]
            if periodic:
                nb = [v % m for v, m in zip(nb, n)]
            elif any(v < 0 or v >= m for v, m in zip(nb, n)):
                continue
            cols.add(sum(v * st for v, st in zip(nb, strides)))
        total += len(cols)
    return total


def _multi_indices(dim: int, total: int):
    if dim == 1:
        yield (total,)
        return
    for first in range(total, -1, -1):
        for rest in _multi_indices(dim - 1, total - first):
            yield (first,) + rest


# -- the named stencils used throughout ---------------------------------------

def central_first() -> RStencil:
    """(f_1 - f_-1)/(2h), eq. (f'stencil)."""
    return stencil1d([1, -1], [Fraction(1, 2), Fraction(-1, 2)], 1)


def central_first_4th() -> RStencil:
    """(8 f_1 - f_2 + f_-2 - 8 f_-1)/(12h), eq. (4orderf')."""
    return stencil1d([1, 2, -2, -1], [Fraction(8, 12), Fraction(-1, 12), Fraction(1, 12), Fraction(-8, 12)], 1)


def central_second() -> RStencil:
    """(f_1 - 2 f_0 + f_-1)/h^2, eq. (CenterSecondDerivative)."""
    return stencil1d([1, 0, -1], [1, -2, 1], 2)


def central_second_4th() -> RStencil:
    """(-f_-2 + 16 f_-1 - 30 f_0 + 16 f_1 - f_2)/(12 h^2), fourth-order."""
    return stencil1d([-2, -1, 0, 1, 2], [Fraction(-1, 12), Fraction(16, 12), Fraction(-30, 12),
                                         Fraction(16, 12), Fraction(-1, 12)], 2)


def forward_first() -> RStencil:
    """(f_1 - f_0)/h, first-order forward difference (Sec. 2.2.1)."""
    return stencil1d([1, 0], [1, -1], 1)


def forward_second() -> RStencil:
    """(f_2 - 2 f_1 + f_0)/h^2, first-order forward difference (Sec. 2.2.1)."""
    return stencil1d([2, 1, 0], [1, -2, 1], 2)


def laplacian(dim: int, fourth_order: bool = False) -> RStencil:
    """Sum over axes of the 1D second-derivative stencil (5/7-point, or the
    9/13-point cross for the fourth-order factor)."""
    one = central_second_4th() if fourth_order else central_second()
    out = embed(one, 0, dim)
    for ax in range(1, dim):
        out = add(out, embed(one, ax, dim))
    return out


def biharmonic(dim: int, fourth_order: bool = False) -> RStencil:
    """L o L, the Laplacian composed with itself (Sec. 3.3)."""
    L = laplacian(dim, fourth_order)
    return compose(L, L)


def ch_operator(dim: int, eps_over_h: Fraction, dt_over_h2: Fraction, S: Fraction) -> RStencil:
    """I + dt eps^2 L o L - dt S L, the linearly stabilised implicit operator.

    With eps = e h and dt = k h^2 the coefficients are dt eps^2 = k e^2 h^4 and
    dt S = k S h^2, so the operator is dimensionless (p = 0).
    """
    L = laplacian(dim)
    LL = compose(L, L)
    e, k = Fraction(eps_over_h), Fraction(dt_over_h2)
    return lincomb([(1, 0, identity(dim)), (k * e * e, 4, LL), (-k * Fraction(S), 2, L)])
