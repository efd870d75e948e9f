"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and samples the manufactured fields
that define the test problems; it contains none of the stencil-composition
arithmetic. Every generator is seeded (numpy PCG64) and returns FP64 numpy
arrays with x as the last axis (x unit stride).

Grid conventions
* Boundary-value problems: nodes x_i = (i + 1) h for the unknowns
  i = 0 .. n-1, so the boundary nodes sit at i = -1 (x = 0) and i = n
  (x = 1). In 2D a grid is named by its node count N including the boundary
  (h = 1/(N-1), n = N-2); in 3D by its unknown count n (h = 1/(n+1)).
  The prescribed ring of width ``halo`` around the unknowns holds the exact
  solution sampled at those nodes (the boundary nodes and the ghost nodes
  outside them).
* Periodic problems: N points per side at x_i = i/N, h = 1/N.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Tuple

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_field(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """U[lo, hi) FP64 field."""
    return rng(seed).uniform(lo, hi, size=tuple(shape)).astype(np.float64)


def integer_field(shape, seed: int, lo: int = -512, hi: int = 512) -> np.ndarray:
    """Integers in [lo, hi] stored as FP64 (exact in FP32 and FP64)."""
    return rng(seed).integers(lo, hi + 1, size=tuple(shape)).astype(np.float64)


def zero_mean_uniform(shape, seed: int, amp: float = 0.05) -> np.ndarray:
    """U[-amp, amp] with the FP64 sample mean subtracted (Cahn-Hilliard start)."""
    u = rng(seed).uniform(-amp, amp, size=tuple(shape)).astype(np.float64)
    return u - u.mean()


@dataclass
class BVP:
    """A manufactured biharmonic boundary-value problem on the unit square/cube."""

    dim: int
    n: int          # unknowns per side
    h: float
    halo: int
    f: np.ndarray   # forcing at the unknowns, shape (n,)*dim
    g: np.ndarray   # ring data, shape (n+2*halo,)*dim, zero at the unknowns
    u: np.ndarray   # exact solution at the unknowns


def _sinprod(dim: int, n: int, h: float, halo: int) -> np.ndarray:
    idx = np.arange(-halo, n + halo, dtype=np.float64)
    s = np.sin(math.pi * (idx + 1.0) * h)
    out = s
    for _ in range(dim - 1):
        out = np.multiply.outer(out, s)
    return out


def biharmonic_bvp(dim: int, size: int, halo: int = 2) -> BVP:
    """u = prod_k sin(pi x_k), f = Delta^2 u = (dim pi^2)^2 u.

    2D: ``size`` is the node count N (h = 1/(N-1)); 3D: the unknown count n
    (h = 1/(n+1)).
    """
    if dim == 2:
        N = size
        n, h = N - 2, 1.0 / (N - 1)
    elif dim == 3:
        n = size
        h = 1.0 / (n + 1)
    else:
        raise ValueError("dim must be 2 or 3")
    full = _sinprod(dim, n, h, halo)
    inner = tuple(slice(halo, halo + n) for _ in range(dim))
    u = full[inner].copy()
    g = full.copy()
    g[inner] = 0.0
    f = (dim * math.pi ** 2) ** 2 * u
    return BVP(dim, n, h, halo, np.ascontiguousarray(f), np.ascontiguousarray(g), np.ascontiguousarray(u))


def periodic_sin_mode(dim: int, N: int, k: int = 1) -> Tuple[np.ndarray, float]:
    """prod_d sin(2 pi k x_d) on an N^dim periodic grid; returns (field, h)."""
    h = 1.0 / N
    s = np.sin(2.0 * math.pi * k * np.arange(N) * h)
    out = s
    for _ in range(dim - 1):
        out = np.multiply.outer(out, s)
    return np.ascontiguousarray(out), h


def periodic_cos_mode(shape, kvec) -> np.ndarray:
    """cos(2 pi sum_d k_d i_d / N_d) on a periodic grid (x last)."""
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    phase = np.zeros(shape)
    # axis order: numpy axis a corresponds to lattice axis dim-1-a
    dim = len(shape)
    for a in range(dim):
        phase = phase + 2.0 * math.pi * kvec[dim - 1 - a] * grids[a] / shape[a]
    return np.cos(phase)


def spinodal_initial(dim: int, n: int, h: float = 1.0, c0: float = 0.5, amp: float = 0.01) -> np.ndarray:
    """Initial concentration of the spinodal-decomposition benchmark (Sec. 4.1):
    c0 plus amp times a sum of three cosine products, sampled at x_i = i h,
    i = 0 .. n-1, on every axis (the 200^2 and 64^3 unit domains are n = 200 and
    n = 64 with h = 1). Arrays are (y, x) or (z, y, x)."""
    c = np.arange(n, dtype=np.float64) * h
    if dim == 2:
        Y, X = np.meshgrid(c, c, indexing="ij")
        s = (np.cos(0.105 * X) * np.cos(0.11 * Y)
             + (np.cos(0.13 * X) * np.cos(0.087 * Y)) ** 2
             + np.cos(0.025 * X - 0.15 * Y) * np.cos(0.07 * X - 0.02 * Y))
    elif dim == 3:
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        s = (np.cos(0.105 * X) * np.cos(0.11 * Y) * np.cos(0.11 * Z)
             + (np.cos(0.13 * X) * np.cos(0.087 * Y) * np.cos(0.1 * Z)) ** 2
             + np.cos(0.025 * X - 0.15 * Y - 0.1 * Z) * np.cos(0.07 * X - 0.02 * Y + 0.01 * Z))
    else:
        raise ValueError("dim must be 2 or 3")
    return c0 + amp * s
