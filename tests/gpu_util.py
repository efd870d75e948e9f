"""Helpers shared by the GPU parity tests (no method arithmetic here)."""

from __future__ import annotations

import numpy as np

from oracle import capi
from oracle import rational as R


def lib_stencil(native, st: R.RStencil):
    """Hand an exact oracle stencil to the library (integer numerators over
    one denominator; the library re-derives its own canonical form)."""
    nums, den = st.integer_form()
    offs = sorted(nums)
    return native.Stencil.create(st.dim, offs, [nums[o] for o in offs], den, st.p)


def abs_stencil(st: R.RStencil) -> R.RStencil:
    return R.RStencil(st.dim, st.p, {k: abs(v) for k, v in st.weights.items()})


def scaled_error(got: np.ndarray, ref: np.ndarray, st: R.RStencil, x: np.ndarray, mode: int,
                 halo: int = 0, h: float = 1.0) -> float:
    """max |got - ref| / max (|W| |x|): the error relative to the magnitude of
    the summed terms, which is what rounding can be measured against."""
    scale = capi.apply(abs_stencil(st), np.abs(x), mode, halo, h)
    den = float(np.max(scale))
    return float(np.max(np.abs(got - ref))) / (den if den > 0 else 1.0)


def padded(arr: np.ndarray, halo: int, fill_seed=None) -> np.ndarray:
    """Embed `arr` in a ring of width `halo` (ring filled with seeded values
    when fill_seed is given, else zeros)."""
    shape = tuple(s + 2 * halo for s in arr.shape)
    if fill_seed is None:
        out = np.zeros(shape)
    else:
        out = np.random.Generator(np.random.PCG64(fill_seed)).uniform(-1, 1, size=shape)
    inner = tuple(slice(halo, halo + s) for s in arr.shape)
    out[inner] = arr
    return out
