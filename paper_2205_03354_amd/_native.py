"""ctypes binding of ``libscomp.so`` (the gfx950 stencil-composition library).

Argument marshalling only: every computation happens in the library (exact
stencil algebra on the host, everything else in HIP kernels on the GPU).
PyTorch supplies device memory and the current HIP stream. If the library
is not built, importing this module raises; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscomp.so")

(SC_OK, SC_EINVAL, SC_EOVERFLOW, SC_EDEVICE, SC_ENOMEM, SC_ENOTCONV, SC_EBREAKDOWN, SC_EUNSUPPORTED,
 SC_ECANCELLED) = range(9)
SC_REQ_BVP, SC_REQ_CH_STEP = 0, 1
SC_PC_NONE, SC_PC_FASTPOISSON = 0, 1
SC_F64, SC_F32 = 0, 1
SC_BC_PERIODIC, SC_BC_HALO = 0, 1
SC_PREC_F64, SC_PREC_F32_IR, SC_PREC_F32_RU = 0, 1, 2
SC_CSR_PERIODIC, SC_CSR_ZERO_RING = 0, 1
SC_CSR_ROWSPLIT, SC_CSR_ADAPTIVE = 0, 1

EXPORTED = (
    "sc_stencil_create", "sc_compose_stencil", "sc_stencil_lincomb", "sc_stencil_get",
    "sc_stencil_radius", "sc_stencil_free", "sc_apply_composed", "sc_apply_varcoef", "sc_solve_opts_default",
    "sc_solve_biharmonic", "sc_ch_step", "sc_grid_diagnostics", "sc_status_str",
    "sc_last_error", "sc_version", "sc_server_create", "sc_server_submit", "sc_server_poll",
    "sc_server_cancel", "sc_server_load", "sc_server_destroy", "sc_spinodal_steps", "sc_spinodal_energy",
    "sc_solve_biharmonic_batch",
    "sc_csr_assemble", "sc_csr_info",
    "sc_csr_spmv", "sc_csr_export", "sc_csr_free",
)


class ScError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class SCGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("halo", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
                ("pitch", ctypes.c_int64 * 2), ("dtype", ctypes.c_int32), ("data", ctypes.c_void_p)]


class SCSolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("check_every", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("onchip", ctypes.c_int32)]


class SCSolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("outer", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("seconds", ctypes.c_double)]


class SCSpinodalParams(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("dt", ctypes.c_double), ("mobility", ctypes.c_double),
                ("kappa", ctypes.c_double), ("rho", ctypes.c_double), ("c_alpha", ctypes.c_double),
                ("c_beta", ctypes.c_double), ("order", ctypes.c_int32)]


class SCSpinodalStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("solves", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("max_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


class SCChParams(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("eps", ctypes.c_double), ("dt", ctypes.c_double), ("S", ctypes.c_double)]


class SCServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_slots", ctypes.c_int32), ("solve", SCSolveOpts),
                ("fake_device", ctypes.c_int32)]


class SCRequest(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dim", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double),
                ("op", ctypes.c_void_p), ("f", ctypes.c_void_p), ("g", ctypes.c_void_p), ("u0", ctypes.c_void_p),
                ("u_out", ctypes.c_void_p), ("ch", SCChParams), ("precision", ctypes.c_int32)]


class SCResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("iterations", ctypes.c_int64),
                ("outer", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("device_bytes", ctypes.c_uint64)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_2205_03354_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    L.sc_stencil_create.argtypes = [I32, I32, P, P, I64, I32, PP]
    L.sc_compose_stencil.argtypes = [P, P, PP]
    L.sc_stencil_lincomb.argtypes = [I32, P, P, P, P, PP]
    L.sc_stencil_get.argtypes = [P, P, P, I32, P, P, P, P]
    L.sc_stencil_radius.argtypes = [P]
    L.sc_stencil_radius.restype = I32
    L.sc_stencil_free.argtypes = [P]
    L.sc_stencil_free.restype = None
    L.sc_apply_composed.argtypes = [P, D, ctypes.POINTER(SCGrid), ctypes.POINTER(SCGrid), ctypes.c_int, P]
    L.sc_apply_varcoef.argtypes = [I32, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), D,
                                   ctypes.POINTER(SCGrid), ctypes.POINTER(SCGrid), ctypes.POINTER(SCGrid),
                                   ctypes.c_int, P]
    L.sc_solve_opts_default.argtypes = [ctypes.POINTER(SCSolveOpts)]
    L.sc_solve_opts_default.restype = None
    L.sc_solve_biharmonic.argtypes = [P, D, ctypes.POINTER(SCGrid), ctypes.POINTER(SCGrid),
                                      ctypes.POINTER(SCSolveOpts), ctypes.POINTER(SCGrid),
                                      ctypes.POINTER(SCSolveStats), P]
    L.sc_ch_step.argtypes = [P, ctypes.POINTER(SCChParams), ctypes.POINTER(SCSolveOpts),
                             ctypes.POINTER(SCGrid), ctypes.POINTER(SCSolveStats), P]
    L.sc_grid_diagnostics.argtypes = [ctypes.POINTER(SCGrid), D, D, P, P, P]
    L.sc_server_create.argtypes = [ctypes.POINTER(SCServerOpts), PP]
    L.sc_server_submit.argtypes = [P, ctypes.POINTER(SCRequest), ctypes.POINTER(ctypes.c_uint64)]
    L.sc_server_poll.argtypes = [P, ctypes.POINTER(SCResult), I32, ctypes.POINTER(ctypes.c_int32), I32]
    L.sc_server_cancel.argtypes = [P, ctypes.c_uint64]
    L.sc_server_load.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64)]
    L.sc_server_destroy.argtypes = [P]
    L.sc_server_destroy.restype = None
    for name in ("sc_server_create", "sc_server_submit", "sc_server_poll", "sc_server_cancel", "sc_server_load"):
        getattr(L, name).restype = ctypes.c_int
    L.sc_solve_biharmonic_batch.argtypes = [P, P, I32, ctypes.POINTER(SCGrid), ctypes.POINTER(SCGrid),
                                            ctypes.POINTER(SCSolveOpts), ctypes.POINTER(SCGrid),
                                            ctypes.POINTER(SCSolveStats), P]
    L.sc_solve_biharmonic_batch.restype = ctypes.c_int
    L.sc_spinodal_steps.argtypes = [P, ctypes.POINTER(SCSpinodalParams), I32, ctypes.POINTER(SCSolveOpts),
                                    ctypes.POINTER(SCGrid), ctypes.POINTER(SCSpinodalStats), P]
    L.sc_spinodal_energy.argtypes = [ctypes.POINTER(SCGrid), ctypes.POINTER(SCSpinodalParams), P, P, P]
    L.sc_spinodal_steps.restype = ctypes.c_int
    L.sc_spinodal_energy.restype = ctypes.c_int
    L.sc_csr_assemble.argtypes = [P, D, I32, P, I32, I32, I32, P, PP]
    L.sc_csr_info.argtypes = [P, P, P, P]
    L.sc_csr_spmv.argtypes = [P, ctypes.POINTER(SCGrid), ctypes.POINTER(SCGrid), P]
    L.sc_csr_export.argtypes = [P, P, P, P]
    L.sc_csr_free.argtypes = [P]
    L.sc_csr_free.restype = None
    for name in ("sc_csr_assemble", "sc_csr_info", "sc_csr_spmv", "sc_csr_export"):
        getattr(L, name).restype = ctypes.c_int
    L.sc_status_str.argtypes = [ctypes.c_int]
    L.sc_status_str.restype = ctypes.c_char_p
    L.sc_last_error.argtypes = []
    L.sc_last_error.restype = ctypes.c_char_p
    L.sc_version.argtypes = []
    L.sc_version.restype = ctypes.c_char_p
    for name in ("sc_stencil_create", "sc_compose_stencil", "sc_stencil_lincomb", "sc_stencil_get",
                 "sc_apply_composed", "sc_apply_varcoef", "sc_solve_biharmonic", "sc_ch_step",
                 "sc_grid_diagnostics"):
        getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


def _check(status: int):
    if status != SC_OK:
        msg = lib.sc_last_error().decode()
        raise ScError(status, f"{lib.sc_status_str(status).decode()}: {msg}")


# ---------------------------------------------------------------- stencils

class Stencil:
    """Library-owned exact stencil: weight t is num[t] / (den h^hpow)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.sc_stencil_free(h)
            self._h = None

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    @classmethod
    def create(cls, dim: int, offsets: Sequence[Sequence[int]], num: Sequence[int], den: int = 1,
               hpow: int = 0) -> "Stencil":
        n = len(num)
        offs = (ctypes.c_int32 * (3 * n))()
        for t, o in enumerate(offsets):
            o = list(o) + [0] * (3 - len(o))
            offs[3 * t:3 * t + 3] = o[:3]
        nums = (ctypes.c_int64 * n)(*[int(v) for v in num])
        out = ctypes.c_void_p()
        _check(lib.sc_stencil_create(dim, n, offs, nums, int(den), int(hpow), ctypes.byref(out)))
        return cls(out.value)

    def get(self) -> Tuple[int, list, list, int, int]:
        """(dim, offsets [(x,y,z)], num, den, hpow) in canonical order."""
        dim, npts, den, hp = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib.sc_stencil_get(self._h, ctypes.byref(dim), ctypes.byref(npts), 0, None, None,
                                  ctypes.byref(den), ctypes.byref(hp)))
        n = npts.value
        offs = (ctypes.c_int32 * (3 * n))()
        nums = (ctypes.c_int64 * n)()
        _check(lib.sc_stencil_get(self._h, None, None, n, offs, nums, None, None))
        return dim.value, [tuple(offs[3 * t:3 * t + 3]) for t in range(n)], list(nums), den.value, hp.value

    @property
    def radius(self) -> int:
        return int(lib.sc_stencil_radius(self._h))


def compose_stencil(a: Stencil, b: Stencil) -> Stencil:
    """C = B(A): `a` is the inner stencil, `b` the outer one."""
    out = ctypes.c_void_p()
    _check(lib.sc_compose_stencil(a.handle, b.handle, ctypes.byref(out)))
    return Stencil(out.value)


def stencil_lincomb(terms: Sequence[Tuple[int, int, int, Stencil]]) -> Stencil:
    """sum (cnum/cden) h^chpow S over terms (cnum, cden, chpow, S)."""
    n = len(terms)
    hs = (ctypes.c_void_p * n)(*[t[3].handle.value for t in terms])
    cn = (ctypes.c_int64 * n)(*[int(t[0]) for t in terms])
    cd = (ctypes.c_int64 * n)(*[int(t[1]) for t in terms])
    cp = (ctypes.c_int32 * n)(*[int(t[2]) for t in terms])
    out = ctypes.c_void_p()
    _check(lib.sc_stencil_lincomb(n, hs, cn, cd, cp, ctypes.byref(out)))
    return Stencil(out.value)


# ------------------------------------------------------------------- grids

def grid_of(t, halo: int = 0) -> SCGrid:
    """Describe a CUDA tensor holding a grid *including* its ring of width
    `halo` (x is the last axis, unit stride)."""
    import torch

    if not t.is_cuda:
        raise ValueError("grid tensors must live on the GPU")
    if t.dtype == torch.float64:
        dt = SC_F64
    elif t.dtype == torch.float32:
        dt = SC_F32
    else:
        raise ValueError("grid dtype must be float64 or float32")
    if t.dim() not in (2, 3) or t.stride(-1) != 1:
        raise ValueError("grid tensors must be 2D/3D with unit stride along x")
    g = SCGrid()
    g.dim = t.dim()
    g.halo = halo
    shape = list(t.shape)[::-1]  # x first
    for a in range(3):
        g.n[a] = (shape[a] - 2 * halo) if a < t.dim() else 1
    g.pitch[0] = t.stride(-2)
    g.pitch[1] = t.stride(-3) if t.dim() == 3 else 0
    g.dtype = dt
    g.data = t.data_ptr()
    return g


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def apply_composed(st: Stencil, x, y, bc: int = SC_BC_PERIODIC, h: float = 1.0, halo: int = 0,
                   out_halo: Optional[int] = None, stream=None):
    """y = S x on the interior (asynchronous on the current stream)."""
    gi = grid_of(x, halo)
    go = grid_of(y, halo if out_halo is None else out_halo)
    _check(lib.sc_apply_composed(st.handle, float(h), ctypes.byref(gi), ctypes.byref(go), int(bc),
                                 _stream(stream)))
    return y


def apply_varcoef(terms, mob, x, y, bc: int = SC_BC_PERIODIC, h: float = 1.0, halo: int = 0,
                  mob_halo: int = 0, out_halo: int = 0, stream=None):
    """y = sum_t outer_t(mob * inner_t(x)) for terms [(inner_t, outer_t)]
    (see sc_apply_varcoef); returns after the work completes."""
    n = len(terms)
    inner = (ctypes.c_void_p * n)(*[t[0].handle.value for t in terms])
    outer = (ctypes.c_void_p * n)(*[t[1].handle.value for t in terms])
    gm, gi, go = grid_of(mob, mob_halo), grid_of(x, halo), grid_of(y, out_halo)
    _check(lib.sc_apply_varcoef(n, inner, outer, float(h), ctypes.byref(gm), ctypes.byref(gi), ctypes.byref(go),
                                int(bc), _stream(stream)))
    return y


class ApplyPlan:
    """A pre-marshalled y = S x launch for repeated use on fixed buffers:
    the grid descriptors and stream are built once, each call only crosses
    the C ABI."""

    def __init__(self, st: Stencil, x, y, bc: int = SC_BC_PERIODIC, h: float = 1.0, halo: int = 0,
                 out_halo: Optional[int] = None, stream=None):
        self._st = st
        self._gi = grid_of(x, halo)
        self._go = grid_of(y, halo if out_halo is None else out_halo)
        self._keep = (x, y)
        self._h = float(h)
        self._bc = int(bc)
        self._stream = _stream(stream)
        self._fn = lib.sc_apply_composed
        self._args = (st.handle, ctypes.c_double(self._h), ctypes.byref(self._gi), ctypes.byref(self._go),
                      self._bc, self._stream)

    def __call__(self):
        rc = self._fn(*self._args)
        if rc != SC_OK:
            _check(rc)


class Csr:
    """The stencil assembled as a CSR matrix on the device (sc_csr_assemble);
    ``spmv(x, y)`` is y = A x by rocSPARSE on contiguous grids without a ring."""

    def __init__(self, st: Stencil, shape, bc: int = SC_CSR_PERIODIC, h: float = 1.0, dtype=None,
                 alg: int = SC_CSR_ROWSPLIT, stream=None):
        import torch

        dtype = torch.float64 if dtype is None else dtype
        self.dtype = dtype
        self.shape = tuple(int(s) for s in shape)
        dim = len(self.shape)
        n = (ctypes.c_int64 * 3)(*(list(self.shape[::-1]) + [1] * (3 - dim)))
        self._h = ctypes.c_void_p()
        dt = SC_F64 if dtype == torch.float64 else SC_F32
        _check(lib.sc_csr_assemble(st.handle, float(h), dim, n, int(bc), dt, int(alg), _stream(stream),
                                   ctypes.byref(self._h)))
        rows, nnz, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint64()
        _check(lib.sc_csr_info(self._h, ctypes.byref(rows), ctypes.byref(nnz), ctypes.byref(nb)))
        self.rows, self.nnz, self.bytes = rows.value, nnz.value, nb.value

    def spmv(self, x, y, stream=None):
        gx, gy = grid_of(x), grid_of(y)
        _check(lib.sc_csr_spmv(self._h, ctypes.byref(gx), ctypes.byref(gy), _stream(stream)))
        return y

    def export(self):
        """(row_ptr int64, col int32, val) as numpy arrays."""
        import numpy as np

        rp = np.empty(self.rows + 1, dtype=np.int64)
        col = np.empty(self.nnz, dtype=np.int32)
        import torch

        val = np.empty(self.nnz, dtype=np.float64 if self.dtype == torch.float64 else np.float32)
        _check(lib.sc_csr_export(self._h, rp.ctypes.data, col.ctypes.data, val.ctypes.data))
        return rp, col, val

    def close(self):
        if self._h:
            lib.sc_csr_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class SolveStats:
    iterations: int
    outer: int
    rel_residual: float
    bnorm: float
    seconds: float
    status: int


def _opts(tol, max_iter, precision, inner_tol, check_every, use_graph=True, precond=SC_PC_NONE,
          onchip=True) -> SCSolveOpts:
    o = SCSolveOpts()
    lib.sc_solve_opts_default(ctypes.byref(o))
    o.tol = tol
    o.max_iter = int(max_iter)
    o.precision = int(precision)
    o.inner_tol = inner_tol
    o.check_every = int(check_every)
    o.use_graph = 1 if use_graph else 0
    o.precond = int(precond)
    o.onchip = 1 if onchip else 0
    return o


def _stats(s: SCSolveStats, status: int) -> SolveStats:
    return SolveStats(int(s.iterations), int(s.outer), float(s.rel_residual), float(s.bnorm), float(s.seconds), status)


def solve_biharmonic(op: Stencil, h: float, f, u, g=None, g_halo: int = 0, tol: float = 1e-10,
                     max_iter: int = 10**7, precision: int = SC_PREC_F64, inner_tol: float = 0.0,
                     check_every: int = 64, use_graph: bool = True, precond: int = SC_PC_NONE,
                     onchip: bool = True, raise_on_error: bool = True, stream=None) -> SolveStats:
    """A u = f at the unknowns with the ring prescribed by g (see scomp.h)."""
    gf, gu = grid_of(f, 0), grid_of(u, 0)
    gg = ctypes.byref(grid_of(g, g_halo)) if g is not None else None
    o = _opts(tol, max_iter, precision, inner_tol, check_every, use_graph, precond, onchip)
    st = SCSolveStats()
    status = lib.sc_solve_biharmonic(op.handle, float(h), ctypes.byref(gf), gg, ctypes.byref(o), ctypes.byref(gu),
                                     ctypes.byref(st), _stream(stream))
    if raise_on_error:
        _check(status)
    return _stats(st, status)


def solve_biharmonic_batch(op: Stencil, problems, tol: float = 1e-10, max_iter: int = 10**6,
                           raise_on_error: bool = True, stream=None):
    """Solve a batch of small 2D BVPs, one workgroup each (sc_solve_biharmonic_batch).
    problems: sequence of (h, f, u, g, g_halo) with g None for a zero ring.
    Returns (status, [SolveStats per problem])."""
    n = len(problems)
    hs = (ctypes.c_double * max(n, 1))(*[float(p[0]) for p in problems])
    fs = (SCGrid * max(n, 1))(*[grid_of(p[1], 0) for p in problems])
    us = (SCGrid * max(n, 1))(*[grid_of(p[2], 0) for p in problems])
    gs = (SCGrid * max(n, 1))()
    for i, p in enumerate(problems):
        if p[3] is not None:
            gs[i] = grid_of(p[3], p[4])
    o = _opts(tol, max_iter, SC_PREC_F64, 0.0, 64, True, SC_PC_NONE)
    st = (SCSolveStats * max(n, 1))()
    status = lib.sc_solve_biharmonic_batch(op.handle, hs, n, fs, gs, ctypes.byref(o), us, st, _stream(stream))
    if raise_on_error:
        _check(status)
    return status, [_stats(st[i], status) for i in range(n)]


def ch_step(lap: Stencil, u, h: float, eps: float, dt: float, S: float, tol: float = 1e-10,
            max_iter: int = 10**6, precision: int = SC_PREC_F64, inner_tol: float = 0.0,
            check_every: int = 32, use_graph: bool = True, raise_on_error: bool = True,
            stream=None) -> SolveStats:
    """One linearly stabilised semi-implicit Cahn-Hilliard step, in place on u."""
    gu = grid_of(u, 0)
    prm = SCChParams(h, eps, dt, S)
    o = _opts(tol, max_iter, precision, inner_tol, check_every, use_graph)
    st = SCSolveStats()
    status = lib.sc_ch_step(lap.handle, ctypes.byref(prm), ctypes.byref(o), ctypes.byref(gu), ctypes.byref(st),
                            _stream(stream))
    if raise_on_error:
        _check(status)
    return _stats(st, status)


@dataclass
class SpinodalStats:
    steps: int
    solves: int
    iterations: int
    max_rel_residual: float
    seconds: float
    status: int


def spinodal_params(h: float = 1.0, dt: float = 0.05, mobility: float = 5.0, kappa: float = 2.0,
                    rho: float = 5.0, c_alpha: float = 0.3, c_beta: float = 0.7, order: int = 1) -> SCSpinodalParams:
    """Parameters of the spinodal-decomposition benchmark (defaults: the
    benchmark's M, kappa, rho and well minima on h = 1)."""
    return SCSpinodalParams(h, dt, mobility, kappa, rho, c_alpha, c_beta, int(order))


def spinodal_steps(lap: Stencil, c, params: SCSpinodalParams, nsteps: int, tol: float = 1e-10,
                   max_iter: int = 10**6, precision: int = SC_PREC_F64, inner_tol: float = 0.0,
                   check_every: int = 16, use_graph: bool = True, raise_on_error: bool = True,
                   halo: int = 0, stream=None) -> SpinodalStats:
    """Advance c (FP64, periodic) by nsteps IMEX steps in place (sc_spinodal_steps)."""
    gc = grid_of(c, halo)
    o = _opts(tol, max_iter, precision, inner_tol, check_every, use_graph)
    st = SCSpinodalStats()
    status = lib.sc_spinodal_steps(lap.handle, ctypes.byref(params), int(nsteps), ctypes.byref(o), ctypes.byref(gc),
                                   ctypes.byref(st), _stream(stream))
    if raise_on_error:
        _check(status)
    return SpinodalStats(int(st.steps), int(st.solves), int(st.iterations), float(st.max_rel_residual),
                         float(st.seconds), status)


def spinodal_energy(c, params: SCSpinodalParams, halo: int = 0, stream=None) -> Tuple[float, float]:
    """(mass, free energy) of c (sc_spinodal_energy)."""
    gc = grid_of(c, halo)
    m, e = ctypes.c_double(), ctypes.c_double()
    _check(lib.sc_spinodal_energy(ctypes.byref(gc), ctypes.byref(params), ctypes.byref(m), ctypes.byref(e),
                                  _stream(stream)))
    return m.value, e.value


def grid_diagnostics(u, h: float, eps: float, stream=None) -> Tuple[float, float]:
    """(mass, free energy) of a periodic FP64 grid."""
    gu = grid_of(u, 0)
    m, e = ctypes.c_double(), ctypes.c_double()
    _check(lib.sc_grid_diagnostics(ctypes.byref(gu), float(h), float(eps), ctypes.byref(m), ctypes.byref(e),
                                   _stream(stream)))
    return m.value, e.value


class Server:
    """Continuous-batching request server (see sc_server_* in scomp.h).

    Host arrays are numpy FP64 with x as the last axis; each submit returns
    the request id, and the solution lands in the array returned by
    ``result_array(id)`` once its result has been polled."""

    def __init__(self, hbm_budget: int = 0, max_slots: int = 16, tol: float = 1e-10,
                 precision: int = SC_PREC_F64, inner_tol: float = 0.0, check_every: int = 64,
                 use_graph: bool = True, max_iter: int = 10**7, fake_device: bool = False,
                 precond: int = SC_PC_NONE, onchip: bool = True):
        o = SCServerOpts()
        o.hbm_budget = int(hbm_budget)
        o.max_slots = int(max_slots)
        o.solve = _opts(tol, max_iter, precision, inner_tol, check_every, use_graph, precond, onchip)
        o.fake_device = 1 if fake_device else 0
        h = ctypes.c_void_p()
        _check(lib.sc_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._out = {}
        self._keep = {}

    def _submit(self, req: SCRequest, out, keep) -> int:
        rid = ctypes.c_uint64()
        _check(lib.sc_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        self._out[rid.value] = out
        self._keep[rid.value] = keep
        return rid.value

    @staticmethod
    def _shape(a):
        n = list(a.shape)[::-1] + [1, 1]
        return a.ndim, n[:3]

    def submit_bvp(self, op: Stencil, h: float, f, g=None, u0=None, precision: int = -1) -> int:
        import numpy as np

        f = np.ascontiguousarray(f, dtype=np.float64)
        dim, n = self._shape(f)
        out = np.zeros_like(f)
        req = SCRequest()
        req.kind, req.dim = SC_REQ_BVP, dim
        for a in range(3):
            req.n[a] = n[a]
        req.h = float(h)
        req.op = op.handle.value
        req.f = f.ctypes.data
        gg = np.ascontiguousarray(g, dtype=np.float64) if g is not None else None
        uu = np.ascontiguousarray(u0, dtype=np.float64) if u0 is not None else None
        req.g = gg.ctypes.data if gg is not None else None
        req.u0 = uu.ctypes.data if uu is not None else None
        req.u_out = out.ctypes.data
        req.precision = int(precision)
        return self._submit(req, out, (op, f, gg, uu))

    def submit_ch(self, lap: Stencil, u0, h: float, eps: float, dt: float, S: float, precision: int = -1) -> int:
        import numpy as np

        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        dim, n = self._shape(u0)
        out = np.zeros_like(u0)
        req = SCRequest()
        req.kind, req.dim = SC_REQ_CH_STEP, dim
        for a in range(3):
            req.n[a] = n[a]
        req.h = float(h)
        req.op = lap.handle.value
        req.u0 = u0.ctypes.data
        req.u_out = out.ctypes.data
        req.ch = SCChParams(h, eps, dt, S)
        req.precision = int(precision)
        return self._submit(req, out, (lap, u0))

    def poll(self, max_results: int = 256, wait_ms: int = 0):
        buf = (SCResult * max_results)()
        n = ctypes.c_int32()
        _check(lib.sc_server_poll(self._h, buf, max_results, ctypes.byref(n), int(wait_ms)))
        res = []
        for i in range(n.value):
            r = buf[i]
            self._keep.pop(r.id, None)
            res.append({"id": r.id, "status": r.status, "iterations": r.iterations, "outer": r.outer,
                        "rel_residual": r.rel_residual, "t_submit": r.t_submit, "t_admit": r.t_admit,
                        "t_done": r.t_done, "device_bytes": r.device_bytes})
        return res

    def result_array(self, rid: int):
        return self._out.pop(rid)

    def cancel(self, rid: int):
        _check(lib.sc_server_cancel(self._h, rid))

    def load(self):
        q, a, f, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_uint64()
        _check(lib.sc_server_load(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(f), ctypes.byref(b)))
        return {"queued": q.value, "active": a.value, "finished": f.value, "device_bytes": b.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.sc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def version() -> str:
    return lib.sc_version().decode()
