"""GPU parity of the Krylov solves (biharmonic BVP, Cahn-Hilliard step).

Bars (from the arithmetic): the GPU solution's true relative residual,
recomputed by the oracle's own FP64 apply, is <= the requested 1e-10; the
distance to the oracle's CG solution is bounded by kappa * tol (the systems
are SPD, the solution unique), checked as 1e-6 relative for the BVPs
(kappa <= 3e6 at these sizes) and 1e-9 for the well-conditioned
Cahn-Hilliard step (kappa ~ 105 / 234). Iteration counts are not compared.
"""

import math

import numpy as np
import pytest
import torch

import synthetic as S
from oracle import capi
from oracle import problems as OP
from oracle import rational as R
from tests.gpu_util import lib_stencil

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")

_PREC = {"f64": lambda m: m.SC_PREC_F64, "f32ir": lambda m: m.SC_PREC_F32_IR, "f32ru": lambda m: m.SC_PREC_F32_RU}


@pytest.fixture(scope="module")
def native():
    from paper_2205_03354_amd import _native

    return _native


def _gpu_bvp(native, dim, size, precision, tol=1e-10, **kw):
    from paper_2205_03354_amd import stencils

    bvp = S.biharmonic_bvp(dim, size)
    f = torch.from_numpy(bvp.f).to(DEV)
    g = torch.from_numpy(bvp.g).to(DEV)
    u = torch.zeros_like(f)
    st = native.solve_biharmonic(stencils.biharmonic(dim), bvp.h, f, u, g=g, g_halo=bvp.halo, tol=tol,
                                 precision=precision, **kw)
    return bvp, u.cpu().numpy(), st


@pytest.mark.parametrize("N", [17, 33, 65])
@pytest.mark.parametrize("prec", ["f64", "f32ir", "f32ru"])
def test_bvp2d_parity(native, N, prec):
    precision = _PREC[prec](native)
    bvp, x, st = _gpu_bvp(native, 2, N, precision)
    op = R.biharmonic(2)
    b = OP.bvp_rhs(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    rel = OP.true_relres(op, x, b, capi.ZERO_RING, bvp.h)
    assert rel <= 1e-10, rel
    assert st.rel_residual <= 1e-10
    xo, it, rel_o, rc = OP.bvp_solve(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    dx = np.max(np.abs(x - xo)) / np.max(np.abs(xo))
    assert dx <= 1e-6, dx
    e_gpu, e_or = np.max(np.abs(x - bvp.u)), np.max(np.abs(xo - bvp.u))
    assert abs(e_gpu - e_or) <= 1e-3 * e_or


@pytest.mark.parametrize("N", [33, 65])
def test_bvp2d_grid_solver_on_small_grids(native, N):
    # the grid solver itself (small 2D problems otherwise run on chip)
    bvp, x, st = _gpu_bvp(native, 2, N, native.SC_PREC_F64, onchip=False)
    op = R.biharmonic(2)
    b = OP.bvp_rhs(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert OP.true_relres(op, x, b, capi.ZERO_RING, bvp.h) <= 1e-10
    xo, it, rel_o, rc = OP.bvp_solve(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert np.max(np.abs(x - xo)) / np.max(np.abs(xo)) <= 1e-6
    assert st.iterations > 0 and st.outer >= 1


def test_bvp2d_second_order_on_gpu(native):
    errs, hs = [], []
    for N in (17, 33, 65):
        bvp, x, st = _gpu_bvp(native, 2, N, native.SC_PREC_F64)
        errs.append(np.max(np.abs(x - bvp.u)))
        hs.append(bvp.h)
    rate = math.log(errs[1] / errs[2]) / math.log(hs[1] / hs[2])
    assert abs(rate - 2) < 0.1


@pytest.mark.parametrize("n", [7, 15, 31])
@pytest.mark.parametrize("prec", ["f64", "f32ir", "f32ru"])
def test_bvp3d_parity(native, n, prec):
    precision = _PREC[prec](native)
    bvp, x, st = _gpu_bvp(native, 3, n, precision)
    op = R.biharmonic(3)
    b = OP.bvp_rhs(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert OP.true_relres(op, x, b, capi.ZERO_RING, bvp.h) <= 1e-10
    xo, it, rel_o, rc = OP.bvp_solve(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert np.max(np.abs(x - xo)) / np.max(np.abs(xo)) <= 1e-6


def test_bvp_zero_ring_and_initial_guess(native):
    # g = None (zero ring); starting from the oracle solution converges at once
    from paper_2205_03354_amd import stencils

    n = 40
    f_np = S.uniform_field((n, n + 3), seed=8)
    op = R.biharmonic(2)
    xo, it, rel, rc = capi.cg(op, f_np, None, capi.ZERO_RING, 1e-12)
    f = torch.from_numpy(f_np).to(DEV)
    u = torch.zeros_like(f)
    st = native.solve_biharmonic(stencils.biharmonic(2), 1.0, f, u, tol=1e-10)
    x = u.cpu().numpy()
    assert OP.true_relres(op, x, f_np, capi.ZERO_RING, 1.0) <= 1e-10
    u2 = torch.from_numpy(xo).to(DEV)
    st2 = native.solve_biharmonic(stencils.biharmonic(2), 1.0, f, u2, tol=1e-10)
    assert st2.iterations == 0


def test_bvp_deterministic(native):
    _, x1, s1 = _gpu_bvp(native, 2, 33, native.SC_PREC_F64)
    _, x2, s2 = _gpu_bvp(native, 2, 33, native.SC_PREC_F64)
    assert np.array_equal(x1, x2) and s1.iterations == s2.iterations


def test_breakdown_and_not_converged(native):
    from paper_2205_03354_amd import stencils

    n = 16
    f = torch.from_numpy(S.uniform_field((n, n), seed=1)).to(DEV)
    neg = native.stencil_lincomb([(-1, 1, 0, stencils.biharmonic(2))])  # negative definite
    u = torch.zeros_like(f)
    st = native.solve_biharmonic(neg, 1.0, f, u, raise_on_error=False)
    assert st.status == native.SC_EBREAKDOWN
    u = torch.zeros_like(f)
    st = native.solve_biharmonic(stencils.biharmonic(2), 1.0, f, u, max_iter=5, check_every=2,
                                 raise_on_error=False)
    assert st.status == native.SC_ENOTCONV and 5 <= st.iterations <= 6 and st.rel_residual > 1e-10


def _ch_gpu(native, u_np, h, eps, dt, Sst, steps, precision, tol=1e-10):
    from paper_2205_03354_amd import stencils

    u = torch.from_numpy(u_np).to(DEV)
    L = stencils.laplacian(u_np.ndim)
    stats = []
    for _ in range(steps):
        stats.append(native.ch_step(L, u, h, eps, dt, Sst, tol=tol, precision=precision))
    return u.cpu().numpy(), stats


@pytest.mark.parametrize("dim,N", [(2, 64), (3, 16)])
@pytest.mark.parametrize("prec", ["f64", "f32ir", "f32ru"])
def test_ch_step_parity(native, dim, N, prec):
    precision = _PREC[prec](native)
    h = 1.0 / N
    eps, dt, Sst = 4 * h, 0.1 * h * h, 2.0
    u0 = S.zero_mean_uniform((N,) * dim, seed=3)
    ug, _ = _ch_gpu(native, u0, h, eps, dt, Sst, 3, precision)
    uo = u0
    for _ in range(3):
        uo, it, rel, rc = OP.ch_step(uo, h, eps, dt, Sst)
    assert np.max(np.abs(ug - uo)) <= 1e-9 * max(1.0, np.max(np.abs(uo)))


def test_ch_single_mode_closed_form_gpu(native):
    from tests.test_oracle_numeric import _ch_mode_closed_form

    N = 32
    h = 1.0 / N
    eps, dt, Sst = 4 * h, 0.1 * h * h, 2.0
    u0, expect = _ch_mode_closed_form(0.3, N, (2, 1), eps, dt, Sst)
    ug, _ = _ch_gpu(native, u0, h, eps, dt, Sst, 1, native.SC_PREC_F64, tol=1e-14)
    assert np.max(np.abs(ug - expect)) <= 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32ir", "f32ru"])
def test_ch_mass_energy_gpu(native, prec):
    precision = _PREC[prec](native)
    N = 128
    h = 1.0 / N
    eps, dt, Sst = 4 * h, 0.1 * h * h, 2.0
    u0 = S.zero_mean_uniform((N, N), seed=9)
    from paper_2205_03354_amd import stencils

    u = torch.from_numpy(u0).to(DEV)
    L = stencils.laplacian(2)
    m0, E0 = native.grid_diagnostics(u, h, eps)
    assert abs(m0 - OP.mass(u0, h)) <= 1e-15
    assert abs(E0 - OP.ch_energy(u0, h, eps)) <= 1e-12 * abs(E0)
    E_prev = E0
    for _ in range(20):
        native.ch_step(L, u, h, eps, dt, Sst, precision=precision)
        m, E = native.grid_diagnostics(u, h, eps)
        assert abs(m - m0) <= 1e-12
        assert E <= E_prev + 1e-14 * abs(E_prev)
        E_prev = E
    assert E_prev < E0


@pytest.mark.parametrize("dim,N", [(2, 1024), (3, 256)])
@pytest.mark.parametrize("prec", ["f64", "f32ir", "f32ru"])
def test_ch_step_full_size(native, dim, N, prec):
    # the benchmark's CH configurations at their full sizes, one step in each
    # precision: the oracle's own apply confirms the step's true relative
    # residual on the whole grid; mass is conserved and the free energy does
    # not increase
    h = 1.0 / N
    eps, dt, Sst = 4 * h, 0.1 * h * h, 2.0
    u0 = S.zero_mean_uniform((N,) * dim, seed=5)
    ug, st = _ch_gpu(native, u0, h, eps, dt, Sst, 1, _PREC[prec](native))
    A = OP.ch_operator(dim, h, eps, dt, Sst)
    rel = OP.true_relres(A, ug, OP.ch_rhs(u0, h, dt, Sst), capi.PERIODIC, 1.0)
    assert rel <= 1e-10 and st[0].rel_residual <= 1e-10, (rel, st[0])
    assert abs(OP.mass(ug, h) - OP.mass(u0, h)) <= 1e-12
    E0, E1 = OP.ch_energy(u0, h, eps), OP.ch_energy(ug, h, eps)
    assert E1 <= E0 + 1e-14 * abs(E0)


# --------------------------------------------------------------- preconditioned
@pytest.mark.parametrize("N", [17, 33, 65, 129])
@pytest.mark.parametrize("prec", ["f64", "f32ir", "f32ru"])
def test_bvp2d_fast_poisson_parity(native, N, prec):
    # Same bars as the plain solve; the preconditioner must also cut the
    # iteration count to a few dozen at every size (plain CG: 43..2268).
    precision = _PREC[prec](native)
    bvp, x, st = _gpu_bvp(native, 2, N, precision, precond=native.SC_PC_FASTPOISSON)
    op = R.biharmonic(2)
    b = OP.bvp_rhs(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert OP.true_relres(op, x, b, capi.ZERO_RING, bvp.h) <= 1e-10
    xo, it, rel_o, rc = OP.bvp_solve(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert np.max(np.abs(x - xo)) / np.max(np.abs(xo)) <= 1e-6
    if prec == "f64":
        assert st.iterations <= 30, st.iterations
    else:
        assert st.iterations <= 150, st.iterations


@pytest.mark.parametrize("n", [7, 15, 31])
@pytest.mark.parametrize("prec", ["f64", "f32ru"])
def test_bvp3d_fast_poisson_parity(native, n, prec):
    precision = _PREC[prec](native)
    bvp, x, st = _gpu_bvp(native, 3, n, precision, precond=native.SC_PC_FASTPOISSON)
    op = R.biharmonic(3)
    b = OP.bvp_rhs(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert OP.true_relres(op, x, b, capi.ZERO_RING, bvp.h) <= 1e-10
    xo, it, rel_o, rc = OP.bvp_solve(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert np.max(np.abs(x - xo)) / np.max(np.abs(xo)) <= 1e-6
    if prec == "f64":
        assert st.iterations <= 40, st.iterations


def test_fast_poisson_fourth_order_operator(native):
    # The 33-point operator (the 4th-order Laplacian composed with itself)
    # with the 5-point-based preconditioner: spectrally equivalent, so still
    # few iterations, and the same solution as the oracle's CG.
    from paper_2205_03354_amd import stencils

    bvp = S.biharmonic_bvp(2, 65, halo=4)
    f = torch.from_numpy(bvp.f).to(DEV)
    g = torch.from_numpy(bvp.g).to(DEV)
    u = torch.zeros_like(f)
    st = native.solve_biharmonic(stencils.biharmonic(2, True), bvp.h, f, u, g=g, g_halo=4, tol=1e-10,
                                 precond=native.SC_PC_FASTPOISSON)
    op = R.biharmonic(2, True)
    x = u.cpu().numpy()
    b = OP.bvp_rhs(op, bvp.f, bvp.g, 4, bvp.h)
    assert OP.true_relres(op, x, b, capi.ZERO_RING, bvp.h) <= 1e-10
    xo, *_ = OP.bvp_solve(op, bvp.f, bvp.g, 4, bvp.h)
    assert np.max(np.abs(x - xo)) / np.max(np.abs(xo)) <= 1e-6
    assert st.iterations <= 80, st.iterations


def test_fast_poisson_rejects_unknown_option(native):
    from paper_2205_03354_amd import stencils

    bvp = S.biharmonic_bvp(2, 17)
    f = torch.from_numpy(bvp.f).to(DEV)
    u = torch.zeros_like(f)
    with pytest.raises(native.ScError):
        native.solve_biharmonic(stencils.biharmonic(2), bvp.h, f, u, precond=7)


def test_large_bvp_reaches_tolerance_with_compensated_residual(native):
    # 2049^2 nodes: an FP64 stencil sum rounds the residual near 1e-10 of |b|
    # here (|A||x| ~ 1e15 in the interior); the double-double residual lets
    # the preconditioned solve stop at the requested 1e-10. The solution is
    # checked against the manufactured u at the discretisation error O(h^2)
    # (1.6e-7 at this h, from the 2nd-order rate pinned on small grids), and
    # the oracle recomputes the residual with extended-precision sums.
    bvp, x, st = _gpu_bvp(native, 2, 2049, native.SC_PREC_F64, precond=native.SC_PC_FASTPOISSON)
    assert st.status == native.SC_OK and st.rel_residual <= 1e-10
    assert np.max(np.abs(x - bvp.u)) <= 2.5e-7
    rel = OP.bvp_relres_extended(R.biharmonic(2), x, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert rel <= 1e-10, rel


@pytest.mark.parametrize("n", [63, 127, 255])
def test_bvp3d_full_sizes(native, n):
    # the 3D BVP configuration's sizes (64^3 - 256^3 grids, 25-point L o L,
    # 2-ring halo from the exact u), preconditioned FP64 CG: the oracle
    # recomputes the residual with extended-precision sums, and the error
    # against the manufactured solution is second order (0.79 h^2 at n = 63
    # from the pinned rates, bounded here by h^2)
    bvp, x, st = _gpu_bvp(native, 3, n, native.SC_PREC_F64, precond=native.SC_PC_FASTPOISSON)
    assert st.status == native.SC_OK and st.rel_residual <= 1e-10, st
    rel = OP.bvp_relres_extended(R.biharmonic(3), x, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert rel <= 1e-10, rel
    assert np.max(np.abs(x - bvp.u)) <= bvp.h ** 2


@pytest.mark.parametrize("N", [1922, 1968, 2036])
def test_large_bvps_reach_tolerance_through_restarts(native, N):
    # Near 2000 nodes a side, |b| of these BVPs comes from the ring terms and
    # rounding the solution itself to FP64 leaves a true relative residual of
    # about 6e-11, close under the 1e-10 target. A run whose recurrence stops
    # at the tolerance then confirms a true residual just above it; restarts
    # therefore aim at half the tolerance, and every size reaches 1e-10
    # (sizes of the serving stream; one of them stagnated at 1.003e-10 when
    # restarts stopped at the tolerance itself).
    bvp, x, st = _gpu_bvp(native, 2, N, native.SC_PREC_F64, precond=native.SC_PC_FASTPOISSON)
    assert st.status == native.SC_OK and st.rel_residual <= 1e-10, st
    rel = OP.bvp_relres_extended(R.biharmonic(2), x, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert rel <= 1e-10, rel


def _mixed_spd_3d():
    # -L + d_x d_y in 3D: symmetric (w(-u) = w(u)) but not mirror-symmetric,
    # so its direction sweep is the general 3D kernel; SPD since
    # |sin tx sin ty| <= 2 (sin^2(tx/2) + sin^2(ty/2))
    dxdy = R.compose(R.embed(R.central_first(), 0, 3), R.embed(R.central_first(), 1, 3))
    return R.lincomb([(-1, 0, R.laplacian(3)), (1, 0, dxdy)])


@pytest.mark.parametrize("case", ["bvp2d", "ch3d", "mixed3d"])
def test_folded_update_finish_is_bit_identical(native, case):
    # Within a graph block the CG update's finish (beta, stop test) is formed
    # by the next direction sweep in the finish kernel's own summation
    # order; with one iteration per block nothing is folded. Both must give
    # the same solution bit for bit and the same iteration count.
    from paper_2205_03354_amd import stencils

    def run(every):
        if case == "ch3d":
            u0 = S.zero_mean_uniform((24, 24, 24), seed=61)
            u = torch.from_numpy(u0).to(DEV)
            h = 1.0 / 24
            st = native.ch_step(stencils.laplacian(3), u, h, 4 * h, 0.1 * h * h, 2.0, tol=1e-10, check_every=every)
            return u.cpu().numpy(), st
        if case == "bvp2d":
            op, shape, h = stencils.biharmonic(2), (127, 127), 1.0 / 128
        else:
            op, shape, h = lib_stencil(native, _mixed_spd_3d()), (20, 21, 22), 1.0 / 23
        f = torch.from_numpy(S.uniform_field(shape, seed=62)).to(DEV)
        u = torch.zeros_like(f)
        st = native.solve_biharmonic(op, h, f, u, tol=1e-10, check_every=every, onchip=False)
        return u.cpu().numpy(), st

    x1, s1 = run(1)
    x2, s2 = run(16)
    assert s1.rel_residual <= 1e-10 and s2.rel_residual <= 1e-10
    assert s1.iterations == s2.iterations, (s1, s2)
    assert np.array_equal(x1, x2)


@pytest.mark.parametrize("N", [801, 900])
def test_split_sine_transforms_match_full_products(native, monkeypatch, N):
    # 2D sides >= 768 split each GEMM sine transform by the matrix's even /
    # odd symmetry (odd and even interior sizes here); the preconditioned
    # solve converges either way, the oracle confirms both residuals, and
    # the two solutions agree to kappa times the tolerance
    sols = []
    for mode in ("1", "0"):
        monkeypatch.setenv("SCOMP_PCSPLIT", mode)
        bvp, x, st = _gpu_bvp(native, 2, N, native.SC_PREC_F64, precond=native.SC_PC_FASTPOISSON)
        assert st.status == native.SC_OK and st.rel_residual <= 1e-10, (mode, st)
        rel = OP.bvp_relres_extended(R.biharmonic(2), x, bvp.f, bvp.g, bvp.halo, bvp.h)
        assert rel <= 1e-10, (mode, rel)
        sols.append(x)
    assert np.max(np.abs(sols[0] - sols[1])) <= 1e-7 * np.max(np.abs(sols[1]))
