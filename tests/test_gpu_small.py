"""GPU parity of the batched small-grid BVP solver (one workgroup per problem).

The same bars as the large-grid solver: the oracle recomputes the true
relative residual of the returned solution (<= 1e-10), the solution agrees
with the oracle's CG solution to 1e-6 (kappa times the tolerance), and the
discretisation error against the manufactured solution matches the
oracle's. A problem solved inside a mixed batch is bit-identical to the same
problem solved alone.
"""

import numpy as np
import pytest
import torch

import synthetic as S
from oracle import capi
from oracle import problems as OP
from oracle import rational as R

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def native():
    from paper_2205_03354_amd import _native

    return _native


def _problem(N, fourth=False, seed=None):
    bvp = S.biharmonic_bvp(2, N, halo=4 if fourth else 2)
    f = torch.from_numpy(bvp.f).to(DEV)
    g = torch.from_numpy(bvp.g).to(DEV)
    u0 = np.zeros_like(bvp.f) if seed is None else S.uniform_field(bvp.f.shape, seed=seed)
    u = torch.from_numpy(u0).to(DEV)
    return bvp, (bvp.h, f, u, g, bvp.halo)


@pytest.mark.parametrize("N", [17, 33, 65])
def test_batched_bvp_parity(native, N):
    from paper_2205_03354_amd import stencils

    bvp, prob = _problem(N)
    status, st = native.solve_biharmonic_batch(stencils.biharmonic(2), [prob])
    x = prob[2].cpu().numpy()
    op = R.biharmonic(2)
    b = OP.bvp_rhs(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    rel = OP.true_relres(op, x, b, capi.ZERO_RING, bvp.h)
    assert rel <= 1e-10 and st[0].rel_residual <= 1e-10, (rel, st[0])
    xo, it, rel_o, rc = OP.bvp_solve(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert np.max(np.abs(x - xo)) / np.max(np.abs(xo)) <= 1e-6
    e_gpu, e_or = np.max(np.abs(x - bvp.u)), np.max(np.abs(xo - bvp.u))
    assert abs(e_gpu - e_or) <= 1e-3 * e_or


def test_fourth_order_operator(native):
    from paper_2205_03354_amd import stencils

    bvp, prob = _problem(33, fourth=True)
    native.solve_biharmonic_batch(stencils.biharmonic(2, True), [prob])
    op = R.biharmonic(2, True)
    x = prob[2].cpu().numpy()
    b = OP.bvp_rhs(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert OP.true_relres(op, x, b, capi.ZERO_RING, bvp.h) <= 1e-10


def test_batch_members_equal_alone(native):
    from paper_2205_03354_amd import stencils

    op = stencils.biharmonic(2)
    sizes = [(65, None), (17, 3), (33, None), (65, 5), (20, 7)]
    alone = []
    for N, seed in sizes:
        _, prob = _problem(N, seed=seed)
        _, st = native.solve_biharmonic_batch(op, [prob])
        alone.append((prob[2].cpu().numpy(), st[0].iterations, st[0].rel_residual))
    probs = [_problem(N, seed=seed)[1] for N, seed in sizes]
    _, sts = native.solve_biharmonic_batch(op, probs)
    for (x, it, rel), p, st in zip(alone, probs, sts):
        got = p[2].cpu().numpy()
        assert np.array_equal(got, x), float(np.max(np.abs(got - x)))
        assert st.iterations == it and st.rel_residual == rel


def test_zero_ring_and_initial_guess(native):
    # g omitted: b = f; a converged initial guess returns at once
    from paper_2205_03354_amd import stencils

    op = R.biharmonic(2)
    n, h = 30, 1.0 / 31
    f = S.uniform_field((n, n), seed=9)
    ft = torch.from_numpy(f).to(DEV)
    u = torch.zeros_like(ft)
    native.solve_biharmonic_batch(stencils.biharmonic(2), [(h, ft, u, None, 0)])
    x = u.cpu().numpy()
    assert OP.true_relres(op, x, f, capi.ZERO_RING, h) <= 1e-10
    _, st = native.solve_biharmonic_batch(stencils.biharmonic(2), [(h, ft, u, None, 0)])
    assert st[0].iterations == 0 and np.array_equal(u.cpu().numpy(), x)


def test_matches_the_large_grid_solver(native):
    from paper_2205_03354_amd import stencils

    bvp, prob = _problem(65)
    native.solve_biharmonic_batch(stencils.biharmonic(2), [prob])
    u2 = torch.zeros_like(prob[1])
    native.solve_biharmonic(stencils.biharmonic(2), bvp.h, prob[1], u2, g=prob[3], g_halo=bvp.halo)
    a, b = prob[2].cpu().numpy(), u2.cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-7 * np.max(np.abs(b))


def test_iteration_limit_and_errors(native):
    from paper_2205_03354_amd import stencils

    op = stencils.biharmonic(2)
    _, prob = _problem(33)
    status, st = native.solve_biharmonic_batch(op, [prob], max_iter=5, raise_on_error=False)
    assert status == native.SC_ENOTCONV and st[0].iterations == 5 and st[0].rel_residual > 1e-10
    big = torch.zeros((65, 65), dtype=torch.float64, device=DEV)  # 4225 unknowns > 4096
    with pytest.raises(native.ScError):
        native.solve_biharmonic_batch(op, [(1.0 / 66, big, big.clone(), None, 0)])
    f32 = torch.zeros((16, 16), dtype=torch.float32, device=DEV)
    with pytest.raises(native.ScError):
        native.solve_biharmonic_batch(op, [(0.1, f32, f32.clone(), None, 0)])
    with pytest.raises(native.ScError):
        native.solve_biharmonic_batch(stencils.biharmonic(3), [(0.1, big, big.clone(), None, 0)])
    status, st = native.solve_biharmonic_batch(op, [])
    assert status == native.SC_OK and st == []


def test_blocking_solve_runs_small_problems_on_chip(native):
    # sc_solve_biharmonic takes the on-chip kernel for problems that fit, so
    # its result equals the batch call's; the grid solver agrees to kappa tol
    from paper_2205_03354_amd import stencils

    op = stencils.biharmonic(2)
    bvp, prob = _problem(33)
    u1 = torch.zeros_like(prob[1])
    st1 = native.solve_biharmonic(op, bvp.h, prob[1], u1, g=prob[3], g_halo=bvp.halo)
    _, st2 = native.solve_biharmonic_batch(op, [prob])
    assert np.array_equal(u1.cpu().numpy(), prob[2].cpu().numpy())
    assert st1.iterations == st2[0].iterations and st1.rel_residual == st2[0].rel_residual
    u3 = torch.zeros_like(prob[1])
    st3 = native.solve_biharmonic(op, bvp.h, prob[1], u3, g=prob[3], g_halo=bvp.halo, onchip=False)
    assert st3.rel_residual <= 1e-10
    a, b = u1.cpu().numpy(), u3.cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-7 * np.max(np.abs(b))
