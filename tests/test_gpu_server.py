"""GPU tests of the graph-captured CG blocks and of the request server.

Bars: bit-identical. A graph replay launches the same kernels with the same
arguments as the eager launches, and a served request runs the same kernels
on buffers of its own, so the solution, iteration count and residual must be
equal to the last bit, alone or in a mix of concurrent requests.
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
def nat():
    from paper_2205_03354_amd import _native

    return _native


@pytest.fixture(scope="module")
def ops():
    from paper_2205_03354_amd import stencils

    return {2: stencils.biharmonic(2), 3: stencils.biharmonic(3),
            "L2": stencils.laplacian(2), "L3": stencils.laplacian(3)}


def _blocking_bvp(nat, op, bvp, precision, use_graph, check_every=64):
    f = torch.from_numpy(bvp.f).to(DEV)
    g = torch.from_numpy(bvp.g).to(DEV)
    u = torch.zeros_like(f)
    st = nat.solve_biharmonic(op, bvp.h, f, u, g=g, g_halo=bvp.halo, tol=1e-10, precision=precision,
                              check_every=check_every, use_graph=use_graph)
    return u.cpu().numpy(), st


def _blocking_ch(nat, lap, u0, h, eps, dt, Sst, precision, use_graph):
    u = torch.from_numpy(u0.copy()).to(DEV)
    st = nat.ch_step(lap, u, h, eps, dt, Sst, tol=1e-10, precision=precision, use_graph=use_graph)
    return u.cpu().numpy(), st


@pytest.mark.parametrize("prec", ["f64", "f32ir", "f32ru"])
@pytest.mark.parametrize("check_every", [7, 8, 64])
def test_graph_blocks_bit_identical_bvp(nat, ops, prec, check_every):
    precision = {"f64": nat.SC_PREC_F64, "f32ir": nat.SC_PREC_F32_IR, "f32ru": nat.SC_PREC_F32_RU}[prec]
    bvp = S.biharmonic_bvp(2, 33)
    x0, s0 = _blocking_bvp(nat, ops[2], bvp, precision, False, check_every)
    # Several solves with graphs: each replays its captured block many times,
    # with eager work and synchronisation between the solves.
    for rep in range(3):
        x1, s1 = _blocking_bvp(nat, ops[2], bvp, precision, True, check_every)
        assert s1.iterations == s0.iterations and s1.outer == s0.outer
        assert s1.rel_residual == s0.rel_residual
        assert np.array_equal(x1, x0), f"replay set {rep} differs"
        torch.cuda.synchronize()
    assert s0.iterations > 2 * check_every  # the graph really was replayed


def test_graph_blocks_bit_identical_3d_and_ch(nat, ops):
    bvp = S.biharmonic_bvp(3, 15)
    x0, s0 = _blocking_bvp(nat, ops[3], bvp, nat.SC_PREC_F64, False, 16)
    x1, s1 = _blocking_bvp(nat, ops[3], bvp, nat.SC_PREC_F64, True, 16)
    assert s1.iterations == s0.iterations and np.array_equal(x1, x0)
    u0 = S.zero_mean_uniform((64, 64), seed=5)
    prm = (1.0 / 64, 0.05, 1e-4, 2.0)
    y0, t0 = _blocking_ch(nat, ops["L2"], u0, *prm, nat.SC_PREC_F64, False)
    y1, t1 = _blocking_ch(nat, ops["L2"], u0, *prm, nat.SC_PREC_F64, True)
    assert t1.iterations == t0.iterations and np.array_equal(y1, y0)


def _serve(nat, jobs, max_slots, **kw):
    """Submit `jobs` (kind, args...) to a fresh server, return results by index."""
    srv = nat.Server(max_slots=max_slots, tol=1e-10, **kw)
    try:
        ids = []
        for j in jobs:
            if j[0] == "bvp":
                _, op, bvp, prec = j
                ids.append(srv.submit_bvp(op, bvp.h, bvp.f, g=bvp.g, precision=prec))
            else:
                _, lap, u0, prm, prec = j
                ids.append(srv.submit_ch(lap, u0, *prm, precision=prec))
        got = {}
        for _ in range(6000):
            for r in srv.poll(wait_ms=10):
                got[r["id"]] = r
            if len(got) == len(ids):
                break
        assert len(got) == len(ids), srv.load()
        return [(got[i], srv.result_array(i)) for i in ids]
    finally:
        srv.close()


def _job_mix(nat, ops):
    jobs = []
    for k, N in enumerate((17, 33, 65, 33, 17, 49)):
        prec = (nat.SC_PREC_F64, nat.SC_PREC_F32_IR, nat.SC_PREC_F32_RU)[k % 3]
        jobs.append(("bvp", ops[2], S.biharmonic_bvp(2, N), prec))
    jobs.append(("bvp", ops[3], S.biharmonic_bvp(3, 15), nat.SC_PREC_F64))
    jobs.append(("ch", ops["L2"], S.zero_mean_uniform((64, 64), seed=7), (1.0 / 64, 0.05, 1e-4, 2.0),
                 nat.SC_PREC_F64))
    jobs.append(("ch", ops["L3"], S.zero_mean_uniform((16, 16, 16), seed=8), (1.0 / 16, 0.1, 1e-3, 2.0),
                 nat.SC_PREC_F32_IR))
    jobs.append(("ch", ops["L3"], S.zero_mean_uniform((20, 20, 20), seed=9), (1.0 / 20, 0.1, 1e-3, 2.0),
                 nat.SC_PREC_F32_RU))
    return jobs


def test_server_alone_vs_mix_bit_identical(nat, ops):
    jobs = _job_mix(nat, ops)
    alone = [_serve(nat, [j], 1)[0] for j in jobs]
    mixed = _serve(nat, jobs, 16)
    mixed2 = _serve(nat, jobs[::-1], 3)[::-1]
    for (ra, xa), (rm, xm), (r2, x2) in zip(alone, mixed, mixed2):
        assert ra["status"] == nat.SC_OK
        assert rm["status"] == ra["status"] and r2["status"] == ra["status"]
        assert rm["iterations"] == ra["iterations"] == r2["iterations"]
        assert rm["rel_residual"] == ra["rel_residual"]
        assert np.array_equal(xm, xa) and np.array_equal(x2, xa)


def test_server_matches_blocking_entry_points(nat, ops):
    jobs = _job_mix(nat, ops)[:4] + _job_mix(nat, ops)[-2:]
    served = _serve(nat, jobs, 8)
    for j, (r, x) in zip(jobs, served):
        if j[0] == "bvp":
            _, op, bvp, prec = j
            xb, sb = _blocking_bvp(nat, op, bvp, prec, True)
        else:
            _, lap, u0, prm, prec = j
            xb, sb = _blocking_ch(nat, lap, u0, *prm, prec, True)
        assert r["iterations"] == sb.iterations
        assert np.array_equal(x, xb)


def test_served_bvp_against_oracle(nat, ops):
    bvp = S.biharmonic_bvp(2, 33)
    (r, x), = _serve(nat, [("bvp", ops[2], bvp, nat.SC_PREC_F64)], 2)
    op = R.biharmonic(2)
    b = OP.bvp_rhs(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert OP.true_relres(op, x, b, capi.ZERO_RING, bvp.h) <= 1e-10
    xo, *_ = OP.bvp_solve(op, bvp.f, bvp.g, bvp.halo, bvp.h)
    assert np.max(np.abs(x - xo)) / np.max(np.abs(xo)) <= 1e-6


def test_server_cancel_and_budget_on_device(nat, ops):
    srv = nat.Server(max_slots=1, tol=1e-10)
    try:
        big = srv.submit_bvp(ops[2], 1.0 / 256, np.ones((255, 255)))
        small = srv.submit_bvp(ops[2], 1.0 / 18, np.ones((16, 16)))
        srv.cancel(big)
        got = {}
        for _ in range(3000):
            for r in srv.poll(wait_ms=10):
                got[r["id"]] = r
            if len(got) == 2:
                break
        assert got[big]["status"] == nat.SC_ECANCELLED
        assert got[small]["status"] == nat.SC_OK
        assert srv.load()["device_bytes"] == 0
    finally:
        srv.close()
    srv = nat.Server(max_slots=2, hbm_budget=1 << 16)
    try:
        rid = srv.submit_bvp(ops[2], 1.0 / 66, np.ones((64, 64)))
        res = []
        for _ in range(300):
            res += srv.poll(wait_ms=10)
            if res:
                break
        assert res[0]["id"] == rid and res[0]["status"] == nat.SC_ENOMEM
    finally:
        srv.close()


def test_server_preconditioned_alone_vs_mix(nat, ops):
    # Preconditioned BVPs (library GEMMs on each request's stream) next to
    # plain and CH requests: still bit-identical alone and in the mix.
    jobs = _job_mix(nat, ops)
    alone = [_serve(nat, [j], 1, precond=nat.SC_PC_FASTPOISSON)[0] for j in jobs]
    mixed = _serve(nat, jobs, 16, precond=nat.SC_PC_FASTPOISSON)
    for j, (ra, xa), (rm, xm) in zip(jobs, alone, mixed):
        assert ra["status"] == nat.SC_OK and rm["status"] == nat.SC_OK
        assert rm["iterations"] == ra["iterations"]
        assert np.array_equal(xm, xa)
        if j[0] == "bvp" and j[3] == nat.SC_PREC_F64:
            assert ra["iterations"] <= 40
