"""Request-server scheduling on the host (no device work).

The server's fake-device mode runs the real admission, budget, cancellation
and retirement logic with every device call left out, so the scheduler is
checked here without a GPU. What the device path computes is checked by the
GPU tests (alone-vs-mix identity and parity with the blocking solve).
"""

import time

import numpy as np
import pytest

from paper_2205_03354_amd import _native as nat
from paper_2205_03354_amd import stencils


def _op():
    return stencils.biharmonic(2, fourth_order=False)


def _lap():
    return stencils.laplacian(2, fourth_order=False)


def _drain(srv, n, timeout=20.0):
    got = []
    t_end = time.time() + timeout
    while len(got) < n and time.time() < t_end:
        got += srv.poll(wait_ms=50)
    assert len(got) == n, f"only {len(got)} of {n} results"
    return {r["id"]: r for r in got}


def test_fifo_admission_and_completion():
    op = _op()
    srv = nat.Server(fake_device=True, max_slots=2)
    try:
        ids = [srv.submit_bvp(op, 1.0 / 33, np.ones((31 + 8 * k, 31))) for k in range(6)]
        assert ids == sorted(ids) and len(set(ids)) == 6
        res = _drain(srv, 6)
        admits = [res[i]["t_admit"] for i in ids]
        assert admits == sorted(admits), "requests must be admitted in arrival order"
        for i in ids:
            r = res[i]
            assert r["status"] == nat.SC_OK
            assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
            assert r["device_bytes"] > 0
        assert srv.load() == {"queued": 0, "active": 0, "finished": 0, "device_bytes": 0}
    finally:
        srv.close()


def test_footprint_grows_with_size_and_budget_serialises():
    op = _op()
    srv = nat.Server(fake_device=True, max_slots=4)
    try:
        a = srv.submit_bvp(op, 1.0 / 33, np.ones((31, 31)))
        b = srv.submit_bvp(op, 1.0 / 65, np.ones((63, 63)))
        res = _drain(srv, 2)
        assert res[b]["device_bytes"] > res[a]["device_bytes"]
        one = res[b]["device_bytes"]
    finally:
        srv.close()
    # A budget that holds one request at a time: each admission waits for the
    # previous retirement, even though slots are free.
    srv = nat.Server(fake_device=True, max_slots=4, hbm_budget=int(one * 1.5))
    try:
        ids = [srv.submit_bvp(op, 1.0 / 65, np.ones((63, 63))) for _ in range(4)]
        res = _drain(srv, 4)
        for prev, nxt in zip(ids, ids[1:]):
            assert res[nxt]["t_admit"] >= res[prev]["t_done"]
    finally:
        srv.close()


def test_request_larger_than_budget_is_rejected():
    op = _op()
    srv = nat.Server(fake_device=True, max_slots=2, hbm_budget=4096)
    try:
        rid = srv.submit_bvp(op, 1.0 / 33, np.ones((31, 31)))
        res = _drain(srv, 1)
        assert res[rid]["status"] == nat.SC_ENOMEM
    finally:
        srv.close()


def test_cancel_queued_and_unknown():
    op = _op()
    # One slot and a long-running head keep the later requests queued while
    # one of them is cancelled.
    srv = nat.Server(fake_device=True, max_slots=1)
    try:
        big = srv.submit_bvp(op, 1.0 / 1025, np.ones((1023, 1023)))
        queued = [srv.submit_bvp(op, 1.0 / 33, np.ones((31, 31))) for _ in range(3)]
        srv.cancel(queued[1])
        res = _drain(srv, 4)
        assert res[queued[1]]["status"] == nat.SC_ECANCELLED
        assert res[big]["status"] == nat.SC_OK
        assert res[queued[0]]["status"] == nat.SC_OK and res[queued[2]]["status"] == nat.SC_OK
        with pytest.raises(nat.ScError):
            srv.cancel(queued[1])  # already finished
        with pytest.raises(nat.ScError):
            srv.cancel(10**9)
    finally:
        srv.close()


def test_ch_requests_and_bad_requests():
    lap = _lap()
    srv = nat.Server(fake_device=True, max_slots=3)
    try:
        u0 = np.zeros((32, 32))
        rid = srv.submit_ch(lap, u0, 1.0 / 32, 0.05, 1e-3, 2.0)
        res = _drain(srv, 1)
        assert res[rid]["status"] == nat.SC_OK
        with pytest.raises(nat.ScError):
            srv.submit_bvp(stencils.biharmonic(3, fourth_order=False), 0.1, np.ones((8, 8)))
        with pytest.raises(nat.ScError):
            srv.submit_ch(lap, u0, 1.0 / 32, -1.0, 1e-3, 2.0)  # eps must be positive
    finally:
        srv.close()


def test_destroy_with_queued_requests_returns():
    op = _op()
    srv = nat.Server(fake_device=True, max_slots=1)
    for _ in range(20):
        srv.submit_bvp(op, 1.0 / 257, np.ones((255, 255)))
    t = time.time()
    srv.close()
    assert time.time() - t < 10.0


def test_precision_validation():
    op = _op()
    with pytest.raises(nat.ScError):
        nat.Server(fake_device=True, precision=9)
    srv = nat.Server(fake_device=True, max_slots=2)
    try:
        with pytest.raises(nat.ScError):
            srv.submit_bvp(op, 1.0 / 33, np.ones((31, 31)), precision=7)
        ids = [srv.submit_bvp(op, 1.0 / 33, np.ones((31, 31)), precision=p)
               for p in (nat.SC_PREC_F64, nat.SC_PREC_F32_IR, nat.SC_PREC_F32_RU)]
        res = _drain(srv, 3)
        assert all(res[i]["status"] == nat.SC_OK for i in ids)
    finally:
        srv.close()
