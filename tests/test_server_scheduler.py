"""Admission and scheduling of the request server, on the CPU: the fake
executor runs the real scheduler with simulated chunk times and no device."""
import time

import numpy as np
import pytest

from paper_1702_02207_amd import osc


@pytest.fixture(scope="module")
def lib():
    import os
    if not os.path.exists(osc.LIB_PATH):
        pytest.skip("libosc.so not built")
    return osc.load()


def _chain(s, rng):
    m = rng.uniform(0.5, 2.0, s)
    k = np.exp(rng.uniform(np.log(1e2), np.log(1e4), s))
    return m, k


def _submit_chain(srv, s, nsteps, rng, stride=0):
    m, k = _chain(s, rng)
    return srv.submit("chain", "rk4", "f32", m, k, [1e-4], rng.normal(size=s), np.zeros(s), nsteps, stride)


def test_all_requests_complete_within_budget(lib):
    rng = np.random.default_rng(0)
    one = None
    with osc.Server(hbm_budget=0, max_slots=1, fake_executor=True) as probe:
        t = _submit_chain(probe, 64, 100, rng)
        one = probe.wait(t)["bytes"]
    budget = 5 * one + one // 2          # room for five requests of this size
    with osc.Server(hbm_budget=budget, max_slots=64, fake_executor=True) as srv:
        tickets = [_submit_chain(srv, 64, 20000, rng) for _ in range(40)]
        peak_seen = 0
        for t in tickets:
            r = srv.wait(t, timeout=30.0)
            assert r["latency_s"] >= r["queue_s"] >= 0.0
            peak_seen = max(peak_seen, srv.stats()["hbm_peak"])
        st = srv.stats()
    assert st["completed"] == 40 and st["failed"] == 0
    assert 0 < st["hbm_peak"] <= budget
    assert st["hbm_peak"] >= 4 * one      # several requests really ran together


def test_fifo_order_with_one_slot(lib):
    rng = np.random.default_rng(1)
    with osc.Server(max_slots=1, fake_executor=True) as srv:
        tickets = [_submit_chain(srv, 8, 3000, rng) for _ in range(6)]
        res = [srv.wait(t, timeout=30.0) for t in tickets]
    # with one slot, each request waits for all earlier ones
    q = [r["queue_s"] for r in res]
    assert all(b >= a for a, b in zip(q, q[1:]))


def test_late_short_request_overtakes_long_one(lib):
    rng = np.random.default_rng(2)
    with osc.Server(max_slots=8, fake_executor=True) as srv:
        long_t = _submit_chain(srv, 16, 2_000_000, rng)
        time.sleep(0.02)
        short_t = _submit_chain(srv, 16, 100, rng)
        short = srv.wait(short_t, timeout=10.0)
        with pytest.raises(osc.OscError) as e:
            srv.wait(long_t, timeout=0.0)
        assert e.value.status == osc.OSC_ETIMEOUT
        assert short["queue_s"] < 0.5
        srv.wait(long_t, timeout=60.0)


def test_oversized_and_invalid_requests_rejected(lib):
    rng = np.random.default_rng(3)
    with osc.Server(hbm_budget=1 << 16, max_slots=4, fake_executor=True) as srv:
        with pytest.raises(osc.OscError) as e:
            _submit_chain(srv, 2000, 10, rng, stride=1)      # frames alone exceed 64 KiB
        assert e.value.status == osc.OSC_ENOMEM
        with pytest.raises(ValueError):      # the binding refuses it before the call
            srv.submit("chain", "rk4", "f32", np.ones(3), np.ones(3), [1e-3], np.zeros(3), np.zeros(3), -1)
        # the library itself refuses it too
        import ctypes
        par = np.ones(3)
        st0 = np.zeros(3, dtype=np.float32)
        dtv = np.array([1e-3])
        d = osc.Desc(0, 0, 1, 3, 1, 0, osc.MEM_HOST, par.ctypes.data, par.ctypes.data, dtv.ctypes.data)
        t = ctypes.c_uint64()
        assert lib.osc_server_submit(srv.handle, ctypes.byref(d), st0.ctypes.data, st0.ctypes.data, -1, 0,
                                     ctypes.byref(t)) == osc.OSC_EINVAL
        with pytest.raises(osc.OscError):
            srv.wait(12345, timeout=0.0)
    with pytest.raises(osc.OscError):
        osc.Server(max_slots=0, fake_executor=True)


def test_shutdown_fails_queued_requests(lib):
    rng = np.random.default_rng(4)
    srv = osc.Server(max_slots=1, fake_executor=True)
    for _ in range(5):
        _submit_chain(srv, 4, 5_000_000, rng)
    time.sleep(0.05)
    st = srv.stats()
    assert st["active"] == 1 and st["queued"] == 4
    t0 = time.time()
    srv.close()          # finishes the admitted one, fails the four queued ones
    assert time.time() - t0 < 30.0
