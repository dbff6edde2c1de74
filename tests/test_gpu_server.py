"""GPU tests of the request server: results match the FP64 oracle, each
request's result is bitwise the same alone and in a mix, and late arrivals
are admitted while earlier requests run."""
import numpy as np
import pytest

import oracle
from paper_1702_02207_amd import osc, workloads

pytestmark = pytest.mark.gpu


def _stream(n, seed, s_max=600, nsteps=(200, 3000)):
    return workloads.c5_request_stream(n_requests=n, qps=1e6, s_max=s_max, nsteps_range=nsteps,
                                       seed_salt=seed)


def _submit(srv, req, method="rk4"):
    w = req.system
    if req.kind == "chain":
        return srv.submit("chain", method, "f32", w.m[0], w.k[0], w.dt, w.x0[0], w.v0[0], w.nsteps, w.out_stride)
    return srv.submit("dense", method, "f32", w.M, w.K, w.dt, w.x0[0], w.v0[0], w.nsteps, w.out_stride)


def _oracle(req, method="rk4"):
    w = req.system
    x0 = w.x0.astype(np.float32).astype(np.float64)
    v0 = w.v0.astype(np.float32).astype(np.float64)
    if req.kind == "chain":
        xf, vf, _, _ = oracle.chain(method, w.m, w.k, w.dt, x0, v0, w.nsteps, w.out_stride)
    else:
        xf, vf, _, _ = oracle.dense(method, w.M, w.K, w.dt, x0, v0, w.nsteps, w.out_stride)
    return xf[:, 0], vf[:, 0]


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_served_results_match_oracle_and_are_identical_alone_and_in_mix(method):
    reqs = _stream(20, seed=11)
    with osc.Server(max_slots=64, chunk_us=500) as srv:
        tickets = [_submit(srv, r, method) for r in reqs]
        mixed = [srv.wait(t, timeout=120.0) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    for r, res in zip(reqs, mixed):
        rx, rv = _oracle(r, method)
        ex = oracle.rel_traj_err(res["x_frames"][:, None, :], rx[:, None, :])[0]
        ev = oracle.rel_traj_err(res["v_frames"][:, None, :], rv[:, None, :])[0]
        assert ex < 1e-5 and ev < 1e-5, (r.kind, r.system.s, ex, ev)
    # each request alone on a fresh server
    for i in (0, 3, 7, 12, 19):
        with osc.Server(max_slots=4, chunk_us=500) as srv:
            alone = srv.wait(_submit(srv, reqs[i], method), timeout=120.0)
        for key in ("x_frames", "v_frames", "x_end", "v_end"):
            np.testing.assert_array_equal(alone[key], mixed[i][key])


def test_budget_respected_on_device():
    reqs = _stream(16, seed=5, s_max=300)
    with osc.Server(max_slots=64) as srv:
        sizes = [srv.wait(t, timeout=120.0)["bytes"] for t in [_submit(srv, r) for r in reqs]]
    budget = 2 * max(sizes) + (1 << 20)      # at most a few requests fit at once
    with osc.Server(hbm_budget=budget, max_slots=64) as srv:
        tickets = [_submit(srv, r) for r in reqs]
        for t in tickets:
            srv.wait(t, timeout=120.0)
        st = srv.stats()
    assert st["completed"] == len(reqs)
    assert max(sizes) <= st["hbm_peak"] <= budget


def test_continuous_admission():
    rng = np.random.default_rng(9)
    s = 512
    m = rng.uniform(0.5, 2.0, s)
    k = np.exp(rng.uniform(np.log(1e2), np.log(1e4), s))
    dt = 0.01 / workloads.chain_omega_max(m[None], k[None])
    with osc.Server(max_slots=16, chunk_us=1000) as srv:
        long_t = srv.submit("chain", "rk4", "f32", m, k, dt, rng.normal(0, 0.1, s), np.zeros(s), 400_000, 0)
        import time
        time.sleep(0.05)
        short_t = srv.submit("chain", "rk4", "f32", m, k, dt, rng.normal(0, 0.1, s), np.zeros(s), 1000, 0)
        short = srv.wait(short_t, timeout=60.0)
        st = srv.stats()
        assert st["active"] >= 1            # the long request is still running
        long = srv.wait(long_t, timeout=120.0)
    assert short["latency_s"] < long["latency_s"]


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_long_chains_in_one_work_list(method):
    """Chains of 1025-2048 DOFs (one instance over the two waves of a
    workgroup, halo across them through LDS) with different step counts and
    frame strides served together: each matches the oracle and is bitwise
    the same as when served alone."""
    rng = np.random.default_rng(21)
    reqs = []
    for s, nsteps, stride in ((1025, 900, 300), (1500, 1400, 700), (2048, 600, 200), (1777, 1100, 0)):
        m, k = workloads.random_chain(rng, 1, s)
        dt = 0.01 / workloads.chain_omega_max(m, k)
        x0 = rng.normal(0, 0.1, s).astype(np.float32)
        v0 = (rng.normal(0, 1.0, s) * 0.01 / dt[0]).astype(np.float32)
        reqs.append((m[0], k[0], dt, x0, v0, nsteps, stride))
    with osc.Server(max_slots=16, chunk_us=300) as srv:
        tickets = [srv.submit("chain", method, "f32", *r) for r in reqs]
        mixed = [srv.wait(t, timeout=120.0) for t in tickets]
    for r, res in zip(reqs, mixed):
        m, k, dt, x0, v0, nsteps, stride = r
        rx, rv, rxe, rve = oracle.chain(method, m[None], k[None], dt, x0[None].astype(np.float64),
                                        v0[None].astype(np.float64), nsteps, stride)
        assert oracle.rel_traj_err(res["x_end"][None], rxe)[0] < 1e-5
        assert oracle.rel_traj_err(res["v_end"][None], rve)[0] < 1e-5
        if stride:
            assert oracle.rel_traj_err(res["x_frames"][:, None, :], rx)[0] < 1e-5
            assert oracle.rel_traj_err(res["v_frames"][:, None, :], rv)[0] < 1e-5
    for r, res in zip(reqs, mixed):
        with osc.Server(max_slots=4, chunk_us=300) as srv:
            alone = srv.wait(srv.submit("chain", method, "f32", *r), timeout=120.0)
        for key in ("x_end", "v_end"):
            np.testing.assert_array_equal(alone[key], res[key])


def test_full_stream_sampled_parity():
    """The served stream at its full size (200 requests, s up to 2048, up to
    1e5 steps, all submitted at once), in the server configuration bench.py
    times; a sample of requests the oracle can integrate in seconds (the
    cheapest chains and dense systems, the longest chain and the cheapest
    dense system of s > 256 within that budget) is compared frame by frame
    at the FP32 tolerance."""
    reqs = workloads.c5_request_stream(n_requests=200, qps=1e6)
    with osc.Server(max_slots=64) as srv:
        tickets = [_submit(srv, r) for r in reqs]
        results = [srv.wait(t, timeout=300.0) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    cost = lambda r: r.system.s * r.system.nsteps * (r.system.s if r.kind == "dense" else 8)
    chains = sorted((r for r in reqs if r.kind == "chain"), key=cost)
    dense = sorted((r for r in reqs if r.kind == "dense"), key=cost)
    longest = max((r for r in chains if cost(r) <= 4e9), key=lambda r: r.system.s)
    large = [r for r in dense if r.system.s > 256 and cost(r) <= 4e9][:1]   # the split path
    sample = {r.rid: r for r in chains[:3] + dense[:2] + [longest] + large}
    for rid, r in sample.items():
        res = results[rid]
        rx, rv = _oracle(r)
        ex = oracle.rel_traj_err(res["x_frames"][:, None, :], rx[:, None, :])[0]
        ev = oracle.rel_traj_err(res["v_frames"][:, None, :], rv[:, None, :])[0]
        assert ex < 1e-5 and ev < 1e-5, (r.kind, r.system.s, r.system.nsteps, ex, ev)


def test_mixed_precisions_in_one_iteration():
    """FP32 and FP64 requests of both kinds served together: their work lists
    share one upload per iteration.  Each result matches the oracle at its
    precision's tolerance and is bitwise the same as the request served
    alone."""
    reqs = _stream(16, seed=23, s_max=300, nsteps=(300, 2000))
    precs = ["f64" if i % 2 else "f32" for i in range(len(reqs))]

    def submit(srv, r, prec):
        w = r.system
        if r.kind == "chain":
            return srv.submit("chain", "rk4", prec, w.m[0], w.k[0], w.dt, w.x0[0], w.v0[0], w.nsteps,
                              w.out_stride)
        return srv.submit("dense", "rk4", prec, w.M, w.K, w.dt, w.x0[0], w.v0[0], w.nsteps, w.out_stride)

    with osc.Server(max_slots=64, chunk_us=300) as srv:
        tickets = [submit(srv, r, p) for r, p in zip(reqs, precs)]
        mixed = [srv.wait(t, timeout=120.0) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert {r.kind for r, p in zip(reqs, precs) if p == "f64"} == {"chain", "dense"}
    for r, p, res in zip(reqs, precs, mixed):
        w = r.system
        x0, v0 = w.x0, w.v0
        if p == "f32":
            x0 = x0.astype(np.float32).astype(np.float64)
            v0 = v0.astype(np.float32).astype(np.float64)
        if r.kind == "chain":
            rx, rv, _, _ = oracle.chain("rk4", w.m, w.k, w.dt, x0, v0, w.nsteps, w.out_stride)
        else:
            rx, rv, _, _ = oracle.dense("rk4", w.M, w.K, w.dt, x0, v0, w.nsteps, w.out_stride)
        tol = 1e-10 if p == "f64" else 1e-5
        ex = oracle.rel_traj_err(res["x_frames"][:, None, :], rx)[0]
        ev = oracle.rel_traj_err(res["v_frames"][:, None, :], rv)[0]
        assert ex < tol and ev < tol, (r.kind, p, w.s, ex, ev)
    for i in range(len(reqs)):
        with osc.Server(max_slots=4, chunk_us=300) as srv:
            alone = srv.wait(submit(srv, reqs[i], precs[i]), timeout=120.0)
        for key in ("x_frames", "v_frames", "x_end", "v_end"):
            np.testing.assert_array_equal(alone[key], mixed[i][key])


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_frame_jumps_serve_large_dense_requests(method):
    """With frame jumps on, a dense request whose frames are far cheaper by
    powers of its one-step matrix is served that way (the scheme's own
    trajectory at the frames, in FP64); the others are stepped as before.
    Every result matches the oracle, and the jump-served one is bitwise the
    same alone and in a mix."""
    rng = np.random.default_rng(4242)
    M, K = workloads.random_dense_system(rng, 300)
    dt = np.array([0.01 / workloads.dense_omega_max(M, K)])
    big = workloads.DenseBatch(M, K, dt, rng.normal(0, 1, (1, 300)), rng.normal(0, 0.01, (1, 300)), 3000, 500,
                               True)
    Ms, Ks = workloads.random_dense_system(rng, 8)
    dts = np.array([0.01 / workloads.dense_omega_max(Ms, Ks)])
    small = workloads.DenseBatch(Ms, Ks, dts, rng.normal(0, 1, (1, 8)), rng.normal(0, 0.01, (1, 8)), 400, 100,
                                 True)
    chain = _stream(1, seed=77, s_max=64)[0]
    reqs = [workloads.Request(0, 0.0, "dense", big), workloads.Request(1, 0.0, "dense", small), chain]
    with osc.Server(max_slots=8, chunk_us=500, frame_jumps=True) as srv:
        mixed = [srv.wait(_submit(srv, r, method), timeout=120.0) for r in reqs]
        st = srv.stats()
    assert st["completed"] == 3 and st["failed"] == 0
    assert [res["frame_jumps"] for res in mixed] == [True, False, False]
    assert mixed[0]["iterations"] == 0
    for r, res in zip(reqs, mixed):
        rx, rv = _oracle(r, method)
        ex = oracle.rel_traj_err(res["x_frames"][:, None, :], rx[:, None, :])[0]
        ev = oracle.rel_traj_err(res["v_frames"][:, None, :], rv[:, None, :])[0]
        assert ex < 1e-5 and ev < 1e-5, (r.kind, r.system.s, ex, ev)
        if r.system.nsteps % r.system.out_stride == 0:       # the last frame is the end state
            np.testing.assert_array_equal(res["x_frames"][-1], res["x_end"])
    with osc.Server(max_slots=2, frame_jumps=True) as srv:
        alone = srv.wait(_submit(srv, reqs[0], method), timeout=120.0)
    for key in ("x_frames", "v_frames", "x_end", "v_end"):
        np.testing.assert_array_equal(alone[key], mixed[0][key])
    with osc.Server(max_slots=2) as srv:               # off: the same request is stepped
        stepped = srv.wait(_submit(srv, reqs[0], method), timeout=120.0)
    assert not stepped["frame_jumps"] and stepped["iterations"] > 0
    assert mixed[0]["bytes"] > stepped["bytes"]        # the jump temporaries are accounted
    # a budget that holds the stepped request but not the jump temporaries:
    # the request is stepped, not refused
    with osc.Server(max_slots=2, frame_jumps=True, hbm_budget=stepped["bytes"]) as srv:
        tight = srv.wait(_submit(srv, reqs[0], method), timeout=120.0)
    assert not tight["frame_jumps"]
    for key in ("x_frames", "v_frames", "x_end", "v_end"):
        np.testing.assert_array_equal(tight[key], stepped[key])
