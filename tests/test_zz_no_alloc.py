"""The allocation-free entry point osc_integrate_static, through the C ABI:
bit for bit the same results as osc_integrate on the same handle and
configuration (and within the FP32 tolerance of the FP64 oracle), on two
calls in a row with the second one smaller, for every path that needs device
scratch (chunked chains, chunked dense MFMA, the split dense path), plus its
error returns."""
import numpy as np
import pytest

import oracle
from paper_1702_02207_amd import osc, workloads
from gpu_util import to_dev, f32_inputs

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


def _chain(seed, batch, s, nsteps, stride):
    rng = np.random.default_rng(seed)
    m, k = workloads.random_chain(rng, batch, s)
    dt = 0.01 / workloads.chain_omega_max(m, k)
    x0 = rng.normal(0.0, 0.1, (batch, s))
    v0 = rng.normal(0.0, 1.0, (batch, s)) * 0.05
    return workloads.ChainBatch(m, k, dt, x0, v0, nsteps, stride)


def _dense(seed, batch, s, nsteps, stride):
    rng = np.random.default_rng(seed)
    M, K = workloads.random_dense_system(rng, s)
    dt = np.array([0.01 / workloads.dense_omega_max(M, K)])
    x0 = rng.normal(0.0, 1.0, (batch, s))
    v0 = rng.normal(0.0, 1.0, (batch, s)) * 0.01
    return workloads.DenseBatch(M, K, dt, x0, v0, nsteps, stride, True)


def _both(sysm, w, config):
    """The same run through osc_integrate and osc_integrate_static."""
    import torch
    for key, value in config:
        sysm.set_config(key, value)
    x0, v0 = to_dev(w.x0, torch.float32), to_dev(w.v0, torch.float32)
    ref = sysm.integrate(x0, v0, w.nsteps, w.out_stride)
    got = sysm.integrate(x0, v0, w.nsteps, w.out_stride, static=True)
    sysm.sync()
    cv = lambda ts: [t.double().cpu().numpy() for t in ts]
    return cv(ref), cv(got)


def _check(ref, got, oracle_out, label):
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b, err_msg=label)
    rx, rv = oracle_out
    ex = oracle.rel_traj_err(got[0], rx).max()
    ev = oracle.rel_traj_err(got[1], rv).max()
    print(f"{label}: static == osc_integrate bitwise; vs oracle x {ex:.2e} v {ev:.2e}")
    assert ex < TOL_F32 and ev < TOL_F32, (label, ex, ev)


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_static_chain_chunked_two_calls(method):
    """Chunked chains (the compensated state between launches lives in the
    static scratch): a large call, then a smaller one."""
    for w in (_chain(501, 48, 300, 2000, 500), _chain(502, 16, 100, 1500, 300)):
        sysm = osc.System("chain", method, "f32", w.m, w.k, w.dt).create()
        try:
            ref, got = _both(sysm, w, [(osc.CFG_STEPS_PER_LAUNCH, 700)])
        finally:
            sysm.close()
        x0, v0 = f32_inputs(w)
        rx, rv, _, _ = oracle.chain(method, w.m, w.k, w.dt, x0, v0, w.nsteps, w.out_stride)
        _check(ref, got, (rx, rv), f"chain {method} batch {w.batch} s {w.s}")


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_static_dense_split_two_calls(method):
    """The split dense path (state, carried product, partial sums and step
    counter all in the static scratch; no captured graph) against the
    graph-replayed osc_integrate: a large call, then a smaller one."""
    import torch
    stream = torch.cuda.Stream()   # a non-null stream: osc_integrate replays captured graphs there
    for w in (_dense(511, 2, 512, 300, 100), _dense(512, 1, 300, 200, 50)):
        with torch.cuda.stream(stream):
            sysm = osc.System("dense", method, "f32", w.M, w.K, w.dt, shared=True, batch=w.batch,
                              stream=stream).create()
            try:
                ref, got = _both(sysm, w, [(osc.CFG_DENSE_KERNEL, 3)])
            finally:
                sysm.close()
        torch.cuda.synchronize()
        x0, v0 = f32_inputs(w)
        rx, rv, _, _ = oracle.dense(method, w.M, w.K, w.dt, x0, v0, w.nsteps, w.out_stride, shared=True)
        _check(ref, got, (rx, rv), f"dense split {method} batch {w.batch} s {w.s}")


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_static_dense_mfma_chunked_two_calls(method):
    """Chunked shared-operator MFMA runs (state and per-instance scale in the
    static scratch)."""
    for w in (_dense(521, 40, 64, 250, 50), _dense(522, 8, 20, 120, 40)):
        sysm = osc.System("dense", method, "f32", w.M, w.K, w.dt, shared=True, batch=w.batch).create()
        try:
            ref, got = _both(sysm, w, [(osc.CFG_DENSE_KERNEL, 2), (osc.CFG_STEPS_PER_LAUNCH, 100)])
        finally:
            sysm.close()
        x0, v0 = f32_inputs(w)
        rx, rv, _, _ = oracle.dense(method, w.M, w.K, w.dt, x0, v0, w.nsteps, w.out_stride, shared=True)
        _check(ref, got, (rx, rv), f"dense mfma {method} batch {w.batch} s {w.s}")


def test_static_rejects_runs_beyond_the_scratch():
    """A chunked run whose state exceeds OSC_STATIC_SCRATCH_BYTES is refused
    before any launch, with the size in the message; per-instance dense MFMA
    operators are not supported; an unchunked run needs no scratch."""
    import torch
    batch, s = 2100, 1024           # 4 * 2100 * 1024 doubles = 68.8 MB > 64 MiB
    w = _chain(531, batch, s, 10, 0)
    sysm = osc.System("chain", "rk4", "f64", w.m, w.k, w.dt).create()
    try:
        sysm.set_config(osc.CFG_STEPS_PER_LAUNCH, 4)
        x0, v0 = to_dev(w.x0, torch.float64), to_dev(w.v0, torch.float64)
        with pytest.raises(osc.OscError) as e:
            sysm.integrate(x0, v0, 10, 0, static=True)
        assert e.value.status == osc.OSC_ENOMEM and "maximum" in str(e.value)
        sysm.set_config(osc.CFG_STEPS_PER_LAUNCH, 0)
        ref = sysm.integrate(x0, v0, 10, 0)
        got = sysm.integrate(x0, v0, 10, 0, static=True)
        sysm.sync()
        np.testing.assert_array_equal(ref[2].cpu().numpy(), got[2].cpu().numpy())
    finally:
        sysm.close()
    rng = np.random.default_rng(532)
    Ms, Ks = zip(*[workloads.random_dense_system(rng, 16) for _ in range(3)])
    dts = np.array([0.01 / workloads.dense_omega_max(M, K) for M, K in zip(Ms, Ks)])
    sysm = osc.System("dense", "rk4", "f32", np.array(Ms), np.array(Ks), dts, shared=False, batch=3).create()
    try:
        x0 = to_dev(rng.normal(0, 1, (3, 16)), torch.float32)
        with pytest.raises(osc.OscError) as e:
            sysm.integrate(x0, x0, 10, 0, static=True)
        assert e.value.status == osc.OSC_ENOTSUP
    finally:
        sysm.close()
