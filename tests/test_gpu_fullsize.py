"""GPU parity at the benchmark sizes, in the launch configuration bench.py
times: the whole batch runs on the GPU, and a seeded sample of instances
(always including the first and the last, which sit at the edges of the
launch grid) is integrated by the FP64 oracle and compared element by
element.  Tolerance: the FP32 target 1e-5 on the relative trajectory error
(max over frames and DOFs of |gpu - oracle| / max |oracle|)."""
import numpy as np
import pytest

import oracle
from paper_1702_02207_amd import workloads
from gpu_util import gpu_chain, gpu_dense, f32_inputs

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


def _sample(batch, n, seed):
    rng = np.random.default_rng(seed)
    mid = rng.choice(np.arange(1, batch - 1), size=n - 2, replace=False)
    return np.unique(np.concatenate([[0, batch - 1], mid]))


def _check(got, ref, what):
    e = oracle.rel_traj_err(got, ref)
    print(f"{what}: max {e.max():.3e} median {np.median(e):.3e}")
    assert e.max() < TOL_F32, what


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_two_mass_ensemble_full(method):
    """2^20 two-mass instances, 1e4 steps, frames at 0 and 1e4."""
    w = workloads.c2_two_dof_ensemble()
    w.out_stride = w.nsteps
    xf, vf, xe, ve = gpu_chain(method, "f32", w)
    idx = _sample(w.batch, 512, 11)
    sub = w.subset(idx)
    x0, v0 = f32_inputs(sub)
    rx, rv, _, _ = oracle.chain(method, sub.m, sub.k, sub.dt, x0, v0, w.nsteps, w.out_stride)
    _check(xf[:, idx], rx, f"two-mass {method} x")
    _check(vf[:, idx], rv, f"two-mass {method} v")
    np.testing.assert_array_equal(xf[-1], xe)
    assert np.isfinite(xe).all() and np.isfinite(ve).all()
    from paper_1702_02207_amd import osc
    sysm = osc.System("chain", method, "f32", w.m, w.k, w.dt).create()
    try:
        inv = _invariant(sysm, method, xe, ve)
    finally:
        sysm.close()
    X0, V0 = f32_inputs(w)
    inv0 = (oracle.energy_chain(w.m, w.k, X0, V0) if method == "rk4"
            else oracle.verlet_q_chain(w.m, w.k, w.dt, X0, V0))
    drift = np.abs(inv - inv0) / inv0
    print(f"two-mass {method}: invariant drift max {drift.max():.3e} p99 {np.percentile(drift, 99):.3e}")
    assert drift.max() <= 1e-6


def _invariant(sysm, method, x, v):
    """FP64 invariant of a GPU state from the library: E for RK4, the exact
    discrete invariant Q for Verlet."""
    import torch
    xt = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    vt = torch.as_tensor(v, dtype=torch.float32, device="cuda")
    out = sysm.energy(xt, vt, shadow=(method == "verlet")).cpu().numpy()
    sysm.sync()
    return out


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_spring_chain_full(method):
    """4096 chains of 1024 DOFs, 1e5 steps.  32 instances spread over the
    grid (first and last included) against the oracle element by element;
    every instance's FP64 invariant (E for RK4, Q for Verlet) at the end
    against its initial value: relative drift <= 1e-6."""
    from paper_1702_02207_amd import osc
    w = workloads.c3_spring_chain()
    w.out_stride = w.nsteps
    xf, vf, xe, ve = gpu_chain(method, "f32", w)
    idx = _sample(w.batch, 32, 12)
    sub = w.subset(idx)
    x0, v0 = f32_inputs(sub)
    rx, rv, _, _ = oracle.chain(method, sub.m, sub.k, sub.dt, x0, v0, w.nsteps, w.out_stride)
    _check(xf[:, idx], rx, f"chain {method} x")
    _check(vf[:, idx], rv, f"chain {method} v")
    assert np.isfinite(xe).all() and np.isfinite(ve).all()
    sysm = osc.System("chain", method, "f32", w.m, w.k, w.dt).create()
    try:
        inv = _invariant(sysm, method, xe, ve)
    finally:
        sysm.close()
    # the library's FP64 invariant of these states against the oracle's
    ref_fn = oracle.energy_chain if method == "rk4" else (
        lambda m, k, x, v: oracle.verlet_q_chain(m, k, sub.dt, x, v))
    np.testing.assert_allclose(inv[idx], ref_fn(sub.m, sub.k, xe[idx], ve[idx]), rtol=1e-11)
    X0, V0 = f32_inputs(w)
    inv0 = (oracle.energy_chain(w.m, w.k, X0, V0) if method == "rk4"
            else oracle.verlet_q_chain(w.m, w.k, w.dt, X0, V0))
    drift = np.abs(inv - inv0) / inv0
    print(f"chain {method}: invariant drift max {drift.max():.3e} p99 {np.percentile(drift, 99):.3e}")
    assert drift.max() <= 1e-6


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_dense_shared_full(method):
    """s = 256, one A shared by 8192 instances, 1e4 steps on the MFMA path;
    256 instances spread over the grid against the oracle; every instance's
    FP64 invariant (E for RK4, Q for Verlet) drifts by <= 1e-6."""
    from paper_1702_02207_amd import osc
    w = workloads.c4_dense_shared()
    w.out_stride = w.nsteps
    xf, vf, xe, ve = gpu_dense(method, "f32", w)
    idx = _sample(w.batch, 256, 13)
    x0, v0 = f32_inputs(w)
    rx, rv, _, _ = oracle.dense(method, w.M, w.K, w.dt, x0[idx], v0[idx], w.nsteps, w.out_stride, shared=True)
    _check(xf[:, idx], rx, f"dense {method} x")
    _check(vf[:, idx], rv, f"dense {method} v")
    assert np.isfinite(xe).all() and np.isfinite(ve).all()
    sysm = osc.System("dense", method, "f32", w.M, w.K, w.dt, shared=True, batch=w.batch).create()
    try:
        inv = _invariant(sysm, method, xe, ve)
    finally:
        sysm.close()
    if method == "rk4":
        inv0 = oracle.energy_dense(w.M, w.K, x0, v0)
        ref = oracle.energy_dense(w.M, w.K, xe[idx], ve[idx])
    else:
        inv0 = oracle.verlet_q_dense(w.M, w.K, w.dt, x0, v0)
        ref = oracle.verlet_q_dense(w.M, w.K, w.dt, xe[idx], ve[idx])
    np.testing.assert_allclose(inv[idx], ref, rtol=1e-11)
    drift = np.abs(inv - inv0) / inv0
    print(f"dense {method}: invariant drift max {drift.max():.3e} p99 {np.percentile(drift, 99):.3e}")
    assert drift.max() <= 1e-6
