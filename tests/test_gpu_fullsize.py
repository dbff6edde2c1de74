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


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_spring_chain_full(method):
    """4096 chains of 1024 DOFs, 1e5 steps; three sampled instances."""
    import torch
    from paper_1702_02207_amd import osc
    w = workloads.c3_spring_chain()
    w.out_stride = w.nsteps
    xf, vf, xe, ve = gpu_chain(method, "f32", w)
    idx = _sample(w.batch, 3, 12)
    sub = w.subset(idx)
    x0, v0 = f32_inputs(sub)
    rx, rv, _, _ = oracle.chain(method, sub.m, sub.k, sub.dt, x0, v0, w.nsteps, w.out_stride)
    _check(xf[:, idx], rx, f"chain {method} x")
    _check(vf[:, idx], rv, f"chain {method} v")
    assert np.isfinite(xe).all() and np.isfinite(ve).all()
    # FP64 energy of the whole final GPU state: the GPU's energy kernel against
    # the oracle's on the same (sampled) states, and conservation against the
    # initial energy
    sysm = osc.System("chain", method, "f32", w.m, w.k, w.dt).create()
    try:
        E = sysm.energy(torch.as_tensor(xe, dtype=torch.float32, device="cuda"),
                        torch.as_tensor(ve, dtype=torch.float32, device="cuda")).cpu().numpy()
        sysm.sync()
    finally:
        sysm.close()
    np.testing.assert_allclose(E[idx], oracle.energy_chain(sub.m, sub.k, xe[idx], ve[idx]), rtol=1e-12)
    E0 = oracle.energy_chain(sub.m, sub.k, x0, v0)
    assert np.all(np.abs(E[idx] - E0) <= 1e-4 * E0)


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_dense_shared_full(method):
    """s = 256, one A shared by 8192 instances, 1e4 steps on the MFMA path;
    four sampled instances."""
    w = workloads.c4_dense_shared()
    w.out_stride = w.nsteps
    xf, vf, xe, ve = gpu_dense(method, "f32", w)
    idx = _sample(w.batch, 4, 13)
    x0, v0 = f32_inputs(w)
    rx, rv, _, _ = oracle.dense(method, w.M, w.K, w.dt, x0[idx], v0[idx], w.nsteps, w.out_stride, shared=True)
    _check(xf[:, idx], rx, f"dense {method} x")
    _check(vf[:, idx], rv, f"dense {method} v")
    assert np.isfinite(xe).all() and np.isfinite(ve).all()
