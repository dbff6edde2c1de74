"""GPU parity of dense eq. (1) systems (A = M^-1 K by FP64 Cholesky on the
GPU) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_1702_02207_amd import workloads
from gpu_util import gpu_dense, oracle_dense, f32_inputs

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
TOL_F64 = 1e-10


def _err(got, ref):
    return oracle.rel_traj_err(got, ref)


def _dense_batch(seed, s, batch, nsteps, stride, shared=True, vscale=0.0):
    rng = np.random.default_rng(seed)
    if shared:
        M, K = workloads.random_dense_system(rng, s)
        dt = np.array([0.01 / workloads.dense_omega_max(M, K)])
    else:
        Ms, Ks = zip(*[workloads.random_dense_system(rng, s) for _ in range(batch)])
        M, K = np.array(Ms), np.array(Ks)
        dt = np.array([0.01 / workloads.dense_omega_max(M[b], K[b]) for b in range(batch)])
    x0 = rng.normal(0, 1, (batch, s))
    v0 = rng.normal(0, 1, (batch, s)) * vscale
    return workloads.DenseBatch(M, K, dt, x0, v0, nsteps, stride, shared)


def test_operator_matches_oracle_cholesky():
    import torch
    from paper_1702_02207_amd import osc
    for s in (1, 2, 7, 64, 200):
        w = _dense_batch(40 + s, s, 2, 10, 0)
        sysm = osc.System("dense", "rk4", "f64", w.M, w.K, w.dt, shared=True, batch=2).create()
        A = sysm.dense_operator().cpu().numpy()[0]
        sysm.sync()
        sysm.close()
        ref = oracle.form_a(w.M, w.K)
        assert np.abs(A - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("s,batch", [(1, 3), (2, 5), (9, 4), (64, 3), (100, 2), (257, 2)])
def test_dense_shared(method, prec, s, batch):
    w = _dense_batch(100 + s, s, batch, 2000, 250, vscale=0.01)
    xf, vf, xe, ve = gpu_dense(method, prec, w)
    x0, v0 = f32_inputs(w) if prec == "f32" else (w.x0, w.v0)
    rx, rv, rxe, rve = oracle_dense(method, w, x0=x0, v0=v0)
    tol = TOL_F32 if prec == "f32" else TOL_F64
    assert _err(xf, rx).max() < tol
    assert _err(vf, rv).max() < tol
    assert _err(xe, rxe).max() < tol


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_dense_per_instance(method, prec):
    w = _dense_batch(7, 33, 4, 1500, 500, shared=False, vscale=0.01)
    xf, vf, xe, ve = gpu_dense(method, prec, w)
    x0, v0 = f32_inputs(w) if prec == "f32" else (w.x0, w.v0)
    rx, rv, _, _ = oracle_dense(method, w, x0=x0, v0=v0)
    tol = TOL_F32 if prec == "f32" else TOL_F64
    assert _err(xf, rx).max() < tol
    assert _err(vf, rv).max() < tol


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_dense_energy(prec):
    import torch
    from paper_1702_02207_amd import osc
    w = _dense_batch(9, 50, 6, 10, 0, vscale=1.0)
    sysm = osc.System("dense", "verlet", prec, w.M, w.K, w.dt, shared=True, batch=6).create()
    tdt = torch.float32 if prec == "f32" else torch.float64
    x = torch.as_tensor(w.x0, dtype=tdt, device="cuda")
    v = torch.as_tensor(w.v0, dtype=tdt, device="cuda")
    E = sysm.energy(x, v).cpu().numpy()
    sysm.sync()
    sysm.close()
    ref = oracle.energy_dense(w.M, w.K, x.double().cpu().numpy(), v.double().cpu().numpy())
    np.testing.assert_allclose(E, ref, rtol=1e-12)


def test_dense_rejects_non_spd_and_unstable():
    from paper_1702_02207_amd import osc
    M = np.array([[1.0, 2.0], [2.0, 1.0]])
    K = np.eye(2)
    with pytest.raises(osc.OscError) as e:
        osc.System("dense", "rk4", "f32", M, K, [1e-3], shared=True, batch=1).create()
    assert e.value.status == osc.OSC_ENOTSPD
    # SPD system, omega_max = 10: dt = 0.5 gives h omega = 5 (unstable); dt = 0.25 gives 2.5,
    # stable for RK4 (limit 2.78 after the 2 % margin) but not for Verlet (limit 1.99)
    M, K = np.eye(3), np.diag([1.0, 25.0, 100.0])
    with pytest.raises(osc.OscError) as e:
        osc.System("dense", "rk4", "f32", M, K, [0.5], shared=True, batch=1).create()
    assert e.value.status == osc.OSC_EUNSTABLE
    osc.System("dense", "rk4", "f32", M, K, [0.25], shared=True, batch=1).create().close()
    with pytest.raises(osc.OscError) as e:
        osc.System("dense", "verlet", "f32", M, K, [0.25], shared=True, batch=1).create()
    assert e.value.status == osc.OSC_EUNSTABLE
