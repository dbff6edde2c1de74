"""Real-time periodic stepping (osc_rt_*) through the C ABI: the states after
the ticks are bit for bit the frames of one osc_integrate call (and match the
oracle / the closed form), for every supported path; the periodic loop
reports its latencies."""
import numpy as np
import pytest

import oracle
from oracle import closed_form as cf
from paper_1702_02207_amd import osc, workloads
from gpu_util import to_dev, f32_inputs

pytestmark = pytest.mark.gpu


def _integrate_frames(sysm, x0, v0, nticks, k):
    xf, vf, _, _ = sysm.integrate(x0, v0, nticks * k, k)
    sysm.sync()
    return xf[1:].cpu().numpy(), vf[1:].cpu().numpy()


def _ticks(rt, nticks):
    xs, vs = [], []
    for _ in range(nticks):
        x, v = rt.tick()
        xs.append(x.clone())
        vs.append(v.clone())
    rt.system.sync()
    import torch
    return torch.stack(xs).cpu().numpy(), torch.stack(vs).cpu().numpy()


def test_periodic_loop_on_the_paper_system():
    """The paper's two-mass system (eq. (3), FP64), one step per period: the
    periodic trajectory equals osc_integrate bit for bit and the closed-form
    normal-mode solution within 1e-10; the loop reports its latencies."""
    import torch
    w = workloads.c1_paper_two_mass(nsteps=2000, out_stride=1)
    sysm = osc.System("chain", "rk4", "f64", w.m, w.k, w.dt).create()
    x0, v0 = to_dev(w.x0, torch.float64), to_dev(w.v0, torch.float64)
    try:
        ref_x, ref_v = _integrate_frames(sysm, x0, v0, 2000, 1)
        with osc.Realtime(sysm, x0, v0, 1) as rt:
            xf, vf, lat, stats = rt.run(50e-6, 2000)
            assert rt.steps == 2000
            xf, vf = xf.cpu().numpy(), vf.cpu().numpy()
    finally:
        sysm.close()
    np.testing.assert_array_equal(xf, ref_x)
    np.testing.assert_array_equal(vf, ref_v)
    t = np.arange(1, 2001) * w.dt[0]
    xr, vr = cf.two_mass_equal(t, 2.0, 2025.0, w.x0[0], w.v0[0])
    assert oracle.rel_traj_err(xf, xr[:, None, :])[0] < 1e-10
    assert oracle.rel_traj_err(vf, vr[:, None, :])[0] < 1e-10
    assert stats["ticks"] == 2000 and len(lat) == 2000
    assert np.all(lat > 0) and stats["gpu_p50_s"] > 0
    print(f"paper system, 50 us period: latency p50 {stats['p50_s'] * 1e6:.1f} us, "
          f"p99 {stats['p99_s'] * 1e6:.1f} us, max {stats['max_s'] * 1e6:.1f} us, "
          f"jitter {stats['jitter_s'] * 1e6:.2f} us, missed {stats['missed']}, "
          f"gpu {stats['gpu_p50_s'] * 1e6:.1f} us")


def test_periodic_loop_meets_a_1ms_period():
    import torch
    w = workloads.c1_paper_two_mass(nsteps=10, out_stride=1)
    sysm = osc.System("chain", "rk4", "f64", w.m, w.k, w.dt).create()
    try:
        with osc.Realtime(sysm, to_dev(w.x0, torch.float64), to_dev(w.v0, torch.float64), 10) as rt:
            _, _, lat, stats = rt.run(1e-3, 300, frames=False)
    finally:
        sysm.close()
    print(f"1 ms period: p50 {stats['p50_s'] * 1e6:.1f} us p99 {stats['p99_s'] * 1e6:.1f} us "
          f"missed {stats['missed']}")
    assert stats["p50_s"] < 1e-3
    assert stats["missed"] <= 3


def _chain(seed, batch, s):
    rng = np.random.default_rng(seed)
    m, k = workloads.random_chain(rng, batch, s)
    dt = 0.01 / workloads.chain_omega_max(m, k)
    return m, k, dt, rng.normal(0, 0.1, (batch, s)), rng.normal(0, 1, (batch, s)) * 0.05


@pytest.mark.parametrize("case", ["chain_f32", "chain_verlet", "chain_long", "dense_mfma", "dense_f64", "driven",
                                  "per_step_propagator"])
def test_ticks_are_the_frames_of_one_integration(case):
    import torch
    k, nticks = 7, 40
    if case.startswith("chain") or case in ("driven", "per_step_propagator"):
        s = {"chain_long": 1024, "per_step_propagator": 2}.get(case, 8)
        m, kk, dt, x0, v0 = _chain(1000 + len(case), 6, s)
        method = "verlet" if case == "chain_verlet" else "rk4"
        sysm = osc.System("chain", method, "f32", m, kk, dt).create()
        if case == "driven":
            rng = np.random.default_rng(1001)
            sysm.set_excitation(0.2, 1e-4, rng.normal(size=(6, s)) * 10.0, rng.uniform(5, 20, 6))
        if case == "per_step_propagator":
            sysm.set_config(osc.CFG_PROPAGATOR, 2)
        dtype = torch.float32
    else:
        rng = np.random.default_rng(1002)
        M, K = workloads.random_dense_system(rng, 40)
        dt = np.array([0.01 / workloads.dense_omega_max(M, K)])
        prec = "f32" if case == "dense_mfma" else "f64"
        sysm = osc.System("dense", "rk4", prec, M, K, dt, shared=True, batch=20).create()
        x0, v0 = rng.normal(size=(20, 40)), rng.normal(size=(20, 40)) * 0.01
        dtype = torch.float32 if prec == "f32" else torch.float64
    X0, V0 = to_dev(x0, dtype), to_dev(v0, dtype)
    try:
        ref_x, ref_v = _integrate_frames(sysm, X0, V0, nticks, k)
        with osc.Realtime(sysm, X0, V0, k) as rt:
            xf, vf = _ticks(rt, nticks)
    finally:
        sysm.close()
    np.testing.assert_array_equal(xf, ref_x)
    np.testing.assert_array_equal(vf, ref_v)


def test_realtime_rejects_unsupported_paths():
    import torch
    rng = np.random.default_rng(1010)
    M, K = workloads.random_dense_system(rng, 300)
    dt = np.array([0.01 / workloads.dense_omega_max(M, K)])
    sysm = osc.System("dense", "rk4", "f32", M, K, dt, shared=True, batch=1).create()   # split path
    x0 = to_dev(rng.normal(size=(1, 300)), torch.float32)
    try:
        with pytest.raises(osc.OscError) as e:
            osc.Realtime(sysm, x0, x0, 1)
        assert e.value.status == osc.OSC_ENOTSUP
    finally:
        sysm.close()
    m, k, dt, x0, v0 = _chain(1011, 2, 2)
    sysm = osc.System("chain", "rk4", "f32", m, k, dt).create()
    X0 = to_dev(x0, torch.float32)
    try:
        with pytest.raises(ValueError):
            osc.Realtime(sysm, X0, X0, 0)
        sysm.set_config(osc.CFG_PROPAGATOR, 1)
        with pytest.raises(osc.OscError) as e:
            osc.Realtime(sysm, X0, X0, 1)
        assert e.value.status == osc.OSC_ENOTSUP
    finally:
        sysm.close()


@pytest.mark.parametrize("case", ["chain_f32", "chain_verlet", "chain_long", "chain_f64", "two_wave_chain",
                                  "driven", "driven_long_f64"])
def test_resident_ticks_are_the_frames_of_one_integration(case):
    """osc_rt_run_resident: one kernel stays on the device and advances one
    tick per release; its frames are bit for bit those of osc_integrate, also
    when launch-mode ticks come before and after it."""
    import torch
    k, n_before, n_res, n_after = 5, 3, 30, 2
    s = {"chain_long": 1024, "two_wave_chain": 1500, "driven_long_f64": 1000}.get(case, 8)
    m, kk, dt, x0, v0 = _chain(2000 + len(case), 6, s)
    method = "verlet" if case == "chain_verlet" else "rk4"
    prec = "f64" if case in ("chain_f64", "driven_long_f64") else "f32"
    dtype = torch.float64 if prec == "f64" else torch.float32
    sysm = osc.System("chain", method, prec, m, kk, dt).create()
    if case.startswith("driven"):
        rng = np.random.default_rng(2003)
        sysm.set_excitation(0.2, 1e-4, rng.normal(size=(6, s)) * 10.0, rng.uniform(5, 20, 6))
    X0, V0 = to_dev(x0, dtype), to_dev(v0, dtype)
    try:
        total = n_before + n_res + n_after
        ref_x, ref_v = _integrate_frames(sysm, X0, V0, total, k)
        with osc.Realtime(sysm, X0, V0, k) as rt:
            bx, bv = _ticks(rt, n_before)
            xf, vf, lat, stats = rt.run_resident(200e-6, n_res)
            assert rt.steps == (n_before + n_res) * k
            ax, av = _ticks(rt, n_after)
            xf, vf = xf.cpu().numpy(), vf.cpu().numpy()
    finally:
        sysm.close()
    got_x = np.concatenate([bx, xf, ax])
    got_v = np.concatenate([bv, vf, av])
    np.testing.assert_array_equal(got_x, ref_x)
    np.testing.assert_array_equal(got_v, ref_v)
    assert stats["ticks"] == n_res and len(lat) == n_res and np.all(lat > 0)


def test_resident_loop_on_the_paper_system():
    """The paper's two-mass system (eq. (3), FP64), one step per 50 us period in
    the resident mode: the trajectory equals osc_integrate bit for bit and
    the closed-form normal-mode solution within 1e-10."""
    import torch
    w = workloads.c1_paper_two_mass(nsteps=2000, out_stride=1)
    sysm = osc.System("chain", "rk4", "f64", w.m, w.k, w.dt).create()
    x0, v0 = to_dev(w.x0, torch.float64), to_dev(w.v0, torch.float64)
    try:
        ref_x, ref_v = _integrate_frames(sysm, x0, v0, 2000, 1)
        with osc.Realtime(sysm, x0, v0, 1) as rt:
            _, _, _, launched = rt.run(50e-6, 2000, frames=False)
        with osc.Realtime(sysm, x0, v0, 1) as rt:
            xf, vf, lat, stats = rt.run_resident(50e-6, 2000)
            xf, vf = xf.cpu().numpy(), vf.cpu().numpy()
    finally:
        sysm.close()
    np.testing.assert_array_equal(xf, ref_x)
    np.testing.assert_array_equal(vf, ref_v)
    t = np.arange(1, 2001) * w.dt[0]
    xr, vr = cf.two_mass_equal(t, 2.0, 2025.0, w.x0[0], w.v0[0])
    assert oracle.rel_traj_err(xf, xr[:, None, :])[0] < 1e-10
    assert stats["ticks"] == 2000 and np.all(lat > 0)
    print(f"paper system, 50 us period: resident p50 {stats['p50_s'] * 1e6:.1f} us p99 {stats['p99_s'] * 1e6:.1f} us "
          f"missed {stats['missed']}; one launch per tick p50 {launched['p50_s'] * 1e6:.1f} us "
          f"p99 {launched['p99_s'] * 1e6:.1f} us missed {launched['missed']}")


def test_resident_rejects_unsupported_handles():
    import torch
    rng = np.random.default_rng(2010)
    M, K = workloads.random_dense_system(rng, 40)
    dt = np.array([0.01 / workloads.dense_omega_max(M, K)])
    sysm = osc.System("dense", "rk4", "f32", M, K, dt, shared=True, batch=4).create()
    x0 = to_dev(rng.normal(size=(4, 40)), torch.float32)
    try:
        with osc.Realtime(sysm, x0, x0, 1) as rt:
            with pytest.raises(osc.OscError) as e:
                rt.run_resident(1e-3, 2)
            assert e.value.status == osc.OSC_ENOTSUP
    finally:
        sysm.close()
    # damped chains on the one-workgroup-per-instance kernel
    m, k, dt, x0, v0 = _chain(2011, 4, 8)
    sysm = osc.System("chain", "rk4", "f32", m, k, dt).create()
    X0 = to_dev(x0, torch.float32)
    try:
        sysm.set_excitation(0.1, 0.0, None)
        sysm.set_config(osc.CFG_DENSE_KERNEL, 1)
        with osc.Realtime(sysm, X0, X0, 1) as rt:
            with pytest.raises(osc.OscError) as e:
                rt.run_resident(1e-3, 2)
            assert e.value.status == osc.OSC_ENOTSUP
    finally:
        sysm.close()
    # more workgroups than the device holds at once: refused before any launch
    w = workloads.c2_two_dof_ensemble(batch=1 << 20, nsteps=10)
    sysm = osc.System("chain", "rk4", "f32", w.m, w.k, w.dt).create()
    X0 = to_dev(w.x0, torch.float32)
    try:
        with osc.Realtime(sysm, X0, X0, 1) as rt:
            with pytest.raises(osc.OscError) as e:
                rt.run_resident(1e-3, 2)
            assert e.value.status == osc.OSC_ENOTSUP
            rt.tick()   # the stepper is unharmed
    finally:
        sysm.close()


def test_resident_idle_limit_ends_the_kernel():
    """A release that comes later than the idle limit: every workgroup gives
    up and the kernel ends on its own; the call reports OSC_ETIMEOUT, the
    stepper refuses further use, and a new stepper runs normally."""
    import torch
    m, k, dt, x0, v0 = _chain(2012, 6, 8)
    sysm = osc.System("chain", "rk4", "f32", m, k, dt).create()
    X0, V0 = to_dev(x0, torch.float32), to_dev(v0, torch.float32)
    try:
        with osc.Realtime(sysm, X0, V0, 3) as rt:
            rt.set_idle_limit(1e-3)
            with pytest.raises(osc.OscError) as e:
                rt.run_resident(50e-3, 3)
            assert e.value.status == osc.OSC_ETIMEOUT
            with pytest.raises(osc.OscError) as e:
                rt.tick()
            assert e.value.status == osc.OSC_EDEVICE
        ref_x, _ = _integrate_frames(sysm, X0, V0, 4, 3)
        with osc.Realtime(sysm, X0, V0, 3) as rt:
            xf, _, _, _ = rt.run_resident(1e-3, 4)
            np.testing.assert_array_equal(xf.cpu().numpy(), ref_x)
    finally:
        sysm.close()
