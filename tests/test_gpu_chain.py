"""GPU parity of the chain / two-mass integrators against the FP64 oracle,
through the C ABI.

Error metric (per instance): max over frames and DOFs of |gpu - oracle|
divided by max |oracle| (x and v separately).  Tolerances: FP64 1e-10 on the
paper's system; FP32 1e-5 (the FP32 target), with the oracle started from the
same FP32-rounded initial state.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import closed_form as cf
from paper_1702_02207_amd import workloads
from gpu_util import gpu_chain, oracle_chain, f32_inputs

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
TOL_F64 = 1e-10


def _err(got, ref):
    return oracle.rel_traj_err(got, ref)


def test_c1_paper_system_fp64():
    """eq. (3), m = 2, C = 2025, dt = 1e-5, 1e5 RK4 steps in FP64."""
    w = workloads.c1_paper_two_mass(out_stride=100)
    xf, vf, xe, ve = gpu_chain("rk4", "f64", w)
    rx, rv, rxe, rve = oracle_chain("rk4", w)
    assert _err(xf, rx).max() < TOL_F64
    assert _err(vf, rv).max() < TOL_F64
    t = np.arange(xf.shape[0]) * w.out_stride * w.dt[0]
    xa, va = cf.two_mass_equal(t, 2.0, 2025.0, (1.0, 0.0), (0.0, 0.0))
    assert _err(xf, xa[:, None, :]).max() < TOL_F64
    assert _err(vf, va[:, None, :]).max() < TOL_F64


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_c2_subset_fp32(method):
    """Two-mass ensemble subset: 8191 instances (ragged vs the 256-lane block)."""
    w = workloads.c2_two_dof_ensemble(batch=8191, nsteps=10_000, out_stride=100)
    xf, vf, xe, ve = gpu_chain(method, "f32", w)
    x0, v0 = f32_inputs(w)
    rx, rv, rxe, rve = oracle_chain(method, w, x0=x0, v0=v0)
    ex, ev = _err(xf, rx), _err(vf, rv)
    print(f"c2 {method}: x max {ex.max():.3e} p99 {np.percentile(ex, 99):.3e}; "
          f"v max {ev.max():.3e} p99 {np.percentile(ev, 99):.3e}")
    assert ex.max() < TOL_F32
    assert ev.max() < TOL_F32
    np.testing.assert_array_equal(xf[-1], xe)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("s,batch", [(1, 3), (3, 67), (8, 5), (9, 33), (37, 7), (100, 5), (130, 3),
                                     (513, 2), (1000, 3), (1025, 2), (1500, 3), (2048, 2)])
def test_ragged_chains(method, prec, s, batch):
    rng = np.random.default_rng(1000 + s)
    m, k = workloads.random_chain(rng, batch, s)
    dt = 0.01 / workloads.chain_omega_max(m, k)
    x0 = rng.normal(0, 0.1, (batch, s))
    v0 = rng.normal(0, 1.0, (batch, s)) * 0.01 / dt[:, None]
    w = workloads.ChainBatch(m, k, dt, x0, v0, 2000, 250)
    xf, vf, xe, ve = gpu_chain(method, prec, w)
    if prec == "f32":
        x0, v0 = f32_inputs(w)
    rx, rv, rxe, rve = oracle_chain(method, w, x0=x0, v0=v0)
    tol = TOL_F32 if prec == "f32" else TOL_F64
    assert _err(xf, rx).max() < tol
    assert _err(vf, rv).max() < tol
    assert _err(xe, rxe).max() < tol


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_zero_steps_and_stride_beyond_end(method, prec):
    rng = np.random.default_rng(5)
    m, k = workloads.random_chain(rng, 4, 6)
    dt = 0.01 / workloads.chain_omega_max(m, k)
    w = workloads.ChainBatch(m, k, dt, rng.normal(size=(4, 6)), rng.normal(size=(4, 6)), 0, 1)
    xf, vf, xe, ve = gpu_chain(method, prec, w)
    x0, v0 = f32_inputs(w) if prec == "f32" else (w.x0, w.v0)
    assert xf.shape == (1, 4, 6)
    np.testing.assert_array_equal(xe, x0)
    np.testing.assert_array_equal(ve, v0)
    # out_stride > nsteps: only frame 0
    xf, vf, xe, ve = gpu_chain(method, prec, w, nsteps=7, stride=50)
    assert xf.shape == (1, 4, 6)
    np.testing.assert_array_equal(xf[0], x0)


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_plain_matches_batched(method):
    rng = np.random.default_rng(17)
    for s, batch in ((2, 3), (100, 2)):
        m, k = workloads.random_chain(rng, batch, s)
        dt = 0.01 / workloads.chain_omega_max(m, k)
        w = workloads.ChainBatch(m, k, dt, rng.normal(size=(batch, s)), np.zeros((batch, s)), 500, 0)
        from paper_1702_02207_amd import osc
        import torch
        sysm = osc.System("chain", method, "f32", w.m, w.k, w.dt).create()
        x0 = torch.as_tensor(w.x0, dtype=torch.float32, device="cuda")
        v0 = torch.zeros_like(x0)
        _, _, xe, ve = sysm.integrate(x0, v0, 500, 0)
        xp, vp = sysm.integrate_plain(x0, v0, 500)
        sysm.sync()
        sysm.close()
        assert _err(xp.double().cpu().numpy(), xe.double().cpu().numpy()).max() < 1e-6
        assert _err(vp.double().cpu().numpy(), ve.double().cpu().numpy()).max() < 1e-6


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_energy_matches_oracle(prec):
    import torch
    from paper_1702_02207_amd import osc
    rng = np.random.default_rng(23)
    for s, batch in ((2, 100), (37, 9), (1024, 3)):
        m, k = workloads.random_chain(rng, batch, s)
        dt = 0.01 / workloads.chain_omega_max(m, k)
        sysm = osc.System("chain", "verlet", prec, m, k, dt).create()
        tdt = torch.float32 if prec == "f32" else torch.float64
        x = torch.as_tensor(rng.normal(size=(batch, s)), dtype=tdt, device="cuda")
        v = torch.as_tensor(rng.normal(size=(batch, s)), dtype=tdt, device="cuda")
        E = sysm.energy(x, v).cpu().numpy()
        Q = sysm.energy(x, v, shadow=True).cpu().numpy()
        sysm.sync()
        sysm.close()
        xd, vd = x.double().cpu().numpy(), v.double().cpu().numpy()
        np.testing.assert_allclose(E, oracle.energy_chain(m, k, xd, vd), rtol=1e-12)
        np.testing.assert_allclose(Q, oracle.verlet_q_chain(m, k, dt, xd, vd), rtol=1e-11)


def test_nonfinite_is_reported():
    import torch
    from paper_1702_02207_amd import osc
    m, k = np.ones((2, 3)), np.full((2, 3), 100.0)
    sysm = osc.System("chain", "rk4", "f32", m, k, [1e-3, 1e-3]).create()
    x0 = torch.zeros((2, 3), dtype=torch.float32, device="cuda")
    x0[1, 1] = float("inf")
    sysm.integrate(x0, torch.zeros_like(x0), 10, 0)
    with pytest.raises(osc.OscError) as e:
        sysm.sync()
    assert e.value.status == osc.OSC_ENONFINITE
    sysm.integrate(torch.zeros_like(x0), torch.zeros_like(x0), 10, 0)
    sysm.sync()          # the flag was cleared
    sysm.close()


def test_create_rejects_bad_parameters():
    from paper_1702_02207_amd import osc
    m, k = np.ones((1, 2)), np.full((1, 2), 100.0)
    with pytest.raises(osc.OscError) as e:
        osc.System("chain", "rk4", "f32", m, k, [0.0]).create()
    assert e.value.status == osc.OSC_EINVAL
    with pytest.raises(osc.OscError) as e:
        osc.System("chain", "rk4", "f32", -m, k, [1e-3]).create()
    assert e.value.status == osc.OSC_EINVAL
    # h omega: for this chain omega_max ~ 16.2; dt = 1 is far outside both limits
    for meth in ("rk4", "verlet"):
        with pytest.raises(osc.OscError) as e:
            osc.System("chain", meth, "f32", m, k, [1.0]).create()
        assert e.value.status == osc.OSC_EUNSTABLE


def _stiff_link_chain(s, theta, heavy=100.0):
    """Chain whose Gershgorin bound overstates h omega_max by about sqrt(2):
    light and heavy bodies in turn, a weak wall spring and stiff links."""
    m = np.where(np.arange(s) % 2 == 0, 1.0, heavy)[None, :]
    k = np.full((1, s), 1e4)
    k[0, 0] = 1.0
    dt = np.array([theta / workloads.chain_omega_max(m, k)[0]])
    return m, k, dt


@pytest.mark.parametrize("s", [2, 301])
def test_stability_check_uses_exact_frequency(s):
    """The boundary accepts a step when the exact h omega_max, with a 1 %
    margin, lies within 2.78 (RK4) or 1.99 (Verlet), even where the
    Gershgorin bound alone would refuse it, and rejects it otherwise."""
    from paper_1702_02207_amd import osc
    for meth, ok_theta, bad_theta in (("rk4", 2.6, 2.76), ("verlet", 1.9, 1.975)):
        m, k, dt = _stiff_link_chain(s, ok_theta)
        cl = dt[0] ** 2 * k[0] / m[0]
        cr = dt[0] ** 2 * np.r_[k[0, 1:], 0.0] / m[0]
        assert np.sqrt(2 * (cl + cr)).max() > (2.78 if meth == "rk4" else 1.99)   # Gershgorin refuses
        osc.System("chain", meth, "f32", m, k, dt).create().close()
        m, k, dt = _stiff_link_chain(s, bad_theta)
        with pytest.raises(osc.OscError) as e:
            osc.System("chain", meth, "f32", m, k, dt).create()
        assert e.value.status == osc.OSC_EUNSTABLE


def test_step_near_the_rk4_limit_matches_oracle():
    """A chain accepted at h omega_max = 2.6 (beyond its Gershgorin bound)
    integrates like the oracle in FP64."""
    m, k, dt = _stiff_link_chain(40, 2.6)
    rng = np.random.default_rng(3)
    w = workloads.ChainBatch(m, k, dt, rng.normal(size=(1, 40)), rng.normal(size=(1, 40)), 300, 30)
    xf, vf, _, _ = gpu_chain("rk4", "f64", w)
    rx, rv, _, _ = oracle_chain("rk4", w)
    assert oracle.rel_traj_err(xf, rx).max() < 1e-10
    assert oracle.rel_traj_err(vf, rv).max() < 1e-10


def test_empty_batch():
    import torch
    from paper_1702_02207_amd import osc
    sysm = osc.System("chain", "rk4", "f32", np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0)).create()
    x0 = torch.zeros((0, 4), dtype=torch.float32, device="cuda")
    xf, vf, xe, ve = sysm.integrate(x0, x0, 10, 5)
    sysm.sync()
    assert xe.shape == (0, 4) and xf.shape == (3, 0, 4)
    sysm.close()


def _run_chain(sysm, w, nsteps, stride):
    import torch
    x0 = torch.as_tensor(w.x0, dtype=torch.float32, device="cuda")
    v0 = torch.as_tensor(w.v0, dtype=torch.float32, device="cuda")
    xf, vf, xe, ve = sysm.integrate(x0, v0, nsteps, stride)
    sysm.sync()
    return [t.cpu().numpy() for t in (xf, vf, xe, ve)]


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_chain_layouts_and_chunking_are_bitwise_identical(method):
    """The same instance gives bitwise-identical results whatever lane layout
    holds it and however the run is cut into launches."""
    from paper_1702_02207_amd import osc
    rng = np.random.default_rng(31)
    s, batch = 100, 7
    m, k = workloads.random_chain(rng, batch, s)
    dt = 0.01 / workloads.chain_omega_max(m, k)
    w = workloads.ChainBatch(m, k, dt, rng.normal(0, 0.1, (batch, s)),
                             rng.normal(0, 1, (batch, s)) * 0.01 / dt[:, None], 600, 150)
    sysm = osc.System("chain", method, "f32", m, k, dt).create()
    ref = _run_chain(sysm, w, 600, 150)
    for lpi, dpl in ((16, 8), (32, 8), (64, 4), (64, 8), (64, 16), (128, 16)):
        sysm.set_config(osc.CFG_CHAIN_LAYOUT, (lpi << 16) | dpl)
        got = _run_chain(sysm, w, 600, 150)
        for a, b in zip(ref, got):
            np.testing.assert_array_equal(a, b)
    sysm.set_config(osc.CFG_CHAIN_LAYOUT, 0)
    sysm.set_config(osc.CFG_STEPS_PER_LAUNCH, 77)
    got = _run_chain(sysm, w, 600, 150)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)
    with pytest.raises(osc.OscError):
        sysm.set_config(osc.CFG_CHAIN_LAYOUT, (4 << 16) | 8)     # 32 < s
    sysm.close()


def test_batch_composition_invariance():
    """An instance's result does not depend on which other instances share
    the launch (lane-group layout, ragged tails)."""
    w = workloads.c2_two_dof_ensemble(batch=5000, nsteps=500, out_stride=0)
    _, _, xe_all, ve_all = gpu_chain("rk4", "f32", w)
    idx = np.array([0, 17, 255, 256, 4999])
    _, _, xe_sub, ve_sub = gpu_chain("rk4", "f32", w.subset(idx))
    np.testing.assert_array_equal(xe_all[idx], xe_sub)
    np.testing.assert_array_equal(ve_all[idx], ve_sub)


def test_autotune_picks_a_layout_and_caches_it(tmp_path, monkeypatch):
    import torch
    from paper_1702_02207_amd import osc
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("OSC_AUTOTUNE_CACHE", str(cache))
    rng = np.random.default_rng(41)
    s, batch = 200, 96
    m, k = workloads.random_chain(rng, batch, s)
    dt = 0.01 / workloads.chain_omega_max(m, k)
    w = workloads.ChainBatch(m, k, dt, rng.normal(0, 0.1, (batch, s)), np.zeros((batch, s)), 400, 100)
    sysm = osc.System("chain", "rk4", "f32", m, k, dt).create()
    ref = _run_chain(sysm, w, 400, 100)
    x0 = torch.as_tensor(w.x0, dtype=torch.float32, device="cuda")
    v0 = torch.zeros_like(x0)
    chosen = sysm.autotune(x0, v0, probe_steps=50)
    lpi, dpl = chosen >> 16, chosen & 0xffff
    assert lpi * dpl >= s
    got = _run_chain(sysm, w, 400, 100)
    sysm.close()
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)
    line = cache.read_text().strip().splitlines()[-1]
    assert line.startswith("chain rk4 f32 200 ") and line.endswith(str(chosen))
    # a new handle with the same key picks the cached layout (same results)
    sysm = osc.System("chain", "rk4", "f32", m, k, dt).create()
    got = _run_chain(sysm, w, 400, 100)
    sysm.close()
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)


def test_autotune_dense_prefers_a_feasible_kernel():
    import torch
    from paper_1702_02207_amd import osc
    rng = np.random.default_rng(43)
    M, K = workloads.random_dense_system(rng, 128)
    dt = [0.01 / workloads.dense_omega_max(M, K)]
    sysm = osc.System("dense", "rk4", "f32", M, K, dt, shared=True, batch=256).create()
    x0 = torch.as_tensor(rng.normal(size=(256, 128)), dtype=torch.float32, device="cuda")
    chosen = sysm.autotune(x0, torch.zeros_like(x0), probe_steps=50)
    sysm.close()
    assert chosen in (1, 2, 3)


def _misaligned_like(t):
    """A contiguous tensor like t whose data starts 4 bytes past a 16-byte boundary."""
    import torch
    buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=t.device)
    out = buf[1:].view(t.shape)
    out.copy_(t)
    return out


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_misaligned_buffers_give_identical_results(method):
    """Runs of DOFs move as 16-byte vectors only when aligned; buffers offset
    by one float take the element-wise path and must give the same bits."""
    import torch
    from paper_1702_02207_amd import osc
    rng = np.random.default_rng(37)
    s, batch = 64, 9
    m, k = workloads.random_chain(rng, batch, s)
    dt = 0.01 / workloads.chain_omega_max(m, k)
    sysm = osc.System("chain", method, "f32", m, k, dt).create()
    x0 = torch.as_tensor(rng.normal(0, 0.1, (batch, s)), dtype=torch.float32, device="cuda")
    v0 = torch.as_tensor(rng.normal(0, 1, (batch, s)), dtype=torch.float32, device="cuda") * 0.01
    ref = [t.cpu().numpy() for t in sysm.integrate(x0, v0, 300, 100)]
    xm, vm = _misaligned_like(x0), _misaligned_like(v0)
    outs = tuple(_misaligned_like(torch.zeros_like(t)) for t in
                 (torch.empty((4, batch, s), device="cuda"), torch.empty((4, batch, s), device="cuda"), x0, v0))
    got = [t.cpu().numpy() for t in sysm.integrate(xm, vm, 300, 100, out=outs)]
    sysm.sync()
    sysm.close()
    assert xm.data_ptr() % 16 != 0
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)
