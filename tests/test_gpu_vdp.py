"""Coupled Van der Pol chains (osc_set_van_der_pol) through the C ABI against
the FP64 oracle: every register layout in FP32 and FP64, chunked and
allocation-free runs bit for bit equal to one launch, real-time ticks equal
to the frames of one integration, and the combinations the entry point
refuses."""
import numpy as np
import pytest

import oracle
from paper_1702_02207_amd import osc, workloads
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-10}


def _vdp(seed, batch, s, nsteps, stride):
    """Random chains (masses U[0.5, 2], springs log-U[1e2, 1e4]), dt = 0.01 /
    omega_max, x0 ~ N(0, 1), v0 = 0, and mu of the order of the chains'
    frequencies, so that the elements shape the motion within the run."""
    rng = np.random.default_rng(seed)
    m, k = workloads.random_chain(rng, batch, s)
    wmax = workloads.chain_omega_max(m, k)
    dt = 0.01 / wmax
    mu = float(0.2 * np.median(wmax))
    x0 = rng.normal(0.0, 1.0, (batch, s))
    v0 = np.zeros((batch, s))
    return m, k, dt, mu, x0, v0


def _run(sysm, x0, v0, nsteps, stride, prec, static=False):
    import torch
    dt = torch.float32 if prec == "f32" else torch.float64
    out = sysm.integrate(to_dev(x0, dt), to_dev(v0, dt), nsteps, stride, static=static)
    sysm.sync()
    return [None if t is None else t.double().cpu().numpy() for t in out]


def _inputs(x0, v0, prec):
    if prec == "f32":
        return x0.astype(np.float32).astype(np.float64), v0.astype(np.float32).astype(np.float64)
    return x0, v0


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("s,batch", [(1, 33), (2, 40), (5, 9), (8, 70), (37, 3), (64, 2), (100, 3), (300, 2),
                                     (700, 2), (1024, 2)])
def test_vdp_chains_match_oracle(s, batch, prec):
    """Every register layout (one lane per chain for s <= 8, one wave per
    chain beyond; ragged runs at s = 5, 37, 100, 300, 700) against the
    oracle's stage-form RK4, frames and end state."""
    nsteps, stride = 1500, 250
    m, k, dt, mu, x0, v0 = _vdp(900 + s, batch, s, nsteps, stride)
    sysm = osc.System("chain", "rk4", prec, m, k, dt).create()
    try:
        sysm.set_van_der_pol(mu)
        xf, vf, xe, ve = _run(sysm, x0, v0, nsteps, stride, prec)
    finally:
        sysm.close()
    x0r, v0r = _inputs(x0, v0, prec)
    rx, rv, rxe, rve = oracle.chain_vdp(m, k, dt, mu, x0r, v0r, nsteps, stride)
    ex, ev = oracle.rel_traj_err(xf, rx).max(), oracle.rel_traj_err(vf, rv).max()
    print(f"vdp s={s} {prec}: x {ex:.2e} v {ev:.2e}")
    assert max(ex, ev) < TOL[prec]
    np.testing.assert_array_equal(xf[-1], xe)
    np.testing.assert_array_equal(vf[-1], ve)
    # the elements matter in this run: the linear chain ends elsewhere
    lx, _, _, _ = oracle.chain("rk4", m, k, dt, x0r, v0r, nsteps, stride)
    assert oracle.rel_traj_err(lx, rx).max() > 100 * TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_vdp_chunked_and_static_runs_are_bitwise_one_launch(prec):
    """The compensated state passes between launches: chunks of 333 steps,
    and the allocation-free entry with the same chunks, give the bits of one
    launch."""
    m, k, dt, mu, x0, v0 = _vdp(950, 4, 300, 1200, 200)
    sysm = osc.System("chain", "rk4", prec, m, k, dt).create()
    try:
        sysm.set_van_der_pol(mu)
        whole = _run(sysm, x0, v0, 1200, 200, prec)
        sysm.set_config(osc.CFG_STEPS_PER_LAUNCH, 333)
        chunked = _run(sysm, x0, v0, 1200, 200, prec)
        static = _run(sysm, x0, v0, 1200, 200, prec, static=True)
    finally:
        sysm.close()
    for a, b, c in zip(whole, chunked, static):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)


@pytest.mark.parametrize("prec,s,batch", [("f64", 2, 1), ("f32", 2, 3), ("f32", 300, 2), ("f64", 700, 1)])
def test_vdp_real_time_ticks_are_the_frames_of_one_integration(prec, s, batch):
    """Both real-time steppers on Van der Pol chains (the pair is the two
    coupled oscillators of the paper's section 1): the states after the ticks
    of the launch-per-tick loop and of the resident kernel equal the frames of
    one osc_integrate call bit for bit."""
    import torch
    dtype = torch.float32 if prec == "f32" else torch.float64
    m, k, dt, mu, x0, v0 = _vdp(960 + s, batch, s, 400, 4)
    sysm = osc.System("chain", "rk4", prec, m, k, dt).create()
    try:
        sysm.set_van_der_pol(mu)
        X0, V0 = to_dev(x0, dtype), to_dev(v0, dtype)
        xf, vf, _, _ = sysm.integrate(X0, V0, 400, 4)
        sysm.sync()
        ref_x, ref_v = xf[1:].cpu().numpy(), vf[1:].cpu().numpy()
        with osc.Realtime(sysm, X0, V0, 4) as rt:
            tx, tv, lat, stats = rt.run(100e-6, 100)
            tx, tv = tx.cpu().numpy(), tv.cpu().numpy()
        with osc.Realtime(sysm, X0, V0, 4) as rt:
            rx, rv, rlat, rstats = rt.run_resident(100e-6, 100)
            rx, rv = rx.cpu().numpy(), rv.cpu().numpy()
    finally:
        sysm.close()
    for got in ((tx, tv), (rx, rv)):
        np.testing.assert_array_equal(got[0], ref_x)
        np.testing.assert_array_equal(got[1], ref_v)
    assert stats["ticks"] == 100 and rstats["ticks"] == 100


def test_vdp_rejects_what_it_does_not_cover():
    import torch
    m, k, dt, mu, x0, v0 = _vdp(970, 2, 5, 10, 0)
    vsys = osc.System("chain", "verlet", "f32", m, k, dt).create()
    try:
        with pytest.raises(osc.OscError) as e:      # Verlet
            vsys.set_van_der_pol(mu)
        assert e.value.status == osc.OSC_ENOTSUP
    finally:
        vsys.close()
    rng = np.random.default_rng(1)
    M, K = workloads.random_dense_system(rng, 6)
    dsys = osc.System("dense", "rk4", "f32", M, K, np.array([0.01]), shared=True, batch=2).create()
    try:
        with pytest.raises(osc.OscError) as e:      # dense
            dsys.set_van_der_pol(mu)
        assert e.value.status == osc.OSC_ENOTSUP
    finally:
        dsys.close()
    sysm = osc.System("chain", "rk4", "f32", m, k, dt).create()
    try:
        for bad in (-1.0, float("nan"), float("inf")):
            with pytest.raises(osc.OscError) as e:
                sysm.set_van_der_pol(bad)
            assert e.value.status == osc.OSC_EINVAL
        sysm.set_van_der_pol(mu)
        X0 = to_dev(x0, torch.float32)
        for call in (lambda: sysm.set_excitation(0.1, 0.0),
                     lambda: sysm.set_config(osc.CFG_PROPAGATOR, 1),
                     lambda: sysm.propagator(3),
                     lambda: sysm.integrate_plain(X0, X0, 10),
                     lambda: sysm.autotune(X0, X0, probe_steps=5)):
            with pytest.raises(osc.OscError) as e:
                call()
            assert e.value.status == osc.OSC_ENOTSUP
        sysm.set_van_der_pol(0.0)                   # linear again: the free integrator
        sysm.set_excitation(0.1, 0.0)
        with pytest.raises(osc.OscError) as e:
            sysm.set_van_der_pol(mu)
        assert e.value.status == osc.OSC_ENOTSUP
        with pytest.raises(osc.OscError) as e:      # damped: fixed layouts, nothing to tune
            sysm.autotune(X0, X0, probe_steps=5)
        assert e.value.status == osc.OSC_ENOTSUP
    finally:
        sysm.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_vdp_step_too_long_for_mu_reports_nonfinite(prec):
    """The linear stability check of osc_create cannot bound the nonlinear
    term: with h mu |x|^2 far beyond RK4's region the state overflows, as the
    oracle's does, and osc_sync reports OSC_ENONFINITE."""
    m = np.array([[1.0, 1.0]])
    k = np.array([[1.0, 1.0]])
    dt = np.array([0.05])
    x0 = np.array([[2.0, -1.0]])
    v0 = np.zeros((1, 2))
    _, _, xe, _ = oracle.chain_vdp(m, k, dt, 100.0, x0, v0, 200, 0, frames=False)
    assert not np.isfinite(xe).all()
    sysm = osc.System("chain", "rk4", prec, m, k, dt).create()
    try:
        sysm.set_van_der_pol(100.0)
        with pytest.raises(osc.OscError) as e:
            _run(sysm, x0, v0, 200, 0, prec)
        assert e.value.status == osc.OSC_ENONFINITE
        sysm.set_van_der_pol(1.0)                   # a step that suits mu: finite again
        _run(sysm, x0, v0, 200, 0, prec)
    finally:
        sysm.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("nsteps,stride", [(0, 10), (0, 0), (7, 100), (100, 100), (1, 0)])
def test_vdp_degenerate_runs(prec, nsteps, stride):
    """No step (the caller's state comes back unchanged), a stride beyond the
    run (frame 0 only), a stride equal to the run and a single step."""
    m, k, dt, mu, x0, v0 = _vdp(990 + nsteps, 3, 37, nsteps, stride)
    v0 = np.random.default_rng(5).normal(0.0, 1.0, x0.shape)
    sysm = osc.System("chain", "rk4", prec, m, k, dt).create()
    try:
        sysm.set_van_der_pol(mu)
        xf, vf, xe, ve = _run(sysm, x0, v0, nsteps, stride, prec)
    finally:
        sysm.close()
    x0r, v0r = _inputs(x0, v0, prec)
    rx, rv, rxe, rve = oracle.chain_vdp(m, k, dt, mu, x0r, v0r, nsteps, stride)
    if nsteps == 0:
        np.testing.assert_array_equal(xe, x0r)
        np.testing.assert_array_equal(ve, v0r)
    if rx is not None:
        assert xf.shape == rx.shape
        np.testing.assert_array_equal(xf[0], x0r)
        assert max(oracle.rel_traj_err(xf, rx).max(), oracle.rel_traj_err(vf, rv).max()) < TOL[prec]
    else:
        assert xf is None and vf is None
    scale = np.maximum(np.abs(rxe).max(axis=1), 1e-300)
    assert (np.abs(xe - rxe).max(axis=1) / scale).max() < TOL[prec]


def _force(seed, m, k, batch, s):
    """Forces of the order of the springs' (F ~ N(0, mean k)) at frequencies
    near the chains' own (Omega ~ U[0.5, 2] x the median omega_max / 10)."""
    rng = np.random.default_rng(seed)
    F = rng.normal(0.0, 1.0, (batch, s)) * k.mean(axis=1, keepdims=True)
    W = rng.uniform(0.5, 2.0, batch) * np.median(workloads.chain_omega_max(m, k)) / 10.0
    return F, W


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("s,batch", [(2, 40), (8, 9), (64, 2), (300, 2), (1024, 2)])
def test_forced_vdp_chains_match_oracle(s, batch, prec):
    """The forced Van der Pol chain (a force set by osc_set_excitation on a
    Van der Pol handle) against the oracle on every kind of layout; chunks of
    333 steps (across the force phase's 64-step anchors) and the allocation-
    free entry give the bits of one launch."""
    nsteps, stride = 1500, 250
    m, k, dt, mu, x0, v0 = _vdp(1100 + s, batch, s, nsteps, stride)
    F, W = _force(1200 + s, m, k, batch, s)
    sysm = osc.System("chain", "rk4", prec, m, k, dt).create()
    try:
        sysm.set_van_der_pol(mu)
        sysm.set_excitation(0.0, 0.0, F, W)
        whole = _run(sysm, x0, v0, nsteps, stride, prec)
        sysm.set_config(osc.CFG_STEPS_PER_LAUNCH, 333)
        chunked = _run(sysm, x0, v0, nsteps, stride, prec)
        static = _run(sysm, x0, v0, nsteps, stride, prec, static=True)
    finally:
        sysm.close()
    for a, b, c in zip(whole, chunked, static):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)
    x0r, v0r = _inputs(x0, v0, prec)
    rx, rv, rxe, rve = oracle.chain_vdp(m, k, dt, mu, x0r, v0r, nsteps, stride, F=F, omega=W)
    xf, vf, xe, ve = whole
    ex, ev = oracle.rel_traj_err(xf, rx).max(), oracle.rel_traj_err(vf, rv).max()
    print(f"forced vdp s={s} {prec}: x {ex:.2e} v {ev:.2e}")
    assert max(ex, ev) < TOL[prec]
    # the force matters in this run: the unforced Van der Pol chain ends elsewhere
    ux, _, _, _ = oracle.chain_vdp(m, k, dt, mu, x0r, v0r, nsteps, stride)
    assert oracle.rel_traj_err(ux, rx).max() > 100 * TOL[prec]


def test_forced_vdp_resident_ticks_are_the_frames_of_one_integration():
    """The forced Van der Pol pair stepped by the resident real-time kernel:
    the states after the ticks equal the frames of one integration bit for
    bit (the force's phase follows the global step)."""
    import torch
    m, k, dt, mu, x0, v0 = _vdp(1300, 2, 2, 400, 4)
    F, W = _force(1301, m, k, 2, 2)
    sysm = osc.System("chain", "rk4", "f64", m, k, dt).create()
    try:
        sysm.set_van_der_pol(mu)
        sysm.set_excitation(0.0, 0.0, F, W)
        X0, V0 = to_dev(x0, torch.float64), to_dev(v0, torch.float64)
        xf, vf, _, _ = sysm.integrate(X0, V0, 400, 4)
        sysm.sync()
        ref_x, ref_v = xf[1:].cpu().numpy(), vf[1:].cpu().numpy()
        with osc.Realtime(sysm, X0, V0, 4) as rt:
            rx, rv, _, st = rt.run_resident(100e-6, 100)
            rx, rv = rx.cpu().numpy(), rv.cpu().numpy()
    finally:
        sysm.close()
    np.testing.assert_array_equal(rx, ref_x)
    np.testing.assert_array_equal(rv, ref_v)
    assert st["ticks"] == 100
