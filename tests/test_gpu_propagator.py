"""GPU parity of the propagator form (the scheme as its matrix, for eq. (1)
with the constant first-order matrix of section 3) against the FP64 oracle,
through the C ABI: osc_propagator against the oracle's k-step matrix, frame
jumps and the per-step propagator against the oracle's stage-form
trajectories."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import closed_form as cf
from paper_1702_02207_amd import osc, workloads
from gpu_util import to_dev, f32_inputs

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
TOL_F64 = 1e-10


def _chain(seed, batch, s, nsteps, stride, vscale=0.05):
    rng = np.random.default_rng(seed)
    m, k = workloads.random_chain(rng, batch, s)
    dt = 0.01 / workloads.chain_omega_max(m, k)
    x0 = rng.normal(0.0, 0.1, (batch, s))
    v0 = rng.normal(0.0, 1.0, (batch, s)) * vscale
    return workloads.ChainBatch(m, k, dt, x0, v0, nsteps, stride)


def _dense(seed, batch, s, nsteps, stride, shared=True, theta=0.01):
    rng = np.random.default_rng(seed)
    if shared:
        M, K = workloads.random_dense_system(rng, s)
        dt = np.array([theta / workloads.dense_omega_max(M, K)])
    else:
        Ms, Ks = zip(*[workloads.random_dense_system(rng, s) for _ in range(batch)])
        M, K = np.array(Ms), np.array(Ks)
        dt = np.array([theta / workloads.dense_omega_max(M[b], K[b]) for b in range(batch)])
    x0 = rng.normal(0.0, 1.0, (batch, s))
    v0 = rng.normal(0.0, 1.0, (batch, s)) * 0.01
    return workloads.DenseBatch(M, K, dt, x0, v0, nsteps, stride, shared)


def _blocks_close(got, ref, tol, label):
    """Compare the four s x s blocks of a (2s x 2s) matrix, each relative to
    its own largest entry (position and velocity rows differ in scale)."""
    s = ref.shape[0] // 2
    for bi in range(2):
        for bj in range(2):
            g = got[bi * s:(bi + 1) * s, bj * s:(bj + 1) * s]
            r = ref[bi * s:(bi + 1) * s, bj * s:(bj + 1) * s]
            scale = max(np.abs(r).max(), 1e-300)
            err = np.abs(g - r).max() / scale
            assert err <= tol, (label, bi, bj, err)


@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("s,batch", [(1, 3), (2, 4), (3, 2), (7, 2)])
@pytest.mark.parametrize("k", [0, 1, 7, 1000])
def test_chain_propagator_matches_oracle(method, s, batch, k):
    w = _chain(700 + s, batch, s, 1, 0)
    sysm = osc.System("chain", method, "f64", w.m, w.k, w.dt).create()
    try:
        P = sysm.propagator(k).cpu().numpy()
        sysm.sync()
    finally:
        sysm.close()
    assert P.shape == (batch, 2 * s, 2 * s)
    for b in range(batch):
        ref = oracle.propagator(method, "chain", w.m[b], w.k[b], w.dt[b], k)
        _blocks_close(P[b], ref, 1e-11, f"chain s={s} b={b} k={k}")


@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("s,k", [(2, 1), (2, 1000), (5, 37), (64, 1), (64, 1000), (130, 7), (300, 5)])
def test_dense_propagator_matches_oracle(method, s, k):
    w = _dense(720 + s, 2, s, 1, 0)
    sysm = osc.System("dense", method, "f64", w.M, w.K, w.dt, shared=True, batch=2).create()
    try:
        P = sysm.propagator(k).cpu().numpy()
        sysm.sync()
    finally:
        sysm.close()
    assert P.shape == (1, 2 * s, 2 * s)
    ref = oracle.propagator(method, "dense", w.M, w.K, w.dt[0], k)
    _blocks_close(P[0], ref, 1e-11, f"dense s={s} k={k}")


def test_per_instance_dense_propagator_matches_oracle():
    w = _dense(740, 3, 6, 1, 0, shared=False)
    sysm = osc.System("dense", "rk4", "f64", w.M, w.K, w.dt, shared=False, batch=3).create()
    try:
        P = sysm.propagator(25).cpu().numpy()
        sysm.sync()
    finally:
        sysm.close()
    for b in range(3):
        _blocks_close(P[b], oracle.propagator("rk4", "dense", w.M[b], w.K[b], w.dt[b], 25), 1e-11, f"b={b}")


def _gpu_run(sysm, w, prec, mode, steps_per_launch=0, static=False):
    import torch
    dtype = torch.float32 if prec == "f32" else torch.float64
    sysm.set_config(osc.CFG_PROPAGATOR, mode)
    if steps_per_launch:
        sysm.set_config(osc.CFG_STEPS_PER_LAUNCH, steps_per_launch)
    x0, v0 = to_dev(w.x0, dtype), to_dev(w.v0, dtype)
    out = sysm.integrate(x0, v0, w.nsteps, w.out_stride, static=static)
    sysm.sync()
    return [None if t is None else t.double().cpu().numpy() for t in out]


def _oracle_for(w, method, prec):
    x0, v0 = f32_inputs(w) if prec == "f32" else (w.x0, w.v0)
    if isinstance(w, workloads.ChainBatch):
        return oracle.chain(method, w.m, w.k, w.dt, x0, v0, w.nsteps, w.out_stride)
    return oracle.dense(method, w.M, w.K, w.dt, x0, v0, w.nsteps, w.out_stride, shared=w.shared)


def _check_traj(got, ref, tol, label):
    """Relative trajectory error of the frames; the final state relative to
    the scale of the instance's trajectory (the frames' largest value), since
    a single state of one DOF can sit at a zero crossing."""
    xf, vf, xe, ve = got
    rx, rv, rxe, rve = ref
    if rx is not None:
        ex, ev = oracle.rel_traj_err(xf, rx).max(), oracle.rel_traj_err(vf, rv).max()
        xs = np.maximum(np.abs(rx).max(axis=(0, 2)), np.abs(rxe).max(axis=1))
        vs = np.maximum(np.abs(rv).max(axis=(0, 2)), np.abs(rve).max(axis=1))
        exe = (np.abs(xe - rxe).max(axis=1) / xs).max()
        eve = (np.abs(ve - rve).max(axis=1) / vs).max()
    else:
        ex = ev = 0.0
        exe, eve = oracle.rel_traj_err(xe, rxe).max(), oracle.rel_traj_err(ve, rve).max()
    print(f"{label}: frames x {ex:.2e} v {ev:.2e}, end x {exe:.2e} v {eve:.2e}")
    assert max(ex, ev, exe, eve) < tol, label


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("s,batch,nsteps,stride", [(1, 37, 2000, 250), (2, 300, 3000, 700), (2, 5, 1234, 0),
                                                   (3, 9, 800, 100), (7, 4, 600, 250), (300, 2, 800, 100)])
def test_chain_frame_jumps(method, prec, s, batch, nsteps, stride):
    """Frames by powers of the one-step matrix (registers for s <= 2, batched
    matrix-core products beyond): the scheme's trajectory at the frames;
    nsteps not a multiple of the stride, and no frames at all."""
    w = _chain(760 + s, batch, s, nsteps, stride)
    sysm = osc.System("chain", method, prec, w.m, w.k, w.dt).create()
    try:
        got = _gpu_run(sysm, w, prec, 1)
    finally:
        sysm.close()
    _check_traj(got, _oracle_for(w, method, prec), 1e-6 if prec == "f32" else TOL_F64,
                f"chain jumps {method} {prec} s={s}")


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("s,batch,shared", [(2, 50, True), (5, 3, False), (64, 70, True), (100, 20, True),
                                            (300, 2, True)])
def test_dense_frame_jumps(method, prec, s, batch, shared):
    w = _dense(780 + s, batch, s, 2000, 300, shared=shared)
    sysm = osc.System("dense", method, prec, w.M, w.K, w.dt, shared=shared, batch=batch).create()
    try:
        got = _gpu_run(sysm, w, prec, 1)
    finally:
        sysm.close()
    _check_traj(got, _oracle_for(w, method, prec), 1e-6 if prec == "f32" else TOL_F64,
                f"dense jumps {method} {prec} s={s}")


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_dense_frame_jumps_at_the_largest_size(method):
    """s = 2048, the largest size the library takes: frames by powers of the
    4096 x 4096 one-step matrix, against the exact discrete solution of the
    scheme per normal mode (LAPACK eigh of (K, M); the FP64 oracle's own
    stepping needs minutes at this size).  An FP64 replica of the jumps on
    the CPU meets that closed form to 2e-13."""
    w = _dense(2801, 1, 2048, 1000, 250)
    sysm = osc.System("dense", method, "f64", w.M, w.K, w.dt, shared=True, batch=1).create()
    try:
        xf, vf, xe, ve = _gpu_run(sysm, w, "f64", 1)
    finally:
        sysm.close()
    exact = cf.rk4_discrete if method == "rk4" else cf.verlet_discrete
    rx, rv = exact(np.arange(0, 1001, 250), w.dt[0], w.M, w.K, w.x0[0], w.v0[0])
    ex = oracle.rel_traj_err(xf, rx[:, None, :]).max()
    ev = oracle.rel_traj_err(vf, rv[:, None, :]).max()
    print(f"s=2048 {method} jumps against the modal solution: x {ex:.2e} v {ev:.2e}")
    assert max(ex, ev) < TOL_F64
    np.testing.assert_array_equal(xf[-1], xe)
    np.testing.assert_array_equal(vf[-1], ve)


def test_paper_system_frame_jumps_match_closed_form():
    """The paper's two-mass system (eq. (3), FP64, 1e5 RK4 steps) by frame
    jumps against the closed-form normal-mode solution (eq. (4)-(7))."""
    w = workloads.c1_paper_two_mass(out_stride=1000)
    sysm = osc.System("chain", "rk4", "f64", w.m, w.k, w.dt).create()
    try:
        xf, vf, xe, ve = _gpu_run(sysm, w, "f64", 1)
    finally:
        sysm.close()
    t = np.arange(xf.shape[0]) * w.out_stride * w.dt[0]
    x_ref, v_ref = cf.two_mass_equal(t, 2.0, 2025.0, w.x0[0], w.v0[0])
    assert oracle.rel_traj_err(xf, x_ref[:, None, :]).max() < TOL_F64
    assert oracle.rel_traj_err(vf, v_ref[:, None, :]).max() < TOL_F64


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("s", [1, 2])
def test_per_step_propagator(method, prec, s):
    """One application of the one-step matrix per step; chunked runs equal
    unchunked ones bit for bit, and so does the allocation-free entry."""
    w = _chain(800 + s, 500, s, 3000, 500)
    sysm = osc.System("chain", method, prec, w.m, w.k, w.dt).create()
    try:
        got = _gpu_run(sysm, w, prec, 2)
        chunked = _gpu_run(sysm, w, prec, 2, steps_per_launch=333)
        static = _gpu_run(sysm, w, prec, 2, steps_per_launch=333, static=True)
    finally:
        sysm.close()
    for a, b, c in zip(got, chunked, static):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)
    _check_traj(got, _oracle_for(w, method, prec), TOL_F32 if prec == "f32" else TOL_F64,
                f"per-step propagator {method} {prec} s={s}")


def test_propagator_modes_reject_what_they_do_not_cover():
    w = _chain(820, 4, 3, 10, 0)
    sysm = osc.System("chain", "rk4", "f32", w.m, w.k, w.dt).create()
    try:
        with pytest.raises(osc.OscError) as e:
            sysm.set_config(osc.CFG_PROPAGATOR, 2)
        assert e.value.status == osc.OSC_ENOTSUP
        with pytest.raises(osc.OscError) as e:
            sysm.set_config(osc.CFG_PROPAGATOR, 3)
        assert e.value.status == osc.OSC_EINVAL
        sysm.set_config(osc.CFG_PROPAGATOR, 1)
        import torch
        x0 = to_dev(w.x0, torch.float32)
        with pytest.raises(osc.OscError) as e:
            sysm.integrate(x0, x0, 10, 0, static=True)
        assert e.value.status == osc.OSC_ENOTSUP
        with pytest.raises(ValueError):
            sysm.propagator(-1)
    finally:
        sysm.close()


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_two_mass_ensemble_full_per_step_propagator(method):
    """2^20 two-mass instances, 1e4 steps on the per-step propagator: 512
    sampled instances against the oracle and the FP64 invariant of every
    instance (E for RK4, Q for Verlet) within 1e-6 of its initial value."""
    import torch
    w = workloads.c2_two_dof_ensemble()
    w.out_stride = w.nsteps
    sysm = osc.System("chain", method, "f32", w.m, w.k, w.dt).create()
    try:
        sysm.set_config(osc.CFG_PROPAGATOR, 2)
        x0, v0 = to_dev(w.x0, torch.float32), to_dev(w.v0, torch.float32)
        xf, vf, xe, ve = sysm.integrate(x0, v0, w.nsteps, w.out_stride)
        inv = sysm.energy(xe, ve, shadow=(method == "verlet")).cpu().numpy()
        sysm.sync()
        xf, vf = xf.double().cpu().numpy(), vf.double().cpu().numpy()
    finally:
        sysm.close()
    rng = np.random.default_rng(830)
    idx = np.unique(np.concatenate([[0, w.batch - 1], rng.choice(w.batch, 510, replace=False)]))
    sub = w.subset(idx)
    sx0, sv0 = f32_inputs(sub)
    rx, rv, _, _ = oracle.chain(method, sub.m, sub.k, sub.dt, sx0, sv0, w.nsteps, w.out_stride)
    ex, ev = oracle.rel_traj_err(xf[:, idx], rx), oracle.rel_traj_err(vf[:, idx], rv)
    print(f"two-mass per-step propagator {method}: x max {ex.max():.2e} v max {ev.max():.2e}")
    assert ex.max() < TOL_F32 and ev.max() < TOL_F32
    X0, V0 = f32_inputs(w)
    inv0 = (oracle.energy_chain(w.m, w.k, X0, V0) if method == "rk4"
            else oracle.verlet_q_chain(w.m, w.k, w.dt, X0, V0))
    drift = np.abs(inv - inv0) / inv0
    print(f"two-mass per-step propagator {method}: invariant drift max {drift.max():.3e} "
          f"p99 {np.percentile(drift, 99):.3e}")
    assert drift.max() <= 1e-6


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("nsteps,stride", [(0, 10), (0, 0), (7, 100), (100, 100), (1, 0)])
def test_dense_frame_jumps_degenerate_runs(prec, nsteps, stride):
    """Frame jumps of s > 2 at the degenerate run lengths: no step (the
    caller's state comes back unchanged), a stride beyond the run (frame 0
    only, the end by the remainder power), a stride equal to the run, and a
    single step with no frames."""
    w = _dense(830 + nsteps, 3, 5, nsteps, stride)
    sysm = osc.System("dense", "rk4", prec, w.M, w.K, w.dt, shared=True, batch=3).create()
    try:
        got = _gpu_run(sysm, w, prec, 1)
    finally:
        sysm.close()
    if nsteps == 0:
        x0, v0 = f32_inputs(w) if prec == "f32" else (w.x0, w.v0)
        np.testing.assert_array_equal(got[2], x0)
        np.testing.assert_array_equal(got[3], v0)
    _check_traj(got, _oracle_for(w, "rk4", prec), 1e-6 if prec == "f32" else TOL_F64,
                f"dense jumps {prec} nsteps={nsteps} stride={stride}")
