"""GPU parity of damped and driven systems (eq. (1) with Rayleigh damping and
a harmonic force, classic RK4 on the first-order form of section 3) against
the FP64 oracle, through the C ABI; the adaptive Dormand-Prince reference and
the exact modal solution beside it."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import closed_form as cf
from paper_1702_02207_amd import osc, workloads
from gpu_util import to_dev, f32_inputs

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-10}


def _chain_case(seed, batch, s, nsteps, stride, force=True):
    rng = np.random.default_rng(seed)
    m, k = workloads.random_chain(rng, batch, s)
    wmax = workloads.chain_omega_max(m, k)
    dt = 0.01 / wmax
    x0 = rng.normal(0.0, 0.1, (batch, s))
    v0 = rng.normal(0.0, 1.0, (batch, s)) * 0.05
    F = rng.normal(0.0, 1.0, (batch, s)) * 50.0 if force else None
    W = rng.uniform(0.5, 2.0, batch) * 10.0 if force else None
    alpha, beta = 0.3, 2e-4
    return workloads.ChainBatch(m, k, dt, x0, v0, nsteps, stride), alpha, beta, F, W


def _dense_case(seed, batch, s, nsteps, stride, shared=True, force=True):
    rng = np.random.default_rng(seed)
    if shared:
        M, K = workloads.random_dense_system(rng, s)
        dt = np.array([0.01 / workloads.dense_omega_max(M, K)])
    else:
        Ms, Ks = zip(*[workloads.random_dense_system(rng, s) for _ in range(batch)])
        M, K = np.array(Ms), np.array(Ks)
        dt = np.array([0.01 / workloads.dense_omega_max(M[b], K[b]) for b in range(batch)])
    x0 = rng.normal(0.0, 1.0, (batch, s))
    v0 = rng.normal(0.0, 1.0, (batch, s)) * 0.01
    F = rng.normal(0.0, 1.0, (batch, s)) if force else None
    W = rng.uniform(0.2, 1.0, batch) if force else None
    return workloads.DenseBatch(M, K, dt, x0, v0, nsteps, stride, shared), 0.02, 0.05, F, W


def _run(sysm, w, prec, alpha, beta, F, W, steps_per_launch=0, static=False):
    import torch
    dtype = torch.float32 if prec == "f32" else torch.float64
    sysm.set_excitation(alpha, beta, F, W)
    if steps_per_launch:
        sysm.set_config(osc.CFG_STEPS_PER_LAUNCH, steps_per_launch)
    x0, v0 = to_dev(w.x0, dtype), to_dev(w.v0, dtype)
    out = sysm.integrate(x0, v0, w.nsteps, w.out_stride, static=static)
    sysm.sync()
    return [t.double().cpu().numpy() for t in out]


def _errs(got, ref):
    return (oracle.rel_traj_err(got[0], ref[0]).max(), oracle.rel_traj_err(got[1], ref[1]).max())


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("s,batch", [(1, 20), (2, 64), (7, 9), (256, 4), (300, 3), (1024, 2), (2048, 2)])
def test_driven_chain_matches_oracle(prec, s, batch):
    w, alpha, beta, F, W = _chain_case(900 + s, batch, s, 1500, 250)
    sysm = osc.System("chain", "rk4", prec, w.m, w.k, w.dt).create()
    try:
        got = _run(sysm, w, prec, alpha, beta, F, W)
    finally:
        sysm.close()
    x0, v0 = f32_inputs(w) if prec == "f32" else (w.x0, w.v0)
    ref = oracle.chain_driven(w.m, w.k, w.dt, alpha, beta, F, W, x0, v0, w.nsteps, w.out_stride)
    ex, ev = _errs(got, ref)
    print(f"driven chain {prec} s={s}: x {ex:.2e} v {ev:.2e}")
    assert ex < TOL[prec] and ev < TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("s,batch,shared", [(1, 4, True), (3, 5, True), (64, 6, True), (200, 3, True),
                                            (5, 4, False)])
def test_driven_dense_matches_oracle(prec, s, batch, shared):
    w, alpha, beta, F, W = _dense_case(920 + s, batch, s, 1200, 200, shared=shared)
    sysm = osc.System("dense", "rk4", prec, w.M, w.K, w.dt, shared=shared, batch=batch).create()
    try:
        got = _run(sysm, w, prec, alpha, beta, F, W)
    finally:
        sysm.close()
    x0, v0 = f32_inputs(w) if prec == "f32" else (w.x0, w.v0)
    ref = oracle.dense_driven(w.M, w.K, w.dt, alpha, beta, F, W, x0, v0, w.nsteps, w.out_stride, shared=shared)
    ex, ev = _errs(got, ref)
    print(f"driven dense {prec} s={s} shared={shared}: x {ex:.2e} v {ev:.2e}")
    assert ex < TOL[prec] and ev < TOL[prec]


@pytest.mark.parametrize("kind", ["chain", "dense"])
def test_damping_alone_and_force_alone(kind):
    """Each term on its own: damping without a force, a force without damping."""
    for alpha, beta, force in ((0.5, 1e-3, False), (0.0, 0.0, True)):
        if kind == "chain":
            w, _, _, F, W = _chain_case(940, 8, 40, 1000, 200, force=force)
            sysm = osc.System("chain", "rk4", "f32", w.m, w.k, w.dt).create()
        else:
            w, _, _, F, W = _dense_case(941, 5, 30, 1000, 200, force=force)
            sysm = osc.System("dense", "rk4", "f32", w.M, w.K, w.dt, shared=True, batch=5).create()
        try:
            got = _run(sysm, w, "f32", alpha, beta, F, W)
        finally:
            sysm.close()
        x0, v0 = f32_inputs(w)
        if kind == "chain":
            ref = oracle.chain_driven(w.m, w.k, w.dt, alpha, beta, F, W, x0, v0, w.nsteps, w.out_stride)
        else:
            ref = oracle.dense_driven(w.M, w.K, w.dt, alpha, beta, F, W, x0, v0, w.nsteps, w.out_stride)
        ex, ev = _errs(got, ref)
        assert ex < 1e-5 and ev < 1e-5, (kind, alpha, force, ex, ev)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_driven_chunked_and_static_runs_are_bitwise_identical(prec):
    """Launch chunks end at step indices that are not multiples of the force
    phase's anchor period; the result does not change, nor through the
    allocation-free entry point."""
    w, alpha, beta, F, W = _chain_case(950, 16, 100, 1000, 125)
    sysm = osc.System("chain", "rk4", prec, w.m, w.k, w.dt).create()
    try:
        whole = _run(sysm, w, prec, alpha, beta, F, W)
        chunked = _run(sysm, w, prec, alpha, beta, F, W, steps_per_launch=77)
        static = _run(sysm, w, prec, alpha, beta, F, W, steps_per_launch=77, static=True)
    finally:
        sysm.close()
    for a, b, c in zip(whole, chunked, static):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)


def test_clearing_the_excitation_restores_the_free_integrator():
    import torch
    w, alpha, beta, F, W = _chain_case(960, 10, 12, 500, 100)
    sysm = osc.System("chain", "rk4", "f32", w.m, w.k, w.dt).create()
    try:
        x0, v0 = to_dev(w.x0, torch.float32), to_dev(w.v0, torch.float32)
        free = [t.cpu().numpy() for t in sysm.integrate(x0, v0, w.nsteps, w.out_stride)]
        sysm.set_excitation(alpha, beta, F, W)
        sysm.set_excitation(0.0, 0.0, None)
        again = [t.cpu().numpy() for t in sysm.integrate(x0, v0, w.nsteps, w.out_stride)]
        sysm.sync()
    finally:
        sysm.close()
    for a, b in zip(free, again):
        np.testing.assert_array_equal(a, b)


def test_fp32_gpu_agrees_with_the_adaptive_reference_and_the_exact_solution():
    """A damped chain driven near its lowest resonance, FP32 on the GPU at
    h omega_max = 0.01: within 1e-5 of the Dormand-Prince reference
    (rtol 1e-11) and of the exact modal solution at every frame."""
    import torch
    rng = np.random.default_rng(970)
    s = 5
    m, k = workloads.random_chain(rng, 1, s)
    M, K = cf.chain_matrices(m[0], k[0])
    w2 = scipy.linalg.eigh(K, M, eigvals_only=True)
    wmin, wmax = np.sqrt(w2[0]), np.sqrt(w2[-1])
    h = 0.01 / wmax
    nsteps, stride = 20000, 2000
    alpha, beta = 0.05 * wmin, 0.002 / wmax
    F = rng.normal(size=(1, s)) * 100.0
    Wf = 1.05 * wmin
    x0, v0 = rng.normal(0, 0.1, (1, s)), np.zeros((1, s))
    sysm = osc.System("chain", "rk4", "f32", m, k, np.array([h])).create()
    try:
        sysm.set_excitation(alpha, beta, F, [Wf])
        xf, vf, _, _ = sysm.integrate(to_dev(x0, torch.float32), to_dev(v0, torch.float32), nsteps, stride)
        sysm.sync()
        xf = xf.double().cpu().numpy()
    finally:
        sysm.close()
    X0 = x0.astype(np.float32).astype(np.float64)[0]
    t = np.arange(0, nsteps + 1, stride) * h
    xo, vo, acc, rej = oracle.dopri_driven("chain", m[0], k[0], alpha, beta, F[0], Wf, X0, v0[0], t[-1],
                                           len(t) - 1, 1e-11, 1e-13)
    xr, _ = cf.driven_modal_solution(t, M, K, alpha, beta, F[0], Wf, X0, v0[0])
    e_dopri = oracle.rel_traj_err(xf, xo[:, None, :])[0]
    e_exact = oracle.rel_traj_err(xf, xr[:, None, :])[0]
    print(f"driven FP32 vs Dormand-Prince {e_dopri:.2e} ({acc} steps), vs exact {e_exact:.2e}")
    assert e_dopri < 1e-5 and e_exact < 1e-5


def test_driven_error_returns():
    w, alpha, beta, F, W = _chain_case(980, 4, 6, 10, 0)
    sysm = osc.System("chain", "verlet", "f32", w.m, w.k, w.dt).create()
    try:
        with pytest.raises(osc.OscError) as e:
            sysm.set_excitation(alpha, beta, F, W)
        assert e.value.status == osc.OSC_ENOTSUP
    finally:
        sysm.close()
    sysm = osc.System("chain", "rk4", "f32", w.m, w.k, w.dt).create()
    try:
        with pytest.raises(osc.OscError) as e:        # h (alpha + beta w^2) far above 2.5
            sysm.set_excitation(0.0, 1e3, None)
        assert e.value.status == osc.OSC_EUNSTABLE
        with pytest.raises(osc.OscError) as e:
            sysm.set_excitation(-1.0, 0.0, None)
        assert e.value.status == osc.OSC_EINVAL
        sysm.set_excitation(alpha, beta, F, W)
        import torch
        x0 = to_dev(w.x0, torch.float32)
        with pytest.raises(osc.OscError) as e:
            sysm.integrate_plain(x0, x0, 10)
        assert e.value.status == osc.OSC_ENOTSUP
        sysm.set_config(osc.CFG_PROPAGATOR, 1)
        with pytest.raises(osc.OscError) as e:
            sysm.integrate(x0, x0, 10, 0)
        assert e.value.status == osc.OSC_ENOTSUP
    finally:
        sysm.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("s", [2, 37, 700, 1024])
def test_driven_chain_register_and_workgroup_kernels_agree(prec, s):
    """Chains of s <= 1024 run in registers (DPP halo); the one-workgroup
    kernel (OSC_CFG_DENSE_KERNEL = 1) computes the same scheme: both within
    the tolerance of the oracle and of each other."""
    w, alpha, beta, F, W = _chain_case(990 + s, 6, s, 800, 200)
    out = []
    for kern in (0, 1):
        sysm = osc.System("chain", "rk4", prec, w.m, w.k, w.dt).create()
        try:
            sysm.set_config(osc.CFG_DENSE_KERNEL, kern)
            out.append(_run(sysm, w, prec, alpha, beta, F, W))
        finally:
            sysm.close()
    x0, v0 = f32_inputs(w) if prec == "f32" else (w.x0, w.v0)
    ref = oracle.chain_driven(w.m, w.k, w.dt, alpha, beta, F, W, x0, v0, w.nsteps, w.out_stride)
    for got in out:
        ex, ev = _errs(got, ref)
        assert ex < TOL[prec] and ev < TOL[prec], (s, ex, ev)


@pytest.mark.parametrize("s,batch", [(37, 19), (256, 17)])
@pytest.mark.parametrize("terms", ["alpha", "beta", "force", "all"])
def test_driven_dense_matrix_cores_and_workgroup_kernel_agree(s, batch, terms):
    """A shared dense operator in FP32 runs damped, driven RK4 on the matrix
    cores (the four-level recursion, one kernel per combination of terms);
    OSC_CFG_DENSE_KERNEL = 1 takes the stage-form workgroup kernel instead.
    Both match the oracle within the FP32 tolerance, over ragged 16-instance
    tiles."""
    w, alpha, beta, F, W = _dense_case(960 + s, batch, s, 1500, 300)
    if terms == "alpha":
        beta, F, W = 0.0, None, None
    elif terms == "beta":
        alpha, F, W = 0.0, None, None
    elif terms == "force":
        alpha = beta = 0.0
    out = []
    for kern in (0, 1):
        sysm = osc.System("dense", "rk4", "f32", w.M, w.K, w.dt, shared=True, batch=batch).create()
        try:
            sysm.set_config(osc.CFG_DENSE_KERNEL, kern)
            out.append(_run(sysm, w, "f32", alpha, beta, F, W))
        finally:
            sysm.close()
    x0, v0 = f32_inputs(w)
    ref = oracle.dense_driven(w.M, w.K, w.dt, alpha, beta, F, W, x0, v0, w.nsteps, w.out_stride)
    for kern, got in zip((0, 1), out):
        ex, ev = _errs(got, ref)
        print(f"driven dense s={s} {terms} kernel {kern}: x {ex:.2e} v {ev:.2e}")
        assert ex < 1e-5 and ev < 1e-5, (kern, ex, ev)


def test_driven_dense_matrix_cores_chunked_and_static_are_bitwise_identical():
    w, alpha, beta, F, W = _dense_case(975, 20, 48, 1000, 125)
    sysm = osc.System("dense", "rk4", "f32", w.M, w.K, w.dt, shared=True, batch=20).create()
    try:
        whole = _run(sysm, w, "f32", alpha, beta, F, W)
        chunked = _run(sysm, w, "f32", alpha, beta, F, W, steps_per_launch=77)
        static = _run(sysm, w, "f32", alpha, beta, F, W, steps_per_launch=77, static=True)
    finally:
        sysm.close()
    for a, b, c in zip(whole, chunked, static):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)
