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


@pytest.mark.parametrize("s,nsys", [(1, 1), (2, 1), (7, 1), (64, 1), (65, 1), (200, 1), (700, 1),
                                     (5, 4), (130, 3)])
def test_operator_matches_oracle_cholesky(s, nsys):
    """Blocked FP64 formation (64-wide panels: one block, a ragged second
    block, several blocks) against the oracle's unblocked Cholesky solve."""
    from paper_1702_02207_amd import osc
    w = _dense_batch(40 + s, s, max(nsys, 2), 10, 0, shared=nsys == 1)
    sysm = osc.System("dense", "rk4", "f64", w.M, w.K, w.dt, shared=nsys == 1, batch=max(nsys, 2)).create()
    A = sysm.dense_operator().cpu().numpy()
    sysm.sync()
    sysm.close()
    Ms = w.M.reshape(-1, s, s)
    Ks = w.K.reshape(-1, s, s)
    for b in range(Ms.shape[0]):
        ref = oracle.form_a(Ms[b], Ks[b])
        assert np.abs(A[b] - ref).max() <= 1e-12 * np.abs(ref).max(), b


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


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("shared", [True, False])
def test_dense_shadow_energy(prec, shared):
    """osc_shadow_energy on dense handles (Q = v'Mv + x'Kx - h^2/4 (Kx)'M^-1(Kx))
    against the oracle's dense invariant, shared and per-instance systems."""
    import torch
    from paper_1702_02207_amd import osc
    w = _dense_batch(11, 37, 5, 10, 0, shared=shared, vscale=1.0)
    w.dt = w.dt * 150.0            # h omega_max = 1.5: the correction term is a sizeable part of Q
    sysm = osc.System("dense", "verlet", prec, w.M, w.K, w.dt, shared=shared, batch=5).create()
    tdt = torch.float32 if prec == "f32" else torch.float64
    x = torch.as_tensor(w.x0, dtype=tdt, device="cuda")
    v = torch.as_tensor(w.v0, dtype=tdt, device="cuda")
    Q = sysm.energy(x, v, shadow=True).cpu().numpy()
    sysm.sync()
    sysm.close()
    ref = oracle.verlet_q_dense(w.M, w.K, w.dt, x.double().cpu().numpy(), v.double().cpu().numpy(),
                                shared=shared)
    np.testing.assert_allclose(Q, ref, rtol=1e-11)


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


def _run(sysm, w, nsteps, stride):
    import torch
    x0 = torch.as_tensor(w.x0, dtype=torch.float32, device="cuda")
    v0 = torch.as_tensor(w.v0, dtype=torch.float32, device="cuda")
    xf, vf, xe, ve = sysm.integrate(x0, v0, nsteps, stride)
    sysm.sync()
    return [t.double().cpu().numpy() for t in (xf, vf, xe, ve)]


@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("s,batch", [(3, 5), (64, 17), (100, 33), (200, 16), (256, 40)])
def test_dense_mfma_matches_oracle(method, s, batch):
    """Shared operator, FP32: the MFMA path (FP16 three-term products with
    FP32 accumulation) against the FP64 oracle."""
    from paper_1702_02207_amd import osc
    w = _dense_batch(300 + s, s, batch, 2000, 500, vscale=0.01)
    sysm = osc.System("dense", method, "f32", w.M, w.K, w.dt, shared=True, batch=batch).create()
    sysm.set_config(osc.CFG_DENSE_KERNEL, 2)
    xf, vf, xe, ve = _run(sysm, w, w.nsteps, w.out_stride)
    sysm.close()
    x0, v0 = f32_inputs(w)
    rx, rv, rxe, _ = oracle_dense(method, w, x0=x0, v0=v0)
    ex, ev = _err(xf, rx), _err(vf, rv)
    print(f"mfma {method} s={s}: x {ex.max():.2e} v {ev.max():.2e}")
    assert ex.max() < TOL_F32
    assert ev.max() < TOL_F32
    assert _err(xe, rxe).max() < TOL_F32


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_dense_mfma_and_valu_agree_and_chunking_is_bitwise(method):
    from paper_1702_02207_amd import osc
    w = _dense_batch(77, 130, 37, 900, 300, vscale=0.01)
    sysm = osc.System("dense", method, "f32", w.M, w.K, w.dt, shared=True, batch=37).create()
    whole = _run(sysm, w, 900, 300)
    sysm.set_config(osc.CFG_STEPS_PER_LAUNCH, 250)
    chunked = _run(sysm, w, 900, 300)
    for a, b in zip(whole, chunked):
        np.testing.assert_array_equal(a, b)
    sysm.set_config(osc.CFG_STEPS_PER_LAUNCH, 0)
    sysm.set_config(osc.CFG_DENSE_KERNEL, 1)
    valu = _run(sysm, w, 900, 300)
    sysm.close()
    assert _err(whole[0], valu[0]).max() < 2 * TOL_F32
    assert _err(whole[1], valu[1]).max() < 2 * TOL_F32


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("s,batch,shared", [(300, 1, True), (513, 2, False), (700, 1, True)])
def test_dense_split_matches_oracle(method, prec, s, batch, shared):
    """Large-s path: products split over row blocks and column groups of
    workgroups (ragged last group at s = 300 and 513), three kernels per
    step."""
    import torch
    from paper_1702_02207_amd import osc
    w = _dense_batch(500 + s, s, batch, 600, 100, shared=shared, vscale=0.01)
    tdt = torch.float32 if prec == "f32" else torch.float64
    sysm = osc.System("dense", method, prec, w.M, w.K, w.dt, shared=shared, batch=batch).create()
    sysm.set_config(osc.CFG_DENSE_KERNEL, 3)
    x0 = torch.as_tensor(w.x0, dtype=tdt, device="cuda")
    v0 = torch.as_tensor(w.v0, dtype=tdt, device="cuda")
    xf, vf, xe, ve = [t.double().cpu().numpy() for t in sysm.integrate(x0, v0, 600, 100)]
    sysm.sync()
    sysm.close()
    x0r, v0r = f32_inputs(w) if prec == "f32" else (w.x0, w.v0)
    rx, rv, rxe, rve = oracle_dense(method, w, x0=x0r, v0=v0r)
    tol = TOL_F32 if prec == "f32" else TOL_F64
    assert _err(xf, rx).max() < tol
    assert _err(vf, rv).max() < tol
    assert _err(xe, rxe).max() < tol
    assert _err(ve, rve).max() < tol


@pytest.mark.parametrize("kernel", [1, 2, 3])
@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_rest_state_stays_at_rest(method, kernel):
    """An instance at rest (x0 = v0 = 0) among moving ones stays exactly at
    rest on every dense kernel (the MFMA path's per-instance scale falls back
    to 1 for an all-zero state); the others match the oracle."""
    import torch
    from paper_1702_02207_amd import osc
    w = _dense_batch(77, 64, 20, 300, 100, vscale=0.01)
    w.x0[3] = 0.0
    w.v0[3] = 0.0
    sysm = osc.System("dense", method, "f32", w.M, w.K, w.dt, shared=True, batch=20).create()
    sysm.set_config(osc.CFG_DENSE_KERNEL, kernel)
    x0 = torch.as_tensor(w.x0, dtype=torch.float32, device="cuda")
    v0 = torch.as_tensor(w.v0, dtype=torch.float32, device="cuda")
    xf, vf, xe, ve = [t.double().cpu().numpy() for t in sysm.integrate(x0, v0, w.nsteps, w.out_stride)]
    sysm.sync()
    sysm.close()
    assert not xf[:, 3].any() and not vf[:, 3].any() and not xe[3].any() and not ve[3].any()
    x0r, v0r = f32_inputs(w)
    rx, rv, _, _ = oracle_dense(method, w, x0=x0r, v0=v0r)
    keep = [b for b in range(20) if b != 3]
    assert _err(xf[:, keep], rx[:, keep]).max() < TOL_F32
    assert _err(vf[:, keep], rv[:, keep]).max() < TOL_F32


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_dense_largest_size_against_modal_solution(method):
    """s = 2048, the largest size the library takes: formation of A and the
    automatic kernel choice (the split path, sixteen column groups), 200
    steps with frames, against the exact discrete solution of the scheme per
    normal mode (LAPACK eigh of (K, M); the same closed form pins the FP64
    oracle, whose unblocked Cholesky alone needs minutes at this size)."""
    from oracle import closed_form as cf
    w = _dense_batch(2701, 2048, 1, 200, 50, shared=True, vscale=0.01)
    xf, vf, xe, ve = gpu_dense(method, "f32", w)
    x0, v0 = f32_inputs(w)
    n = np.arange(0, 201, 50)
    exact = cf.rk4_discrete if method == "rk4" else cf.verlet_discrete
    rx, rv = exact(n, w.dt[0], w.M, w.K, x0[0], v0[0])
    assert _err(xf, rx[:, None, :]).max() < TOL_F32
    assert _err(vf, rv[:, None, :]).max() < TOL_F32
    np.testing.assert_array_equal(xf[-1], xe)


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_dense_split_graph_replays_match_eager(method):
    """Every replay of the captured step graph, with other eager GPU work and
    synchronisations in between, equals the eagerly launched run bitwise."""
    import torch
    from paper_1702_02207_amd import osc
    w = _dense_batch(901, 320, 2, 100, 10, shared=False, vscale=0.01)
    sysm = osc.System("dense", method, "f32", w.M, w.K, w.dt, shared=False, batch=2,
                      stream=torch.cuda.current_stream()).create()
    sysm.set_config(osc.CFG_DENSE_KERNEL, 3)
    x0 = torch.as_tensor(w.x0, dtype=torch.float32, device="cuda")
    v0 = torch.as_tensor(w.v0, dtype=torch.float32, device="cuda")
    sysm.set_config(osc.CFG_GRAPH_STEPS, 0)
    ref = [t.cpu().numpy() for t in sysm.integrate(x0, v0, 100, 10)]
    sysm.set_config(osc.CFG_GRAPH_STEPS, 16)
    out = [torch.empty_like(t) for t in (torch.empty((11, 2, 320)), torch.empty((11, 2, 320)))]
    xf = torch.empty((11, 2, 320), dtype=torch.float32, device="cuda")
    vf = torch.empty_like(xf)
    xe, ve = torch.empty_like(x0), torch.empty_like(v0)
    for rep in range(4):
        junk = torch.randn(1 << 20, device="cuda")
        junk = (junk * 2.0).sum()                       # eager work between replays
        torch.cuda.synchronize()
        sysm.integrate(x0, v0, 100, 10, out=(xf, vf, xe, ve))
        sysm.sync()
        got = [t.cpu().numpy() for t in (xf, vf, xe, ve)]
        for a, b in zip(ref, got):
            np.testing.assert_array_equal(a, b)
    sysm.close()


def test_per_instance_stability_check_covers_every_system():
    """An unstable step on any one of several per-instance systems is rejected."""
    from paper_1702_02207_amd import osc
    M = np.stack([np.eye(3)] * 3)
    K = np.stack([np.diag([1.0, 4.0, 9.0])] * 3)
    dt = np.array([0.01, 0.01, 5.0])          # h omega = 15 for the last system
    with pytest.raises(osc.OscError) as e:
        osc.System("dense", "rk4", "f32", M, K, dt, shared=False).create()
    assert e.value.status == osc.OSC_EUNSTABLE


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_dense_split_sixteen_groups_on_a_stream(method):
    """s = 1024 (the most column groups: 16 of 64 columns), one instance, on
    a stream of its own so that 64-step chunks replay a captured graph: 200
    steps = three replays and 8 eager steps."""
    import torch
    from paper_1702_02207_amd import osc
    s = 1024
    w = _dense_batch(1024, s, 1, 200, 50, shared=True, vscale=0.01)
    st = torch.cuda.Stream()
    sysm = osc.System("dense", method, "f32", w.M, w.K, w.dt, shared=True, batch=1, stream=st).create()
    x0 = torch.as_tensor(w.x0, dtype=torch.float32, device="cuda")
    v0 = torch.as_tensor(w.v0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    xf, vf, xe, ve = sysm.integrate(x0, v0, 200, 50)
    sysm.sync()
    xf, vf, xe, ve = [t.double().cpu().numpy() for t in (xf, vf, xe, ve)]
    sysm.close()
    x0r, v0r = f32_inputs(w)
    rx, rv, rxe, rve = oracle_dense(method, w, x0=x0r, v0=v0r)
    assert _err(xf, rx).max() < TOL_F32
    assert _err(vf, rv).max() < TOL_F32
    assert _err(xe, rxe).max() < TOL_F32
    assert _err(ve, rve).max() < TOL_F32


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_mfma_misaligned_buffers_give_identical_results(method):
    """The MFMA kernel moves four rows at a time as 16-byte vectors only when
    aligned; buffers offset by one float must give the same bits."""
    import torch
    from paper_1702_02207_amd import osc

    def misaligned_like(t):
        buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=t.device)
        out = buf[1:].view(t.shape)
        out.copy_(t)
        return out

    w = _dense_batch(91, 64, 20, 300, 100, vscale=0.01)
    sysm = osc.System("dense", method, "f32", w.M, w.K, w.dt, shared=True, batch=20).create()
    sysm.set_config(osc.CFG_DENSE_KERNEL, 2)
    x0 = torch.as_tensor(w.x0, dtype=torch.float32, device="cuda")
    v0 = torch.as_tensor(w.v0, dtype=torch.float32, device="cuda")
    ref = [t.cpu().numpy() for t in sysm.integrate(x0, v0, 300, 100)]
    frames = torch.zeros((4, 20, 64), device="cuda")
    outs = (misaligned_like(frames), misaligned_like(frames), misaligned_like(x0), misaligned_like(v0))
    got = [t.cpu().numpy() for t in sysm.integrate(misaligned_like(x0), misaligned_like(v0), 300, 100, out=outs)]
    sysm.sync()
    sysm.close()
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("prec,shared", [("f32", True), ("f64", True), ("f32", False)])
def test_plain_dense_matches_valu_path_and_oracle(method, prec, shared):
    """osc_integrate_plain on dense systems (one instance at a time, one step
    per launch, state in device memory) equals the VALU integrator bitwise
    (its compensated state survives every launch boundary) and the oracle at
    the precision's tolerance; zero steps copy the input."""
    import torch
    from paper_1702_02207_amd import osc
    w = _dense_batch(41, 45, 3, 300, 0, shared=shared, vscale=0.3)
    tdt = torch.float32 if prec == "f32" else torch.float64
    sysm = osc.System("dense", method, prec, w.M, w.K, w.dt, shared=shared, batch=3).create()
    sysm.set_config(osc.CFG_DENSE_KERNEL, 1)
    x0 = torch.as_tensor(w.x0, dtype=tdt, device="cuda")
    v0 = torch.as_tensor(w.v0, dtype=tdt, device="cuda")
    _, _, xe, ve = sysm.integrate(x0, v0, w.nsteps, 0)
    xp, vp = sysm.integrate_plain(x0, v0, w.nsteps)
    x00, v00 = sysm.integrate_plain(x0, v0, 0)
    sysm.sync()
    sysm.close()
    np.testing.assert_array_equal(xp.cpu().numpy(), xe.cpu().numpy())
    np.testing.assert_array_equal(vp.cpu().numpy(), ve.cpu().numpy())
    np.testing.assert_array_equal(x00.cpu().numpy(), x0.cpu().numpy())
    np.testing.assert_array_equal(v00.cpu().numpy(), v0.cpu().numpy())
    xi, vi = (f32_inputs(w) if prec == "f32" else (w.x0, w.v0))
    _, _, rxe, rve = oracle_dense(method, w, x0=xi, v0=vi, stride=0)
    tol = TOL_F32 if prec == "f32" else TOL_F64
    assert _err(xp.double().cpu().numpy(), rxe).max() < tol
    assert _err(vp.double().cpu().numpy(), rve).max() < tol
