"""Pins of the FP64 oracle to what the paper and the mathematics fix.

Every check compares the oracle's C loops with something computed another way:
the paper's printed roots, closed forms derived from eq. (3)-(7), the exact
discrete solutions of RK4 and Verlet on the normal modes (LAPACK eigenpairs),
invariants and special cases.  None of them re-types the oracle's loops.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import closed_form as cf
from paper_1702_02207_amd import workloads


def _read_golden(path):
    vals = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, val = line.split()
        vals[key] = float(val)
    return vals


# ---------------------------------------------------------------- section 2 --

def test_eq6_roots_match_paper_print(golden_dir):
    g = _read_golden(os.path.join(golden_dir, "eq6_roots_paper.txt"))
    wf, ws = cf.eq6_omegas(g["m"], g["C"])
    assert abs(wf - g["omega_fast"]) / g["omega_fast"] < 5e-4
    assert abs(ws - g["omega_slow"]) / g["omega_slow"] < 5e-4


def test_eq6_roots_exact_values_and_residual():
    m, C = 2.0, 2025.0
    wf, ws = cf.eq6_omegas(m, C)
    # (C/m)(3 +- sqrt5)/2 written independently of the quadratic formula
    assert wf == pytest.approx(math.sqrt(C / m * (3 + math.sqrt(5)) / 2), rel=1e-14)
    assert ws == pytest.approx(math.sqrt(C / m * (3 - math.sqrt(5)) / 2), rel=1e-14)
    for w in (wf, ws):
        lam2 = -w * w
        res = m * m * lam2 ** 2 + 3 * m * C * lam2 + C * C
        assert abs(res) < 1e-9 * C * C


def test_eq6_matches_generalised_eigenproblem():
    m, C = 2.0, 2025.0
    M, K = cf.chain_matrices([m, m], [C, C])
    w = np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True))
    wf, ws = cf.eq6_omegas(m, C)
    np.testing.assert_allclose(np.sort(w), [ws, wf], rtol=1e-13)


def test_chain_matrices_reduce_to_eq2_and_eq3():
    m1, m2, c1, c2 = 1.5, 0.7, 300.0, 55.0
    M, K = cf.chain_matrices([m1, m2], [c1, c2])
    # eq. (2): m1 x1'' + C1 x1 - C2 (x2 - x1) = 0, m2 x2'' + C2 (x2 - x1) = 0
    np.testing.assert_array_equal(K, [[c1 + c2, -c2], [-c2, c2]])
    np.testing.assert_array_equal(M, np.diag([m1, m2]))


def test_eq4_mode_shapes():
    m, C = 2.0, 2025.0
    wf, ws = cf.eq6_omegas(m, C)
    rf, rs = cf.eq4_mode_ratio(m, C, wf), cf.eq4_mode_ratio(m, C, ws)
    assert rf == pytest.approx((1 - math.sqrt(5)) / 2, rel=1e-13)
    assert rs == pytest.approx((1 + math.sqrt(5)) / 2, rel=1e-13)
    # second row of eq. (4) holds for the same shape
    for w, r in ((wf, rf), (ws, rs)):
        assert abs(-C * 1.0 + (-m * w * w + C) * r) < 1e-9 * C


def test_uniform_chain_formula_matches_eigvals():
    for s in (1, 2, 3, 7, 16):
        M, K = cf.chain_matrices(np.full(s, 1.3), np.full(s, 410.0))
        w = np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True))
        np.testing.assert_allclose(w, cf.uniform_chain_omegas(s, 410.0, 1.3), rtol=1e-12)


def test_two_mass_closed_form_is_modal_superposition():
    """eq. (7) read as a modal superposition equals the eq. (3)/(4) closed form."""
    t = np.linspace(0, 1, 57)
    M, K = cf.chain_matrices([2.0, 2.0], [2025.0, 2025.0])
    for x0, v0 in (((1.0, 0.0), (0.0, 0.0)), ((2.0, -3.0), (0.5, 1.0))):
        xa, va = cf.two_mass_equal(t, 2.0, 2025.0, x0, v0)
        xb, vb = cf.modal_solution(t, M, K, x0, v0)
        np.testing.assert_allclose(xa, xb, atol=1e-12)
        np.testing.assert_allclose(va, vb, atol=1e-10)


# ---------------------------------------------------- C1: the paper's system --

@pytest.mark.parametrize("x0", [(1.0, 0.0), (2.0, -3.0)])
def test_c1_rk4_matches_closed_form(x0):
    """The paper's two-mass system, eq. (3): m = 2, C = 2025, dt = 1e-5, 1e5 RK4 steps in FP64;
    (2, -3) are the initial conditions of the paper's MATLAB run (section 3)."""
    w = workloads.c1_paper_two_mass(x0=x0, out_stride=100)
    xf, vf, xe, ve = oracle.chain("rk4", w.m, w.k, w.dt, w.x0, w.v0, w.nsteps, w.out_stride)
    t = np.arange(xf.shape[0]) * w.out_stride * w.dt[0]
    xa, va = cf.two_mass_equal(t, 2.0, 2025.0, x0, (0.0, 0.0))
    assert oracle.rel_traj_err(xf, xa[:, None, :])[0] < 1e-10
    assert oracle.rel_traj_err(vf, va[:, None, :])[0] < 1e-10
    np.testing.assert_array_equal(xf[-1], xe)
    if x0 == (1.0, 0.0):
        # t = 1 values of the closed form (x1, x2), written out independently:
        # x1 = (5+sqrt5)/10 cos wf t + (5-sqrt5)/10 cos ws t, x2 = (cos ws t - cos wf t)/sqrt5
        wf, ws = cf.eq6_omegas(2.0, 2025.0)
        s5 = math.sqrt(5)
        x1 = (5 + s5) / 10 * math.cos(wf) + (5 - s5) / 10 * math.cos(ws)
        x2 = (math.cos(ws) - math.cos(wf)) / s5
        np.testing.assert_allclose(xe[0], [x1, x2], rtol=0, atol=1e-10)
        E = oracle.energy_chain(w.m, w.k, w.x0, w.v0)
        assert E[0] == 2025.0


# ------------------------------------------------ exact discrete solutions ----

def _random_chain(rng, s):
    m = rng.uniform(0.5, 2.0, s)
    k = np.exp(rng.uniform(math.log(1e2), math.log(1e4), s))
    return m, k


@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("s", [1, 2, 3, 5, 8])
def test_chain_matches_discrete_closed_form(method, s):
    """At theta_max = w_max h = 0.5 the scheme differs from the exact flow by
    O(1e-3), so this pins the RK4 tableau / Verlet splitting, not just
    convergence."""
    rng = np.random.default_rng(100 + s)
    m, k = _random_chain(rng, s)
    M, K = cf.chain_matrices(m, k)
    wmax = np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True)[-1])
    h = 0.5 / wmax
    x0, v0 = rng.normal(size=s), rng.normal(size=s) * wmax
    n, stride = 300, 7
    xf, vf, _, _ = oracle.chain(method, m[None], k[None], [h], x0[None], v0[None], n, stride)
    steps = np.arange(0, n + 1, stride)
    ref = cf.rk4_discrete if method == "rk4" else cf.verlet_discrete
    xr, vr = ref(steps, h, M, K, x0, v0)
    assert oracle.rel_traj_err(xf, xr[:, None, :])[0] < 1e-11
    assert oracle.rel_traj_err(vf, vr[:, None, :])[0] < 1e-11
    exact_x, _ = cf.modal_solution(steps * h, M, K, x0, v0)
    assert oracle.rel_traj_err(xf, exact_x[:, None, :])[0] > 1e-5   # the scheme is visible


@pytest.mark.parametrize("method", ["rk4", "verlet"])
@pytest.mark.parametrize("s", [1, 2, 4, 6])
def test_dense_matches_discrete_closed_form(method, s):
    rng = np.random.default_rng(200 + s)
    M, K = workloads.random_dense_system(rng, s)
    wmax = np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True)[-1])
    h = 0.4 / wmax
    x0, v0 = rng.normal(size=(3, s)), rng.normal(size=(3, s))
    n, stride = 250, 25
    xf, vf, _, _ = oracle.dense(method, M, K, [h], x0, v0, n, stride)
    steps = np.arange(0, n + 1, stride)
    ref = cf.rk4_discrete if method == "rk4" else cf.verlet_discrete
    for b in range(3):
        xr, vr = ref(steps, h, M, K, x0[b], v0[b])
        assert oracle.rel_traj_err(xf[:, b:b + 1], xr[:, None, :])[0] < 1e-11
        assert oracle.rel_traj_err(vf[:, b:b + 1], vr[:, None, :])[0] < 1e-11


def test_dense_unshared_equals_per_instance_shared():
    rng = np.random.default_rng(7)
    s, B = 5, 3
    Ms, Ks = zip(*[workloads.random_dense_system(rng, s) for _ in range(B)])
    Ms, Ks = np.array(Ms), np.array(Ks)
    dt = np.array([0.01, 0.02, 0.015])
    x0, v0 = rng.normal(size=(B, s)), rng.normal(size=(B, s))
    _, _, xe, ve = oracle.dense("rk4", Ms, Ks, dt, x0, v0, 40, 0, shared=False)
    for b in range(B):
        _, _, xb, vb = oracle.dense("rk4", Ms[b], Ks[b], dt[b:b + 1], x0[b:b + 1], v0[b:b + 1], 40, 0)
        np.testing.assert_array_equal(xe[b], xb[0])
        np.testing.assert_array_equal(ve[b], vb[0])


def test_chain_as_dense_agrees():
    rng = np.random.default_rng(11)
    s = 6
    m, k = _random_chain(rng, s)
    M, K = cf.chain_matrices(m, k)
    x0, v0 = rng.normal(size=(1, s)), np.zeros((1, s))
    h = 1e-3
    for method in ("rk4", "verlet"):
        _, _, xc, vc = oracle.chain(method, m[None], k[None], [h], x0, v0, 500, 0)
        _, _, xd, vd = oracle.dense(method, M, K, [h], x0, v0, 500, 0)
        np.testing.assert_allclose(xc, xd, rtol=0, atol=1e-12 * np.abs(xc).max())
        np.testing.assert_allclose(vc, vd, rtol=0, atol=1e-12 * np.abs(vc).max())


# ------------------------------------------------------ A = M^-1 K ----------

def test_form_a_solves_m_a_equals_k():
    rng = np.random.default_rng(5)
    for s in (1, 2, 9, 33):
        M, K = workloads.random_dense_system(rng, s)
        A = oracle.form_a(M, K)
        np.testing.assert_allclose(M @ A, K, rtol=0, atol=1e-12 * np.abs(K).max())
        np.testing.assert_allclose(A, np.linalg.solve(M, K), rtol=0, atol=1e-11 * np.abs(A).max())


def test_form_a_rejects_non_spd():
    M = np.array([[1.0, 2.0], [2.0, 1.0]])       # eigenvalues 3, -1
    with pytest.raises(oracle.OracleError, match="status 2"):
        oracle.form_a(M, np.eye(2))


# ------------------------------------------------------ invariants ----------

def test_verlet_shadow_invariant_conserved():
    rng = np.random.default_rng(3)
    s = 12
    m, k = _random_chain(rng, s)
    M, K = cf.chain_matrices(m, k)
    wmax = np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True)[-1])
    h = 0.3 / wmax
    x0, v0 = rng.normal(size=(1, s)), rng.normal(size=(1, s)) * wmax
    xf, vf, _, _ = oracle.chain("verlet", m[None], k[None], [h], x0, v0, 2000, 50)
    Q = np.array([oracle.verlet_q_chain(m[None], k[None], [h], xf[f], vf[f])[0] for f in range(len(xf))])
    E = np.array([oracle.energy_chain(m[None], k[None], xf[f], vf[f])[0] for f in range(len(xf))])
    assert np.abs(Q / Q[0] - 1).max() < 1e-12
    assert np.abs(E / E[0] - 1).max() > 1e-4       # plain E is not the conserved quantity


def _dense_system(seed, s):
    rng = np.random.default_rng(seed)
    M, K = workloads.random_dense_system(rng, s)
    wmax = np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True)[-1])
    return rng, M, K, wmax


def test_verlet_shadow_invariant_dense_conserved():
    """Q = v'Mv + x'Kx - (h^2/4)(Kx)'M^-1(Kx) stays constant along the oracle's
    own dense Verlet trajectory while the plain energy does not."""
    rng, M, K, wmax = _dense_system(31, 9)
    h = 0.3 / wmax
    x0, v0 = rng.normal(size=(2, 9)), rng.normal(size=(2, 9)) * wmax
    xf, vf, _, _ = oracle.dense("verlet", M, K, [h], x0, v0, 2000, 50)
    Q = np.array([oracle.verlet_q_dense(M, K, [h], xf[f], vf[f]) for f in range(len(xf))])
    E = np.array([oracle.energy_dense(M, K, xf[f], vf[f]) for f in range(len(xf))])
    assert np.abs(Q / Q[0] - 1).max() < 1e-12
    assert np.abs(E / E[0] - 1).max() > 1e-4


def test_verlet_shadow_invariant_dense_modal_form():
    """With M-orthonormal modes (q = phi'Mx, p = phi'Mv), Q is the sum over
    modes of p^2 + w^2 q^2 (1 - (w h)^2 / 4): LAPACK eigenpairs, not the
    oracle's Cholesky route.  Per-instance systems give the same as shared."""
    rng, M, K, wmax = _dense_system(32, 7)
    h = 0.7 / wmax
    x, v = rng.normal(size=(3, 7)), rng.normal(size=(3, 7))
    w, phi = cf.modes(M, K)
    q, p = x @ M @ phi, v @ M @ phi
    ref = np.sum(p ** 2 + (w * q) ** 2 * (1.0 - (w * h) ** 2 / 4.0), axis=1)
    got = oracle.verlet_q_dense(M, K, [h], x, v)
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    got_pi = oracle.verlet_q_dense(np.stack([M] * 3), np.stack([K] * 3), [h] * 3, x, v, shared=False)
    np.testing.assert_allclose(got_pi, ref, rtol=1e-12)


def test_verlet_shadow_invariant_dense_equals_chain_form():
    rng = np.random.default_rng(33)
    s = 11
    m, k = _random_chain(rng, s)
    M, K = cf.chain_matrices(m, k)
    h = 0.5 / np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True)[-1])
    x, v = rng.normal(size=(2, s)), rng.normal(size=(2, s))
    Qc = oracle.verlet_q_chain(np.tile(m, (2, 1)), np.tile(k, (2, 1)), [h, h], x, v)
    Qd = oracle.verlet_q_dense(M, K, [h], x, v)
    np.testing.assert_allclose(Qd, Qc, rtol=1e-12)


Q_MUTANTS = [
    ("Q[b] = kin + pot - 0.25 * h * h * corr;", "Q[b] = kin + pot + 0.25 * h * h * corr;"),   # sign
    ("Q[b] = kin + pot - 0.25 * h * h * corr;", "Q[b] = kin + pot - 0.5 * h * h * corr;"),    # factor
    ("ai += A[(size_t)i * s + j] * xb[j];", "ai += A[(size_t)j * s + i] * xb[j];"),           # transposed A
    ("fi += Kb[(size_t)i * s + j] * xb[j];", "fi += Mb[(size_t)i * s + j] * xb[j];"),         # wrong matrix
]


@pytest.mark.parametrize("orig,mut", Q_MUTANTS)
def test_pins_catch_planted_dense_invariant_mistakes(orig, mut, tmp_path):
    """Recompile the oracle with one plausible mistake in the dense invariant
    and check that the modal closed form rejects it (CPU only)."""
    src = open(os.path.join(os.path.dirname(oracle.__file__), "osc_oracle.c")).read()
    assert orig in src
    mpath = tmp_path / "mut.c"
    mpath.write_text(src.replace(orig, mut))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(lib), str(mpath), "-lm"], check=True)
    import ctypes
    L = ctypes.CDLL(str(lib))
    d = ctypes.POINTER(ctypes.c_double)
    L.oracle_verlet_q_dense.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, d, d, d, d, d, d]
    rng, M, K, wmax = _dense_system(34, 6)
    h = 0.7 / wmax
    x, v = rng.normal(size=(1, 6)), rng.normal(size=(1, 6))
    w, phi = cf.modes(M, K)
    q, p = x @ M @ phi, v @ M @ phi
    ref = np.sum(p ** 2 + (w * q) ** 2 * (1.0 - (w * h) ** 2 / 4.0), axis=1)
    args = [np.ascontiguousarray(a, dtype=np.float64) for a in (M, K, [h], x, v)]
    Q = np.empty(1)
    L.oracle_verlet_q_dense(1, 6, 1, *[a.ctypes.data_as(d) for a in args], Q.ctypes.data_as(d))
    assert not np.allclose(Q, ref, rtol=1e-12), "planted mistake not detected"


def test_rk4_energy_decay_matches_amplification():
    rng = np.random.default_rng(4)
    s = 4
    m, k = _random_chain(rng, s)
    M, K = cf.chain_matrices(m, k)
    w, phi = cf.modes(M, K)
    h = 0.6 / w[-1]
    x0, v0 = rng.normal(size=s), rng.normal(size=s)
    n = 400
    _, _, xe, ve = oracle.chain("rk4", m[None], k[None], [h], x0[None], v0[None], n, 0)
    E = oracle.energy_chain(m[None], k[None], xe, ve)[0]
    q0, p0 = phi.T @ M @ x0, phi.T @ M @ v0
    E_ref = 0.5 * np.sum((p0 ** 2 + (w * q0) ** 2) * cf.rk4_energy_factor(w * h) ** n)
    assert E == pytest.approx(E_ref, rel=1e-12)
    # the factor formula itself: |R(-i th)|^2
    th = np.array([0.01, 0.1, 0.5, 1.0])
    np.testing.assert_allclose(np.abs(cf.rk4_amplification(th)) ** 2, cf.rk4_energy_factor(th), rtol=1e-15)


def test_energy_matches_quadratic_forms():
    rng = np.random.default_rng(8)
    s = 7
    m, k = _random_chain(rng, s)
    M, K = cf.chain_matrices(m, k)
    x, v = rng.normal(size=(2, s)), rng.normal(size=(2, s))
    E = oracle.energy_chain(np.tile(m, (2, 1)), np.tile(k, (2, 1)), x, v)
    Ed = oracle.energy_dense(M, K, x, v)
    ref = 0.5 * np.einsum("bi,ij,bj->b", v, M, v) + 0.5 * np.einsum("bi,ij,bj->b", x, K, x)
    np.testing.assert_allclose(E, ref, rtol=1e-13)
    np.testing.assert_allclose(Ed, ref, rtol=1e-13)


def test_verlet_time_reversal():
    rng = np.random.default_rng(9)
    s = 10
    m, k = _random_chain(rng, s)
    x0, v0 = rng.normal(size=(1, s)), rng.normal(size=(1, s))
    h = 1e-3
    _, _, x1, v1 = oracle.chain("verlet", m[None], k[None], [h], x0, v0, 1000, 0)
    _, _, x2, v2 = oracle.chain("verlet", m[None], k[None], [-h], x1, v1, 1000, 0)
    np.testing.assert_allclose(x2, x0, atol=1e-10)
    np.testing.assert_allclose(v2, v0, atol=1e-8)


def test_decoupled_springs_reduce_to_scalar_oscillator_and_free_mass():
    """C2 = 0 in eq. (2): body 1 is a scalar oscillator, body 2 moves freely.
    RK4 integrates uniform motion exactly, and body 1 follows R(-i w h)^n."""
    m1, m2, c1 = 1.7, 0.9, 800.0
    w = math.sqrt(c1 / m1)
    h = 0.2 / w
    x0, v0 = np.array([[0.3, -1.0]]), np.array([[2.0, 0.25]])
    n = 123
    _, _, xe, ve = oracle.chain("rk4", [[m1, m2]], [[c1, 0.0]], [h], x0, v0, n, 0)
    assert xe[0, 1] == pytest.approx(-1.0 + 0.25 * n * h, rel=1e-14)
    assert ve[0, 1] == 0.25
    u = (w * 0.3 + 2.0j) * cf.rk4_amplification(w * h) ** n
    assert xe[0, 0] == pytest.approx(u.real / w, rel=1e-12)
    assert ve[0, 0] == pytest.approx(u.imag, rel=1e-12)


def test_linearity():
    rng = np.random.default_rng(12)
    s = 5
    m, k = _random_chain(rng, s)
    xa, xb = rng.normal(size=(2, 1, s))
    va, vb = rng.normal(size=(2, 1, s))
    h = 2e-3
    _, _, ea, fa = oracle.chain("rk4", m[None], k[None], [h], xa, va, 200, 0)
    _, _, eb, fb = oracle.chain("rk4", m[None], k[None], [h], xb, vb, 200, 0)
    _, _, ec, fc = oracle.chain("rk4", m[None], k[None], [h], 2 * xa - 3 * xb, 2 * va - 3 * vb, 200, 0)
    np.testing.assert_allclose(ec, 2 * ea - 3 * eb, atol=1e-11)
    np.testing.assert_allclose(fc, 2 * fa - 3 * fb, atol=1e-9)


# ------------------------------------------------------ conventions --------

def test_frames_and_zero_steps():
    rng = np.random.default_rng(13)
    m, k = _random_chain(rng, 3)
    x0, v0 = rng.normal(size=(2, 3)), rng.normal(size=(2, 3))
    mm, kk = np.tile(m, (2, 1)), np.tile(k, (2, 1))
    xf, vf, xe, ve = oracle.chain("rk4", mm, kk, [1e-3, 2e-3], x0, v0, 10, 3)
    assert xf.shape == (4, 2, 3)                   # frames at n = 0, 3, 6, 9
    np.testing.assert_array_equal(xf[0], x0)
    _, _, x9, _ = oracle.chain("rk4", mm, kk, [1e-3, 2e-3], x0, v0, 9, 0)
    np.testing.assert_array_equal(xf[3], x9)
    xf0, _, xe0, ve0 = oracle.chain("verlet", mm, kk, [1e-3, 2e-3], x0, v0, 0, 1)
    np.testing.assert_array_equal(xe0, x0)
    np.testing.assert_array_equal(ve0, v0)
    assert xf0.shape == (1, 2, 3)


def test_empty_batch():
    xf, vf, xe, ve = oracle.chain("rk4", np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0),
                                  np.zeros((0, 4)), np.zeros((0, 4)), 10, 2)
    assert xe.shape == (0, 4) and xf.shape == (6, 0, 4)


# ------------------------------------------- planted mistakes are caught -----

MUTANTS = [
    ("2.0 * k2x[i]", "1.0 * k2x[i]"),                       # wrong RK4 weight
    ("x[i] + 0.5 * h * k2x[i]", "x[i] + 0.5 * h * k1x[i]"),  # wrong stage slope
    ("f += k[i + 1] * (x[i + 1] - x[i])", "f -= k[i + 1] * (x[i + 1] - x[i])"),  # sign
    ("(i == 0) ? x[0] : x[i] - x[i - 1]", "(i == 0) ? x[0] : x[i] - x[i]"),     # index
    ("x[i] += h * v[i];         /* drift */", "x[i] += h * a[i];         /* drift */"),
]


@pytest.mark.parametrize("orig,mut", MUTANTS)
def test_pins_catch_planted_oracle_mistakes(orig, mut, tmp_path):
    """Recompile the oracle with one plausible mistake and check that the
    discrete closed-form pin rejects it (CPU only)."""
    src = open(os.path.join(os.path.dirname(oracle.__file__), "osc_oracle.c")).read()
    assert orig in src
    mpath = tmp_path / "mut.c"
    mpath.write_text(src.replace(orig, mut))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(lib), str(mpath), "-lm"], check=True)
    import ctypes
    L = ctypes.CDLL(str(lib))
    d = ctypes.POINTER(ctypes.c_double)
    L.oracle_chain.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, d, d, d, d, d,
                               ctypes.c_int64, ctypes.c_int64, d, d, d, d]
    rng = np.random.default_rng(21)
    s = 4
    m, k = _random_chain(rng, s)
    M, K = cf.chain_matrices(m, k)
    wmax = np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True)[-1])
    h = 0.3 / wmax
    x0, v0 = rng.normal(size=s), rng.normal(size=s) * wmax
    n = 50
    bad = False
    for meth, ref in ((0, cf.rk4_discrete), (1, cf.verlet_discrete)):
        xe, ve = np.empty((1, s)), np.empty((1, s))
        p = lambda a: np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(d)
        args = [np.ascontiguousarray(a, dtype=np.float64) for a in (m[None], k[None], [h], x0[None], v0[None])]
        L.oracle_chain(meth, 1, s, *[p(a) for a in args], n, 0, None, None, p(xe), p(ve))
        xr, vr = ref([n], h, M, K, x0, v0)
        err = max(oracle.rel_traj_err(xe, xr)[0], oracle.rel_traj_err(ve, vr)[0])
        bad = bad or not (err < 1e-11)
    assert bad, "planted mistake not detected"


# ------------------------------------------------ the scheme as a matrix -----

def _first_order_matrix(M, K):
    """L = [[0, I], [-A, 0]] of section 3's first-order system, A = M^-1 K
    by a LAPACK solve (not the oracle's Cholesky)."""
    s = M.shape[0]
    A = scipy.linalg.solve(M, K)
    L = np.zeros((2 * s, 2 * s))
    L[:s, s:] = np.eye(s)
    L[s:, :s] = -A
    return L


@pytest.mark.parametrize("kind,s", [("chain", 1), ("chain", 2), ("chain", 5), ("dense", 3), ("dense", 6)])
def test_rk4_propagator_is_degree4_taylor_polynomial(kind, s):
    """Classic RK4 on y' = L y is exactly sum_{j<=4} (hL)^j / j! (the stage
    form's algebra); the oracle's matrix, formed by stepping unit vectors,
    matches it at h omega_max = 0.5, where higher terms would be visible."""
    rng = np.random.default_rng(600 + s)
    if kind == "chain":
        a, b = _random_chain(rng, s)
        M, K = cf.chain_matrices(a, b)
    else:
        M, K = workloads.random_dense_system(rng, s)
        a, b = M, K
    wmax = np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True)[-1])
    h = 0.5 / wmax
    P = oracle.propagator("rk4", kind, a, b, h, 1)
    hL = h * _first_order_matrix(M, K)
    T = np.eye(2 * s)
    term = np.eye(2 * s)
    for j in range(1, 5):
        term = term @ hL / j
        T = T + term
    scale = np.abs(T).max()
    assert np.abs(P - T).max() <= 1e-13 * scale
    # the fifth-order term is not there (it would be at this step size)
    assert np.abs(P - (T + term @ hL / 5)).max() > 1e-4 * scale


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_propagator_eigenvalues_are_the_modal_amplification(method):
    """On each normal mode (LAPACK eigh(K, M)) one step multiplies by
    R(+-i theta) (RK4) or e^{+-i phi} with cos phi = 1 - theta^2/2 (Verlet),
    theta = omega h."""
    rng = np.random.default_rng(610)
    s = 6
    m, k = _random_chain(rng, s)
    M, K = cf.chain_matrices(m, k)
    w = np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True))
    h = 0.6 / w[-1]
    P = oracle.propagator(method, "chain", m, k, h, 1)
    th = w * h
    if method == "rk4":
        z = 1j * th
        lam = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    else:
        lam = np.exp(1j * np.arccos(1 - th ** 2 / 2))
        assert np.linalg.det(P) == pytest.approx(1.0, abs=1e-12)   # area-preserving
    ref = np.concatenate([lam, lam.conj()])
    got = np.linalg.eigvals(P)
    key = lambda v: (np.round(v.real, 9), np.round(v.imag, 9))
    np.testing.assert_allclose(sorted(got, key=key), sorted(ref, key=key), atol=1e-12)


@pytest.mark.parametrize("method", ["rk4", "verlet"])
def test_propagator_of_k_steps_is_the_kth_power_and_the_trajectory(method):
    """P_k equals P_1 multiplied k times, and P_k y0 equals k steps of the
    integrator from y0 (linearity of the scheme); k = 0 is the identity."""
    rng = np.random.default_rng(620)
    s = 4
    M, K = workloads.random_dense_system(rng, s)
    h = 0.2 / np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True)[-1])
    P1 = oracle.propagator(method, "dense", M, K, h, 1)
    Pk = oracle.propagator(method, "dense", M, K, h, 37)
    np.testing.assert_allclose(Pk, np.linalg.matrix_power(P1, 37), atol=1e-12 * np.abs(Pk).max())
    np.testing.assert_array_equal(oracle.propagator(method, "dense", M, K, h, 0), np.eye(2 * s))
    x0, v0 = rng.normal(size=(1, s)), rng.normal(size=(1, s))
    _, _, xe, ve = oracle.dense(method, M, K, [h], x0, v0, 37, 0)
    y = Pk @ np.concatenate([x0[0], v0[0]])
    np.testing.assert_allclose(np.concatenate([xe[0], ve[0]]), y, atol=1e-12 * np.abs(y).max())


@pytest.mark.parametrize("orig,mut", [
    ("P[(size_t)i * n + j] = ye[i]", "P[(size_t)j * n + i] = ye[i]"),          # transposed
    ("y0[i] = (i == j) ? 1.0 : 0.0", "y0[i] = (i == j) ? 1.0 : 0.5 * (i == j + 1)"),  # wrong start
])
def test_pins_catch_planted_propagator_mistakes(orig, mut, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "osc_oracle.c")).read()
    assert orig in src
    mpath = tmp_path / "mut.c"
    mpath.write_text(src.replace(orig, mut))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(lib), str(mpath), "-lm"], check=True)
    import ctypes
    L = ctypes.CDLL(str(lib))
    d = ctypes.POINTER(ctypes.c_double)
    L.oracle_propagator.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d, ctypes.c_double,
                                    ctypes.c_int64, d]
    rng = np.random.default_rng(630)
    s = 3
    M, K = workloads.random_dense_system(rng, s)
    h = 0.5 / np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True)[-1])
    P = np.empty((2 * s, 2 * s))
    p = lambda a: a.ctypes.data_as(d)
    Mc, Kc = np.ascontiguousarray(M), np.ascontiguousarray(K)
    assert L.oracle_propagator(0, 1, s, p(Mc), p(Kc), h, 1, p(P)) == 0
    hL = h * _first_order_matrix(M, K)
    T = sum(np.linalg.matrix_power(hL, j) / math.factorial(j) for j in range(5))
    assert np.abs(P - T).max() > 1e-6, "planted mistake not detected"


# ------------------------------------------- damped and driven systems -------

def _driven_case(kind, s, seed):
    rng = np.random.default_rng(seed)
    if kind == "chain":
        a, b = _random_chain(rng, s)
        M, K = cf.chain_matrices(a, b)
    else:
        M, K = workloads.random_dense_system(rng, s)
        a, b = M, K
    w = np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True))
    F = rng.normal(size=s) * w[-1] ** 2 * 0.1
    x0, v0 = rng.normal(size=s), rng.normal(size=s) * w[-1]
    return a, b, M, K, w, F, x0, v0


@pytest.mark.parametrize("kind", ["chain", "dense"])
def test_driven_with_no_damping_and_no_force_is_the_free_integrator(kind):
    """alpha = beta = 0 and no force: bit for bit the free RK4 oracle."""
    a, b, M, K, w, F, x0, v0 = _driven_case(kind, 4, 640)
    h = 0.3 / w[-1]
    if kind == "chain":
        ref = oracle.chain("rk4", a[None], b[None], [h], x0[None], v0[None], 200, 20)
        got = oracle.chain_driven(a[None], b[None], [h], 0.0, 0.0, None, 0.0, x0[None], v0[None], 200, 20)
    else:
        ref = oracle.dense("rk4", M, K, [h], x0[None], v0[None], 200, 20)
        got = oracle.dense_driven(M, K, [h], 0.0, 0.0, None, 0.0, x0[None], v0[None], 200, 20)
    for r, g in zip(ref, got):
        np.testing.assert_array_equal(r, g)


@pytest.mark.parametrize("kind,s", [("chain", 1), ("chain", 4), ("dense", 3)])
def test_damped_free_matches_discrete_modal_solution(kind, s):
    """Free damped system at h omega_max = 0.4 (the scheme visibly differs
    from the flow) against R(hL_k)^n on every normal mode."""
    a, b, M, K, w, F, x0, v0 = _driven_case(kind, s, 650 + s)
    h = 0.4 / w[-1]
    alpha, beta = 0.05 * w[0], 0.02 / w[-1]
    n, stride = 120, 15
    if kind == "chain":
        xf, vf, _, _ = oracle.chain_driven(a[None], b[None], [h], alpha, beta, None, 0.0, x0[None], v0[None], n,
                                           stride)
    else:
        xf, vf, _, _ = oracle.dense_driven(M, K, [h], alpha, beta, None, 0.0, x0[None], v0[None], n, stride)
    steps = np.arange(0, n + 1, stride)
    xr, vr = cf.rk4_damped_discrete(steps, h, M, K, alpha, beta, x0, v0)
    assert oracle.rel_traj_err(xf, xr[:, None, :])[0] < 1e-11
    assert oracle.rel_traj_err(vf, vr[:, None, :])[0] < 1e-11
    exact_x, _ = cf.driven_modal_solution(steps * h, M, K, alpha, beta, None, 0.0, x0, v0)
    assert oracle.rel_traj_err(xf, exact_x[:, None, :])[0] > 1e-6    # the scheme is visible


@pytest.mark.parametrize("kind,s", [("chain", 2), ("chain", 5), ("dense", 4)])
def test_driven_matches_continuous_closed_form(kind, s):
    """Damped and driven (force near the lowest resonance), h omega_max =
    0.004 over ~30 periods of the fastest mode: RK4's global error is ~1e-10,
    far below any modelling mistake."""
    a, b, M, K, w, F, x0, v0 = _driven_case(kind, s, 660 + s)
    W = 1.1 * w[0]
    alpha, beta = 0.1 * w[0], 0.01 / w[-1]
    h = 0.004 / w[-1]
    n = int(200 / (w[-1] * h))
    stride = n // 8
    n = stride * 8
    if kind == "chain":
        xf, vf, _, _ = oracle.chain_driven(a[None], b[None], [h], alpha, beta, F[None], [W], x0[None], v0[None],
                                           n, stride)
    else:
        xf, vf, _, _ = oracle.dense_driven(M, K, [h], alpha, beta, F[None], [W], x0[None], v0[None], n, stride)
    t = np.arange(0, n + 1, stride) * h
    xr, vr = cf.driven_modal_solution(t, M, K, alpha, beta, F, W, x0, v0)
    assert oracle.rel_traj_err(xf, xr[:, None, :])[0] < 1e-8
    assert oracle.rel_traj_err(vf, vr[:, None, :])[0] < 1e-8


def test_closed_form_steady_state_is_the_receptance_amplitude():
    """Pin of the pin: once the transient has decayed, each modal coordinate
    of the closed form oscillates with amplitude |f_k| / sqrt((w_k^2 - W^2)^2
    + (g_k W)^2) (the textbook steady-state response)."""
    m, k = np.array([1.0, 2.0]), np.array([300.0, 150.0])
    M, K = cf.chain_matrices(m, k)
    w2, Phi = scipy.linalg.eigh(K, M)
    F, W, alpha, beta = np.array([2.0, -1.0]), 9.0, 1.5, 2e-3
    g = alpha + beta * w2
    T0 = 40.0 / g.min()                       # e^-20 of the transient left
    t = T0 + np.linspace(0.0, 2 * np.pi / W, 4001)
    x, _ = cf.driven_modal_solution(t, M, K, alpha, beta, F, W, np.ones(2), np.zeros(2))
    q = x @ (M @ Phi)                         # modal coordinates
    amp = 0.5 * (q.max(axis=0) - q.min(axis=0))
    np.testing.assert_allclose(amp, cf.steady_amplitude(M, K, alpha, beta, F, W), rtol=1e-6)


@pytest.mark.parametrize("kind", ["chain", "dense"])
def test_dopri_reference_matches_closed_form_and_is_fifth_order(kind):
    """The adaptive Dormand-Prince reference meets the exact solution within
    its tolerance, and its step count grows as rtol^(-1/5) (a fifth-order
    pair): 1e5 times tighter costs about 10 times the steps."""
    a, b, M, K, w, F, x0, v0 = _driven_case(kind, 3, 670)
    W, alpha, beta = 0.8 * w[0], 0.05 * w[0], 0.005 / w[-1]
    T = 20 * 2 * np.pi / w[-1]
    xo, vo, acc, rej = oracle.dopri_driven(kind, a, b, alpha, beta, F, W, x0, v0, T, 10, 1e-11, 1e-13)
    t = np.linspace(0.0, T, 11)
    xr, vr = cf.driven_modal_solution(t, M, K, alpha, beta, F, W, x0, v0)
    assert oracle.rel_traj_err(xo[:, None, :], xr[:, None, :])[0] < 1e-8
    assert oracle.rel_traj_err(vo[:, None, :], vr[:, None, :])[0] < 1e-8
    _, _, acc6, _ = oracle.dopri_driven(kind, a, b, alpha, beta, F, W, x0, v0, T, 10, 1e-6, 1e-8)
    assert 5.0 < acc / acc6 < 20.0, (acc, acc6)


DRIVEN_MUTANTS = [
    ("a[i] += -d->alpha * v[i] + d->beta * tmp[i]", "a[i] += d->alpha * v[i] + d->beta * tmp[i]"),  # damping sign
    ("accel_driven(r, d, t + 0.5 * h, xt, vt, k2v, tmp)", "accel_driven(r, d, t, xt, vt, k2v, tmp)"),  # stage time
    ("a43 = 32.0 / 9", "a43 = 31.0 / 9"),                                                            # tableau
]


@pytest.mark.parametrize("orig,mut", DRIVEN_MUTANTS)
def test_pins_catch_planted_driven_mistakes(orig, mut, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "osc_oracle.c")).read()
    assert src.count(orig) == 1
    mpath = tmp_path / "mut.c"
    mpath.write_text(src.replace(orig, mut))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(lib), str(mpath), "-lm"], check=True)
    import ctypes
    L = ctypes.CDLL(str(lib))
    d = ctypes.POINTER(ctypes.c_double)
    dbl, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
    L.oracle_chain_driven.argtypes = [i64, i32, d, d, d, dbl, dbl, d, d, d, d, i64, i64, d, d, d, d]
    L.oracle_dopri_driven.argtypes = [i32, i32, d, d, dbl, dbl, d, dbl, d, d, dbl, i32, dbl, dbl, d, d,
                                      ctypes.POINTER(ctypes.c_int64)]
    a, b, M, K, w, F, x0, v0 = _driven_case("chain", 3, 680)
    W, alpha, beta = 0.9 * w[0], 0.1 * w[0], 0.01 / w[-1]
    p = lambda arr: np.ascontiguousarray(arr, dtype=np.float64).ctypes.data_as(d)
    keep = [np.ascontiguousarray(z, dtype=np.float64) for z in (a, b, F, x0, v0)]
    a, b, F, x0, v0 = keep
    h = 0.004 / w[-1]
    n = int(100 / (w[-1] * h))
    xe, ve = np.empty((1, 3)), np.empty((1, 3))
    hh, WW = np.array([h]), np.array([W])
    L.oracle_chain_driven(1, 3, p(a), p(b), p(hh), alpha, beta, p(F), p(WW), p(x0), p(v0), n, 0, None, None,
                          p(xe), p(ve))
    xr, vr = cf.driven_modal_solution([n * h], M, K, alpha, beta, F, W, x0, v0)
    bad = oracle.rel_traj_err(xe, xr)[0] > 1e-8 or oracle.rel_traj_err(ve, vr)[0] > 1e-8
    xo, vo = np.empty((2, 3)), np.empty((2, 3))
    st = (ctypes.c_int64 * 2)()
    r = L.oracle_dopri_driven(0, 3, p(a), p(b), alpha, beta, p(F), W, p(x0), p(v0), n * h, 1, 1e-11, 1e-13,
                              p(xo), p(vo), st)
    bad = bad or r != 0 or oracle.rel_traj_err(xo[1:], xr)[0] > 1e-8
    assert bad, "planted mistake not detected"
