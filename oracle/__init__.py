"""FP64 CPU oracle for the coupled harmonic oscillator (arXiv 1702.02207).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may import this package; the product library and its binding never
do.  It shares no code with the HIP path.

``osc_oracle.c`` holds the integrators (classic RK4 and velocity Verlet on the
first-order system of section 3), the Cholesky formation of A = M^-1 K for
eq. (1), the energy and the Verlet invariant.  ``closed_form.py`` holds the
analytic results of section 2 (eq. (4)-(7)) and the exact discrete solutions of
both schemes, which pin the C code to the mathematics.

All arrays are float64, C-contiguous, instance-major: [batch, s]; frames are
[nframes, batch, s] with nframes = nsteps // stride + 1 (stride > 0).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import closed_form  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboscoracle.so")
_lib = None

RK4, VERLET = 0, 1
_METHODS = {"rk4": RK4, "verlet": VERLET}


class OracleError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "osc_oracle.c"))):
        from . import build
        build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    d = ctypes.POINTER(ctypes.c_double)
    i64, i32 = ctypes.c_int64, ctypes.c_int
    lib.oracle_chain.argtypes = [i32, i64, i32, d, d, d, d, d, i64, i64, d, d, d, d]
    lib.oracle_dense.argtypes = [i32, i64, i32, i32, d, d, d, d, d, i64, i64, d, d, d, d]
    lib.oracle_form_a.argtypes = [i32, d, d, d]
    lib.oracle_energy_chain.argtypes = [i64, i32, d, d, d, d, d]
    lib.oracle_energy_dense.argtypes = [i64, i32, i32, d, d, d, d, d]
    lib.oracle_verlet_q_chain.argtypes = [i64, i32, d, d, d, d, d, d]
    lib.oracle_verlet_q_dense.argtypes = [i64, i32, i32, d, d, d, d, d, d]
    lib.oracle_propagator.argtypes = [i32, i32, i32, d, d, ctypes.c_double, i64, d]
    dbl = ctypes.c_double
    lib.oracle_chain_driven.argtypes = [i64, i32, d, d, d, dbl, dbl, d, d, d, d, i64, i64, d, d, d, d]
    lib.oracle_dense_driven.argtypes = [i64, i32, i32, d, d, d, dbl, dbl, d, d, d, d, i64, i64, d, d, d, d]
    lib.oracle_dopri_driven.argtypes = [i32, i32, d, d, dbl, dbl, d, dbl, d, d, dbl, i32, dbl, dbl, d, d,
                                        ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_chain_vdp.argtypes = [i64, i32, d, d, d, dbl, d, d, d, d, i64, i64, d, d, d, d]
    lib.oracle_dopri_vdp.argtypes = [i32, d, d, dbl, d, d, dbl, i32, dbl, dbl, d, d,
                                     ctypes.POINTER(ctypes.c_int64)]
    for f in ("oracle_chain_vdp", "oracle_dopri_vdp", "oracle_chain_driven", "oracle_dense_driven", "oracle_dopri_driven", "oracle_propagator", "oracle_chain", "oracle_dense", "oracle_form_a", "oracle_energy_chain",
              "oracle_energy_dense", "oracle_verlet_q_chain", "oracle_verlet_q_dense"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(st, what):
    if st != 0:
        raise OracleError(f"{what} failed with status {st}")


def _nframes(nsteps, stride):
    return nsteps // stride + 1 if stride > 0 else 0


def chain(method, m, k, dt, x0, v0, nsteps, stride, frames=True):
    """Integrate fixed-free chains (eq. (2) for s bodies).

    Returns (x_frames, v_frames, x_end, v_end); frames are None when
    ``frames`` is False or stride == 0."""
    lib = _load()
    m, k, dt, x0, v0 = map(_f64, (m, k, dt, x0, v0))
    batch, s = x0.shape
    nf = _nframes(nsteps, stride) if frames else 0
    xf = np.empty((nf, batch, s)) if nf else None
    vf = np.empty((nf, batch, s)) if nf else None
    xe = np.empty((batch, s))
    ve = np.empty((batch, s))
    st = lib.oracle_chain(_METHODS[method], batch, s, _p(m), _p(k), _p(dt), _p(x0), _p(v0),
                          int(nsteps), int(stride) if nf else 0, _p(xf), _p(vf), _p(xe), _p(ve))
    _check(st, "oracle_chain")
    return xf, vf, xe, ve


def dense(method, M, K, dt, x0, v0, nsteps, stride, shared=True, frames=True):
    """Integrate eq. (1) with full M, K (A = M^-1 K by Cholesky).  shared: M, K
    are [s, s] and dt[0] is used for every instance."""
    lib = _load()
    M, K, dt, x0, v0 = map(_f64, (M, K, np.atleast_1d(dt), x0, v0))
    batch, s = x0.shape
    nf = _nframes(nsteps, stride) if frames else 0
    xf = np.empty((nf, batch, s)) if nf else None
    vf = np.empty((nf, batch, s)) if nf else None
    xe = np.empty((batch, s))
    ve = np.empty((batch, s))
    st = lib.oracle_dense(_METHODS[method], batch, s, 1 if shared else 0, _p(M), _p(K), _p(dt),
                          _p(x0), _p(v0), int(nsteps), int(stride) if nf else 0,
                          _p(xf), _p(vf), _p(xe), _p(ve))
    _check(st, "oracle_dense")
    return xf, vf, xe, ve


def form_a(M, K):
    """A = M^-1 K via M = L L^T; raises OracleError (status 2) if M is not SPD."""
    lib = _load()
    M, K = _f64(M), _f64(K)
    s = M.shape[0]
    A = np.empty((s, s))
    _check(lib.oracle_form_a(s, _p(M), _p(K), _p(A)), "oracle_form_a")
    return A


def energy_chain(m, k, x, v):
    lib = _load()
    m, k, x, v = map(_f64, (m, k, x, v))
    batch, s = x.shape
    E = np.empty(batch)
    _check(lib.oracle_energy_chain(batch, s, _p(m), _p(k), _p(x), _p(v), _p(E)), "energy_chain")
    return E


def energy_dense(M, K, x, v, shared=True):
    lib = _load()
    M, K, x, v = map(_f64, (M, K, x, v))
    batch, s = x.shape
    E = np.empty(batch)
    _check(lib.oracle_energy_dense(batch, s, 1 if shared else 0, _p(M), _p(K), _p(x), _p(v),
                                   _p(E)), "energy_dense")
    return E


def verlet_q_chain(m, k, dt, x, v):
    lib = _load()
    m, k, dt, x, v = map(_f64, (m, k, dt, x, v))
    batch, s = x.shape
    Q = np.empty(batch)
    _check(lib.oracle_verlet_q_chain(batch, s, _p(m), _p(k), _p(dt), _p(x), _p(v), _p(Q)),
           "verlet_q_chain")
    return Q


def verlet_q_dense(M, K, dt, x, v, shared=True):
    """Q = v^T M v + x^T K x - (dt^2/4) (K x)^T M^-1 (K x) per instance, the
    exact invariant of velocity Verlet for a dense system."""
    lib = _load()
    M, K, dt, x, v = map(_f64, (M, K, np.atleast_1d(dt), x, v))
    batch, s = x.shape
    Q = np.empty(batch)
    _check(lib.oracle_verlet_q_dense(batch, s, 1 if shared else 0, _p(M), _p(K), _p(dt), _p(x), _p(v),
                                     _p(Q)), "verlet_q_dense")
    return Q


def propagator(method, kind, a, b, dt, k=1):
    """The matrix P_k of k steps of the scheme on y = (x, v) (positions
    first): y_{n+k} = P_k y_n, [2s, 2s].  kind "chain": a = m, b = k ([s]);
    "dense": a = M, b = K ([s, s]).  Column j is k oracle steps started from
    the j-th unit vector."""
    lib = _load()
    a, b = _f64(a), _f64(b)
    s = a.shape[0]
    P = np.empty((2 * s, 2 * s))
    _check(lib.oracle_propagator(_METHODS[method], {"chain": 0, "dense": 1}[kind], s, _p(a), _p(b),
                                 float(dt), int(k), _p(P)), "oracle_propagator")
    return P


def _driven_force(F, omega, batch):
    if F is None:
        return None, None
    F = _f64(F).reshape(batch, -1)
    omega = _f64(np.broadcast_to(np.atleast_1d(omega), (batch,)))
    return F, omega


def chain_driven(m, k, dt, alpha, beta, F, omega, x0, v0, nsteps, stride, frames=True):
    """Classic RK4 for damped, driven chains: M x'' + (alpha M + beta K) x' +
    K x = F cos(omega t).  F [batch, s] forces (None: no force), omega [batch]
    (or a scalar).  Returns (x_frames, v_frames, x_end, v_end)."""
    lib = _load()
    m, k, dt, x0, v0 = map(_f64, (m, k, dt, x0, v0))
    batch, s = x0.shape
    F, omega = _driven_force(F, omega, batch)
    nf = _nframes(nsteps, stride) if frames else 0
    xf = np.empty((nf, batch, s)) if nf else None
    vf = np.empty((nf, batch, s)) if nf else None
    xe, ve = np.empty((batch, s)), np.empty((batch, s))
    st = lib.oracle_chain_driven(batch, s, _p(m), _p(k), _p(dt), float(alpha), float(beta), _p(F), _p(omega),
                                 _p(x0), _p(v0), int(nsteps), int(stride) if nf else 0,
                                 _p(xf), _p(vf), _p(xe), _p(ve))
    _check(st, "oracle_chain_driven")
    return xf, vf, xe, ve


def dense_driven(M, K, dt, alpha, beta, F, omega, x0, v0, nsteps, stride, shared=True, frames=True):
    """Classic RK4 for damped, driven dense systems (f = M^-1 F by Cholesky)."""
    lib = _load()
    M, K, dt, x0, v0 = map(_f64, (M, K, np.atleast_1d(dt), x0, v0))
    batch, s = x0.shape
    F, omega = _driven_force(F, omega, batch)
    nf = _nframes(nsteps, stride) if frames else 0
    xf = np.empty((nf, batch, s)) if nf else None
    vf = np.empty((nf, batch, s)) if nf else None
    xe, ve = np.empty((batch, s)), np.empty((batch, s))
    st = lib.oracle_dense_driven(batch, s, 1 if shared else 0, _p(M), _p(K), _p(dt), float(alpha), float(beta),
                                 _p(F), _p(omega), _p(x0), _p(v0), int(nsteps), int(stride) if nf else 0,
                                 _p(xf), _p(vf), _p(xe), _p(ve))
    _check(st, "oracle_dense_driven")
    return xf, vf, xe, ve


def dopri_driven(kind, a, b, alpha, beta, F, omega, x0, v0, t_end, nout, rtol=1e-10, atol=1e-12):
    """Adaptive Dormand-Prince 5(4) reference for one damped, driven instance
    (kind "chain": a = m, b = k; "dense": a = M, b = K).  Returns
    (x [nout+1, s], v [nout+1, s], accepted steps, rejected steps) at
    t_j = j t_end / nout."""
    lib = _load()
    a, b, x0, v0 = map(_f64, (a, b, x0, v0))
    s = x0.shape[-1]
    Fp = None if F is None else _f64(F).reshape(s)
    xo, vo = np.empty((nout + 1, s)), np.empty((nout + 1, s))
    stats = (ctypes.c_int64 * 2)()
    st = lib.oracle_dopri_driven({"chain": 0, "dense": 1}[kind], s, _p(a), _p(b), float(alpha), float(beta),
                                 _p(Fp), float(omega), _p(x0.reshape(s)), _p(v0.reshape(s)), float(t_end),
                                 int(nout), float(rtol), float(atol), _p(xo), _p(vo), stats)
    _check(st, "oracle_dopri_driven")
    return xo, vo, int(stats[0]), int(stats[1])


def chain_vdp(m, k, dt, mu, x0, v0, nsteps, stride, frames=True, F=None, omega=None):
    """Classic RK4 for coupled Van der Pol chains: m_i x_i'' - mu (1 - x_i^2)
    x_i' + (K x)_i = F_i cos(omega t) with the chain's K (F [batch, s] or
    None, omega [batch] or a scalar).  Returns (x_frames, v_frames, x_end,
    v_end)."""
    lib = _load()
    m, k, dt, x0, v0 = map(_f64, (m, k, dt, x0, v0))
    batch, s = x0.shape
    F, omega = _driven_force(F, omega, batch)
    nf = _nframes(nsteps, stride) if frames else 0
    xf = np.empty((nf, batch, s)) if nf else None
    vf = np.empty((nf, batch, s)) if nf else None
    xe, ve = np.empty((batch, s)), np.empty((batch, s))
    st = lib.oracle_chain_vdp(batch, s, _p(m), _p(k), _p(dt), float(mu), _p(F), _p(omega), _p(x0), _p(v0), int(nsteps),
                              int(stride) if nf else 0, _p(xf), _p(vf), _p(xe), _p(ve))
    _check(st, "oracle_chain_vdp")
    return xf, vf, xe, ve


def dopri_vdp(m, k, mu, x0, v0, t_end, nout, rtol=1e-10, atol=1e-12):
    """Adaptive Dormand-Prince 5(4) reference for one Van der Pol chain.
    Returns (x [nout+1, s], v [nout+1, s], accepted, rejected)."""
    lib = _load()
    m, k, x0, v0 = map(_f64, (m, k, x0, v0))
    s = x0.shape[-1]
    xo, vo = np.empty((nout + 1, s)), np.empty((nout + 1, s))
    stats = (ctypes.c_int64 * 2)()
    st = lib.oracle_dopri_vdp(s, _p(m.reshape(s)), _p(k.reshape(s)), float(mu), _p(x0.reshape(s)),
                              _p(v0.reshape(s)), float(t_end), int(nout), float(rtol), float(atol), _p(xo), _p(vo),
                              stats)
    _check(st, "oracle_dopri_vdp")
    return xo, vo, int(stats[0]), int(stats[1])


def rel_traj_err(got, ref):
    """Per-instance max-abs relative trajectory error:
    max over frames and dofs of |got - ref| divided by max |ref|.
    Arrays are [..., batch, s]; returns [batch]."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.ndim == 2:
        got, ref = got[None], ref[None]
    num = np.abs(got - ref).max(axis=(0, 2))
    den = np.abs(ref).max(axis=(0, 2))
    return num / np.where(den > 0, den, 1.0)
