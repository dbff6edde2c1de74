"""Thin ctypes binding of libosc (include/osc.h).

Argument marshalling only: every step of the integration runs in the HIP
library.  torch supplies device memory and the current stream.  If the built
library is missing the import of this module still works, but every call
raises ``OscError`` -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libosc.so")

OSC_OK, OSC_EINVAL, OSC_ENOTSPD, OSC_EUNSTABLE, OSC_ENOMEM, OSC_EDEVICE, OSC_ENONFINITE, \
    OSC_ENOTSUP, OSC_ETIMEOUT, OSC_EBUSY = range(10)
STATUS_NAMES = {0: "OSC_OK", 1: "OSC_EINVAL", 2: "OSC_ENOTSPD", 3: "OSC_EUNSTABLE", 4: "OSC_ENOMEM",
                5: "OSC_EDEVICE", 6: "OSC_ENONFINITE", 7: "OSC_ENOTSUP", 8: "OSC_ETIMEOUT",
                9: "OSC_EBUSY"}
KINDS = {"chain": 0, "dense": 1}
METHODS = {"rk4": 0, "verlet": 1}
PRECS = {"f64": 0, "f32": 1}
MEM_HOST, MEM_DEVICE = 0, 1
CFG_CHAIN_LAYOUT, CFG_DENSE_KERNEL, CFG_STEPS_PER_LAUNCH, CFG_GRAPH_STEPS, CFG_PROPAGATOR = 1, 2, 3, 4, 5


class OscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class RtStats(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_int64), ("missed", ctypes.c_int64), ("p50_s", ctypes.c_double),
                ("p99_s", ctypes.c_double), ("max_s", ctypes.c_double), ("mean_s", ctypes.c_double),
                ("jitter_s", ctypes.c_double), ("launch_p99_s", ctypes.c_double), ("gpu_p50_s", ctypes.c_double)]


class Desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("method", ctypes.c_int), ("prec", ctypes.c_int),
                ("s", ctypes.c_int32), ("batch", ctypes.c_int64), ("shared", ctypes.c_int32),
                ("param_mem", ctypes.c_int), ("M", ctypes.c_void_p), ("K", ctypes.c_void_p),
                ("dt", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("chunk_us", ctypes.c_int32), ("fake_executor", ctypes.c_int32), ("frame_jumps", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("queue_s", ctypes.c_double), ("latency_s", ctypes.c_double),
                ("bytes", ctypes.c_int64), ("iterations", ctypes.c_int64), ("frame_jumps", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("active", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_peak", ctypes.c_size_t),
                ("setup_s", ctypes.c_double), ("iterate_s", ctypes.c_double)]


_lib = None


def load():
    """Load libosc.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OscError(OSC_EDEVICE, f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # torch carries its own HIP runtime under the same soname as the system's:
    # loaded first, it is the one the library's dependency resolves to, so the
    # process holds a single runtime (loaded after the system's, torch finds
    # no device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    sig = {
        "osc_create": (i32, [ctypes.POINTER(Desc), vp, ctypes.POINTER(vp)]),
        "osc_integrate": (i32, [vp, vp, vp, i64, i64, vp, vp, vp, vp]),
        "osc_integrate_static": (i32, [vp, vp, vp, i64, i64, vp, vp, vp, vp]),
        "osc_integrate_plain": (i32, [vp, vp, vp, i64, vp, vp]),
        "osc_energy": (i32, [vp, vp, vp, vp]),
        "osc_shadow_energy": (i32, [vp, vp, vp, vp]),
        "osc_sync": (i32, [vp]),
        "osc_dense_operator": (i32, [vp, vp]),
        "osc_propagator": (i32, [vp, i64, vp]),
        "osc_set_excitation": (i32, [vp, ctypes.c_double, ctypes.c_double, vp, vp, i32]),
        "osc_set_van_der_pol": (i32, [vp, ctypes.c_double]),
        "osc_rt_create": (i32, [vp, vp, vp, i64, ctypes.POINTER(vp)]),
        "osc_rt_tick": (i32, [vp, vp, vp]),
        "osc_rt_steps": (i64, [vp]),
        "osc_rt_run": (i32, [vp, ctypes.c_double, i64, vp, vp, vp, ctypes.POINTER(RtStats)]),
        "osc_rt_run_resident": (i32, [vp, ctypes.c_double, i64, vp, vp, vp, ctypes.POINTER(RtStats)]),
        "osc_rt_set_idle_limit": (i32, [vp, ctypes.c_double]),
        "osc_rt_destroy": (None, [vp]),
        "osc_set_config": (i32, [vp, i32, i64]),
        "osc_autotune": (i32, [vp, vp, vp, i64, ctypes.POINTER(ctypes.c_int64)]),
        "osc_server_create": (i32, [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]),
        "osc_server_submit": (i32, [vp, ctypes.POINTER(Desc), vp, vp, i64, i64,
                                    ctypes.POINTER(ctypes.c_uint64)]),
        "osc_server_wait": (i32, [vp, ctypes.c_uint64, ctypes.c_double, vp, vp, vp, vp,
                                  ctypes.POINTER(RequestInfo)]),
        "osc_server_stats": (i32, [vp, ctypes.POINTER(ServerStats)]),
        "osc_server_destroy": (None, [vp]),
        "osc_destroy": (None, [vp]),
        "osc_last_error": (ctypes.c_char_p, []),
        "osc_abi_version": (i32, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(st: int):
    if st != OSC_OK:
        msg = load().osc_last_error().decode(errors="replace")
        raise OscError(st, msg)


def _dptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class System:
    """A batch of oscillator systems on the current GPU (one osc_sys handle).

    Parameters M, K, dt are float64 numpy arrays (host) or float64 torch CUDA
    tensors (device), laid out as include/osc.h describes.
    """

    def __init__(self, kind: str, method: str, prec: str, M, K, dt, shared: bool = True,
                 batch: Optional[int] = None, stream=None):
        import torch
        load()
        if kind not in KINDS or method not in METHODS or prec not in PRECS:
            raise ValueError(f"unknown kind/method/precision {kind!r}/{method!r}/{prec!r}")
        self.kind, self.method, self.prec = kind, method, prec
        self.dtype = torch.float64 if prec == "f64" else torch.float32
        on_device = isinstance(M, torch.Tensor)
        if on_device != isinstance(K, torch.Tensor):
            raise ValueError("M and K must both be host arrays or both be device tensors")
        if on_device:
            if not (M.is_cuda and K.is_cuda):
                raise ValueError("device parameters must be CUDA tensors")
            dt = dt if isinstance(dt, torch.Tensor) else torch.as_tensor(np.atleast_1d(dt), device=M.device)
            arrs = [t.contiguous().to(torch.float64) for t in (M, K, dt.reshape(-1))]
        else:
            arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (M, K, np.ravel(dt))]
        M_shape, K_shape, ndt = tuple(arrs[0].shape), tuple(arrs[1].shape), int(arrs[2].shape[0])
        given_batch = batch
        if kind == "chain":
            if len(M_shape) != 2 or K_shape != M_shape:
                raise ValueError(f"chain M and K must both be [batch, s]; got {M_shape} and {K_shape}")
            batch, s = M_shape
            shared = False
            want_dt = batch
        elif shared:
            if len(M_shape) != 2 or M_shape[0] != M_shape[1] or K_shape != M_shape:
                raise ValueError(f"shared dense M and K must both be [s, s]; got {M_shape} and {K_shape}")
            s = M_shape[0]
            want_dt = 1
        else:
            if len(M_shape) != 3 or M_shape[1] != M_shape[2] or K_shape != M_shape:
                raise ValueError(f"per-instance dense M and K must be [batch, s, s]; got {M_shape} and {K_shape}")
            batch, s = M_shape[0], M_shape[1]
            want_dt = batch
        if given_batch is not None and int(given_batch) != batch:
            raise ValueError(f"batch {given_batch} disagrees with the parameters' {batch} instances")
        if ndt == 1 and want_dt != 1:
            # one step for every instance
            arrs[2] = (arrs[2].expand(want_dt).contiguous() if on_device
                       else np.full(want_dt, arrs[2][0], dtype=np.float64))
        elif ndt != want_dt:
            raise ValueError(f"dt must hold 1 or {want_dt} values; got {ndt}")
        if batch is None or int(batch) < 0:
            raise ValueError("batch must be given (>= 0) for a shared dense system")
        self._keep = arrs
        ptrs = [t.data_ptr() for t in arrs] if on_device else [a.ctypes.data for a in arrs]
        self.s = int(s)
        self.batch = int(batch)
        self._shared = shared
        self.stream = stream
        self._desc = Desc(KINDS[kind], METHODS[method], PRECS[prec], self.s, self.batch, 1 if shared else 0,
                          MEM_DEVICE if on_device else MEM_HOST, ptrs[0], ptrs[1], ptrs[2])
        self.handle = None

    def create(self, batch: Optional[int] = None):
        if batch is not None:
            if not (self.kind == "dense" and self._shared):
                raise ValueError("batch is fixed by the parameters except for a shared dense system")
            self._desc.batch = int(batch)
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.osc_create(ctypes.byref(self._desc), _stream_handle(self.stream), ctypes.byref(h)))
        self.handle = h
        self.batch = int(self._desc.batch)
        self._keep = None
        return self

    # -- helpers -----------------------------------------------------------
    def _tensor(self, t, shape, dtype, what):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda):
            raise ValueError(f"{what} must be a CUDA tensor")
        if t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{what} must be a contiguous {dtype} tensor; got {t.dtype}"
                             f"{'' if t.is_contiguous() else ' (not contiguous)'}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        return t

    def _state(self, t, what="state"):
        if self.handle is None:
            raise ValueError("the system has not been created (call create())")
        return self._tensor(t, (self.batch, self.s), self.dtype, what)

    def integrate(self, x0, v0, nsteps: int, out_stride: int = 0, frames: bool = True,
                  out=None, static: bool = False):
        """Returns (x_frames, v_frames, x_end, v_end) as new device tensors
        (frames None when out_stride == 0 or frames is False).  static: call
        osc_integrate_static (no device allocation inside the library; pass
        ``out`` to allocate nothing at all)."""
        import torch
        x0, v0 = self._state(x0, "x0"), self._state(v0, "v0")
        if nsteps < 0 or out_stride < 0:
            raise ValueError("nsteps and out_stride must be >= 0")
        nf = nsteps // out_stride + 1 if (out_stride > 0 and frames) else 0
        dev = x0.device
        if out is None:
            xf = torch.empty((nf, self.batch, self.s), dtype=self.dtype, device=dev) if nf else None
            vf = torch.empty((nf, self.batch, self.s), dtype=self.dtype, device=dev) if nf else None
            xe = torch.empty_like(x0)
            ve = torch.empty_like(v0)
        else:
            xf, vf, xe, ve = out
            fshape = (nf, self.batch, self.s)
            for t, what in ((xf, "x_frames"), (vf, "v_frames")):
                if t is not None:
                    if not nf:
                        raise ValueError(f"{what} given but no frames are produced")
                    self._tensor(t, fshape, self.dtype, what)
            for t, what in ((xe, "x_end"), (ve, "v_end")):
                if t is not None:
                    self._state(t, what)
        entry = load().osc_integrate_static if static else load().osc_integrate
        _check(entry(self.handle, _dptr(x0), _dptr(v0), int(nsteps), int(out_stride) if nf else 0,
                     _dptr(xf), _dptr(vf), _dptr(xe), _dptr(ve)))
        return xf, vf, xe, ve

    def integrate_plain(self, x0, v0, nsteps: int):
        import torch
        x0, v0 = self._state(x0, "x0"), self._state(v0, "v0")
        if nsteps < 0:
            raise ValueError("nsteps must be >= 0")
        xe, ve = torch.empty_like(x0), torch.empty_like(v0)
        _check(load().osc_integrate_plain(self.handle, _dptr(x0), _dptr(v0), int(nsteps),
                                          _dptr(xe), _dptr(ve)))
        return xe, ve

    def energy(self, x, v, shadow: bool = False):
        import torch
        x, v = self._state(x), self._state(v)
        E = torch.empty(self.batch, dtype=torch.float64, device=x.device)
        f = load().osc_shadow_energy if shadow else load().osc_energy
        _check(f(self.handle, _dptr(x), _dptr(v), _dptr(E)))
        return E

    def set_config(self, key: int, value: int):
        """osc_set_config: CFG_CHAIN_LAYOUT ((lanes << 16) | dofs_per_lane),
        CFG_DENSE_KERNEL (0 auto, 1 VALU, 2 MFMA), CFG_STEPS_PER_LAUNCH."""
        _check(load().osc_set_config(self.handle, int(key), int(value)))
        return self

    def autotune(self, x0, v0, probe_steps: int = 200) -> int:
        """osc_autotune: time the feasible launch configurations, keep the fastest."""
        x0, v0 = self._state(x0), self._state(v0)
        chosen = ctypes.c_int64(0)
        _check(load().osc_autotune(self.handle, _dptr(x0), _dptr(v0), int(probe_steps), ctypes.byref(chosen)))
        return chosen.value

    def set_excitation(self, alpha: float = 0.0, beta: float = 0.0, F=None, omega=None):
        """osc_set_excitation: Rayleigh damping alpha M + beta K and a force
        F cos(omega t).  F: [batch, s] float64 (numpy or CUDA tensor) or None;
        omega: [batch] (or a scalar for every instance)."""
        import torch
        if self.handle is None:
            raise ValueError("the system has not been created (call create())")
        keep = []
        Fp = Wp = None
        mem = MEM_HOST
        if F is not None:
            if omega is None:
                raise ValueError("a force needs omega")
            if isinstance(F, torch.Tensor):
                if not F.is_cuda or F.dtype != torch.float64 or tuple(F.shape) != (self.batch, self.s):
                    raise ValueError(f"F must be a CUDA float64 tensor of shape {(self.batch, self.s)}")
                F = F.contiguous()
                W = torch.as_tensor(np.broadcast_to(np.atleast_1d(np.asarray(omega, dtype=np.float64)),
                                                    (self.batch,)).copy(), device=F.device)
                mem = MEM_DEVICE
                keep += [F, W]
                Fp, Wp = F.data_ptr(), W.data_ptr()
            else:
                F = np.ascontiguousarray(F, dtype=np.float64)
                if F.shape != (self.batch, self.s):
                    raise ValueError(f"F has shape {F.shape}, expected {(self.batch, self.s)}")
                W = np.ascontiguousarray(np.broadcast_to(np.atleast_1d(np.asarray(omega, dtype=np.float64)),
                                                         (self.batch,)))
                keep += [F, W]
                Fp, Wp = F.ctypes.data, W.ctypes.data
        _check(load().osc_set_excitation(self.handle, float(alpha), float(beta), Fp, Wp, mem))
        return self

    def set_van_der_pol(self, mu: float):
        """osc_set_van_der_pol: a Van der Pol element mu (1 - x_i^2) x_i' on
        every body of a chain (mu = 0: linear again)."""
        if self.handle is None:
            raise ValueError("the system has not been created (call create())")
        _check(load().osc_set_van_der_pol(self.handle, float(mu)))
        return self
    def propagator(self, k: int = 1):
        """osc_propagator: the FP64 matrix of k steps on (x, v), a new device
        tensor [nsys, 2s, 2s] (nsys = batch, or 1 for a shared operator)."""
        import torch
        if self.handle is None:
            raise ValueError("the system has not been created (call create())")
        if k < 0:
            raise ValueError("k must be >= 0")
        nsys = 1 if (self.kind == "dense" and self._shared) else self.batch
        P = torch.empty((nsys, 2 * self.s, 2 * self.s), dtype=torch.float64, device="cuda")
        _check(load().osc_propagator(self.handle, int(k), _dptr(P)))
        return P

    def dense_operator(self):
        """A = M^-1 K as formed on the GPU (FP64), [nsys, s, s]."""
        import torch
        nsys = 1 if self._shared else self.batch
        A = torch.empty((nsys, self.s, self.s), dtype=torch.float64, device="cuda")
        _check(load().osc_dense_operator(self.handle, _dptr(A)))
        return A

    def sync(self):
        _check(load().osc_sync(self.handle))

    def close(self):
        if self.handle is not None:
            load().osc_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Realtime:
    """Real-time periodic stepping of one created System (osc_rt_*): the
    state stays on the device; each tick advances steps_per_tick steps."""

    def __init__(self, system: "System", x0, v0, steps_per_tick: int = 1):
        self.system = system
        x0, v0 = system._state(x0, "x0"), system._state(v0, "v0")
        if steps_per_tick < 1:
            raise ValueError("steps_per_tick must be >= 1")
        h = ctypes.c_void_p()
        _check(load().osc_rt_create(system.handle, _dptr(x0), _dptr(v0), int(steps_per_tick), ctypes.byref(h)))
        self.handle = h

    @property
    def steps(self) -> int:
        return int(load().osc_rt_steps(self.handle))

    def tick(self, out=None):
        """One tick; returns (x, v) device tensors of the new state."""
        import torch
        sysm = self.system
        if out is None:
            out = (torch.empty((sysm.batch, sysm.s), dtype=sysm.dtype, device="cuda"),
                   torch.empty((sysm.batch, sysm.s), dtype=sysm.dtype, device="cuda"))
        x, v = (sysm._state(t, "out") for t in out)
        _check(load().osc_rt_tick(self.handle, _dptr(x), _dptr(v)))
        return x, v

    def _run(self, fn, period_s: float, nticks: int, frames: bool):
        import torch
        sysm = self.system
        if nticks < 0:
            raise ValueError("nticks must be >= 0")
        xf = vf = None
        if frames and nticks > 0:
            xf = torch.empty((nticks, sysm.batch, sysm.s), dtype=sysm.dtype, device="cuda")
            vf = torch.empty_like(xf)
        lat = np.zeros(max(nticks, 1))
        st = RtStats()
        _check(fn(self.handle, float(period_s), int(nticks), _dptr(xf), _dptr(vf), lat.ctypes.data, ctypes.byref(st)))
        stats = {name: getattr(st, name) for name, _ in RtStats._fields_}
        return xf, vf, lat[:nticks], stats

    def run(self, period_s: float, nticks: int, frames: bool = True):
        """osc_rt_run: returns (x_frames, v_frames, latencies [s], stats dict);
        frames are the states after each tick, [nticks, batch, s]."""
        return self._run(load().osc_rt_run, period_s, nticks, frames)

    def run_resident(self, period_s: float, nticks: int, frames: bool = True):
        """osc_rt_run_resident: the same loop with one kernel resident on the
        device for the whole run (chains); same return values."""
        return self._run(load().osc_rt_run_resident, period_s, nticks, frames)

    def set_idle_limit(self, seconds: float):
        """osc_rt_set_idle_limit (0 restores the default)."""
        _check(load().osc_rt_set_idle_limit(self.handle, float(seconds)))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().osc_rt_destroy(self.handle)
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chain_system(method: str, prec: str, m, k, dt, stream=None) -> System:
    return System("chain", method, prec, m, k, dt, stream=stream).create()


class Server:
    """Continuous-batching request server (osc_server_*).  Requests are single
    instances given as host numpy arrays; results come back as numpy arrays."""

    def __init__(self, hbm_budget: int = 0, max_slots: int = 256, chunk_us: int = 0,
                 fake_executor: bool = False, frame_jumps: bool = False):
        lib = load()
        cfg = ServerConfig(int(hbm_budget), int(max_slots), int(chunk_us), 1 if fake_executor else 0,
                           1 if frame_jumps else 0)
        h = ctypes.c_void_p()
        _check(lib.osc_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._meta = {}

    def submit(self, kind: str, method: str, prec: str, M, K, dt, x0, v0, nsteps: int,
               out_stride: int = 0) -> int:
        M = np.ascontiguousarray(M, dtype=np.float64)
        K = np.ascontiguousarray(K, dtype=np.float64)
        dt = np.ascontiguousarray(np.atleast_1d(dt), dtype=np.float64)
        dtype = np.float64 if prec == "f64" else np.float32
        x0 = np.ascontiguousarray(np.ravel(x0), dtype=dtype)
        v0 = np.ascontiguousarray(np.ravel(v0), dtype=dtype)
        s = x0.shape[0]
        if kind not in KINDS or method not in METHODS or prec not in PRECS:
            raise ValueError(f"unknown kind/method/precision {kind!r}/{method!r}/{prec!r}")
        if v0.shape[0] != s:
            raise ValueError(f"x0 and v0 must hold the same number of DOFs; got {s} and {v0.shape[0]}")
        np_want = s if kind == "chain" else s * s
        if M.size != np_want or K.size != np_want:
            raise ValueError(f"a {kind} request of s = {s} needs {np_want} values in M and in K; "
                             f"got {M.size} and {K.size}")
        if dt.size != 1:
            raise ValueError("a request takes one step size")
        if nsteps < 0 or out_stride < 0:
            raise ValueError("nsteps and out_stride must be >= 0")
        d = Desc(KINDS[kind], METHODS[method], PRECS[prec], s, 1, 1 if kind == "dense" else 0,
                 MEM_HOST, M.ctypes.data, K.ctypes.data, dt.ctypes.data)
        t = ctypes.c_uint64()
        _check(load().osc_server_submit(self.handle, ctypes.byref(d), x0.ctypes.data, v0.ctypes.data,
                                        int(nsteps), int(out_stride), ctypes.byref(t)))
        nf = nsteps // out_stride + 1 if out_stride > 0 else 0
        self._meta[t.value] = (s, nf, dtype)
        return t.value

    def wait(self, ticket: int, timeout: float = -1.0):
        """Returns dict(x_frames, v_frames, x_end, v_end, info) or raises OscError
        (OSC_ETIMEOUT if not done within timeout seconds)."""
        s, nf, dtype = self._meta.get(ticket, (0, 0, np.float32))
        xf = np.empty((nf, s), dtype=dtype)
        vf = np.empty((nf, s), dtype=dtype)
        xe = np.empty(s, dtype=dtype)
        ve = np.empty(s, dtype=dtype)
        info = RequestInfo()
        st = load().osc_server_wait(self.handle, ctypes.c_uint64(ticket), float(timeout),
                                    xf.ctypes.data if nf else None, vf.ctypes.data if nf else None,
                                    xe.ctypes.data, ve.ctypes.data, ctypes.byref(info))
        if st == OSC_ETIMEOUT:
            _check(st)
        self._meta.pop(ticket, None)
        _check(st)
        return {"x_frames": xf, "v_frames": vf, "x_end": xe, "v_end": ve,
                "latency_s": info.latency_s, "queue_s": info.queue_s, "bytes": info.bytes,
                "iterations": info.iterations, "frame_jumps": bool(info.frame_jumps)}

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().osc_server_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self.handle is not None:
            load().osc_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
