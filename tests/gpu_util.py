"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
the oracle on the same seeded inputs."""
import numpy as np

import oracle


def torch_dev():
    import torch
    return torch


def to_dev(a, dtype):
    torch = torch_dev()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def gpu_chain(method, prec, w, nsteps=None, stride=None, frames=True):
    """Integrate a ChainBatch on the GPU; returns numpy float64 arrays
    (xf, vf, xe, ve)."""
    from paper_1702_02207_amd import osc
    torch = torch_dev()
    nsteps = w.nsteps if nsteps is None else nsteps
    stride = w.out_stride if stride is None else stride
    dt = torch.float64 if prec == "f64" else torch.float32
    sysm = osc.System("chain", method, prec, w.m, w.k, w.dt).create()
    try:
        x0, v0 = to_dev(w.x0, dt), to_dev(w.v0, dt)
        xf, vf, xe, ve = sysm.integrate(x0, v0, nsteps, stride, frames=frames)
        sysm.sync()
        cv = lambda t: None if t is None else t.double().cpu().numpy()
        return cv(xf), cv(vf), cv(xe), cv(ve)
    finally:
        sysm.close()


def oracle_chain(method, w, nsteps=None, stride=None, frames=True, x0=None, v0=None):
    nsteps = w.nsteps if nsteps is None else nsteps
    stride = w.out_stride if stride is None else stride
    x0 = w.x0 if x0 is None else x0
    v0 = w.v0 if v0 is None else v0
    return oracle.chain(method, w.m, w.k, w.dt, x0, v0, nsteps, stride, frames=frames)


def f32_inputs(w):
    """The FP32 state the GPU actually starts from, widened back to FP64, so
    that the oracle integrates the identical initial condition."""
    return w.x0.astype(np.float32).astype(np.float64), w.v0.astype(np.float32).astype(np.float64)


def gpu_dense(method, prec, w, nsteps=None, stride=None, frames=True):
    """Integrate a DenseBatch on the GPU; numpy float64 (xf, vf, xe, ve)."""
    from paper_1702_02207_amd import osc
    torch = torch_dev()
    nsteps = w.nsteps if nsteps is None else nsteps
    stride = w.out_stride if stride is None else stride
    dt = torch.float64 if prec == "f64" else torch.float32
    sysm = osc.System("dense", method, prec, w.M, w.K, w.dt, shared=w.shared, batch=w.batch).create()
    try:
        x0, v0 = to_dev(w.x0, dt), to_dev(w.v0, dt)
        xf, vf, xe, ve = sysm.integrate(x0, v0, nsteps, stride, frames=frames)
        sysm.sync()
        cv = lambda t: None if t is None else t.double().cpu().numpy()
        return cv(xf), cv(vf), cv(xe), cv(ve)
    finally:
        sysm.close()


def oracle_dense(method, w, nsteps=None, stride=None, frames=True, x0=None, v0=None):
    nsteps = w.nsteps if nsteps is None else nsteps
    stride = w.out_stride if stride is None else stride
    x0 = w.x0 if x0 is None else x0
    v0 = w.v0 if v0 is None else v0
    return oracle.dense(method, w.M, w.K, w.dt, x0, v0, nsteps, stride, shared=w.shared, frames=frames)
