#!/usr/bin/env python3
"""Throughput benchmark of the batched oscillator integrator on one MI355X.

Default workload (c3): 4096 fixed-free spring chains of s = 1024 bodies
(eq. (2) generalised), masses U[0.5, 2], springs LogU[1e2, 1e4],
x0 ~ N(0, sigma = 0.1), v0 = 0, dt = 0.01/omega_max per chain, 10^5 classic
RK4 steps with FP32 state (synthetic, seeded): the largest configuration
that fits one GPU.  --workload picks another (c1, c2, c2v, c3v, c3d, c3n, c4, c4v, c4d, c5;
and the propagator modes: c1p and c2p, the per-step step matrix; c2j and c4j, frames
by powers of the step matrix).

One timed step is one pass of the whole hot path over the batch, with every
input already resident in HBM: osc_create from device-resident FP64
parameters (chains: coefficients h^2 k/m split into FP32 hi + lo and the
stability bound; dense: A = M^-1 K by FP64 Cholesky, the bound and the split
FP16 operator), osc_integrate (every step of the run, frames at n = 0 and
n = nsteps unless stated), osc_energy (FP64 energy of the final state),
osc_sync and osc_destroy.

Printed JSON line: value = DOF-steps/s = batch * s * nsteps / step time.  Also
reported: the plain per-instance GPU integrator (osc_integrate_plain: one
instance at a time, one time step per launch, full step count) on 64
instances and the speedup over it; the roofline of the dominant kernel (live
HIP-event timing of its launch) against the algorithmic flop count of the
method (classic stage form: RK4 48 flop per DOF-step for chains, 44 for the
two-mass system; Verlet 10), with the implementation's own count beside it;
the FP64 oracle timed on the host cores on a bounded sample (instance 0, the
last instance and seeded others); the relative trajectory error of that
sample against the oracle; a served stream (p50/p99 latency, per kind,
and DOF-steps/s of 200 requests at half the measured saturation rate); and
real-time stepping of the paper's system (one step per 20 us / 100 us / 1 ms
period: release-to-result latency, jitter, missed deadlines).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "fp64": 78.6, "fp16_mfma": 2500.0}   # MI355X published, TFLOP/s
TOL = {"f32": 1e-5, "f64": 1e-10}

# Algorithmic flops per DOF-step (FMA = 2) of the method as the paper states
# it (classic four-stage RK4 on the first-order system; velocity Verlet):
# RK4 chains 48 (two-mass system 44), Verlet 10; dense (one operator shared by
# the batch) the products alone, RK4 4 x 2s, Verlet 1 x 2s.
ALG_CHAIN_FLOPS = {"rk4": 48, "verlet": 10}
ALG_CHAIN2_FLOPS = {"rk4": 44, "verlet": 10}
# The implementation's own count at the FP32 target precision (the exact
# Taylor form of the RK4 map): four B-products (B x with split coefficients
# 8, three others 4 each), two update polynomials (6 each) and two
# compensated sums (4 each) = 40; Verlet leapfrog: split B x 8 + two
# compensated sums = 16.  FP64 drops the split and compensation: RK4 28,
# Verlet 8.
IMPL_CHAIN_FLOPS = {("rk4", "f32"): 40, ("verlet", "f32"): 16, ("rk4", "f64"): 28, ("verlet", "f64"): 8}
DENSE_PRODUCTS = {"rk4": 4, "verlet": 1}
DENSE_HW_TERMS = {"rk4": 7, "verlet": 3}     # MFMA products per step with the FP16 splits

# oracle sample sizes (instance 0, the last instance and seeded others)
CPU_SAMPLE = {"c1": 1, "c1p": 1, "c2": 65536, "c2v": 65536, "c2p": 65536, "c2j": 65536, "c3": 32, "c3v": 32, "c3d": 32, "c3n": 32,
              "c4": 256, "c4v": 256, "c4j": 256}
# the per-step propagator's own count for two-mass RK4 at FP32: per DOF, dx
# from the low parts, the w terms and the high parts of one row of the 4x4
# step matrix (6 FMA) plus w (1 add), dw likewise (6 FMA), two compensated
# sums (2 adds) and two state reads (2 adds)
IMPL_PROP_STEP_FLOPS = 29
# classic stage-form RK4 of the damped, driven chain (FMA = 2): per stage two
# stencil products (B X, B W: 5 flop each), the slope -B X - a W - b B W + f c
# (6) and the next stage's arguments (4); four stages less the first one's
# arguments, plus the weighted combination (9)
ALG_DRIVEN_CHAIN_FLOPS = 85
# the register kernel's form of the same map (FMA = 2): B x with split
# coefficients (8), four high-coefficient stencils (4 each), the four levels
# of the recursion with their low-part sums (9 + 10 + 8 + 8) and the two
# Kahan updates (7)
IMPL_DRIVEN_CHAIN_FLOPS = 66
# classic stage-form RK4 of the Van der Pol chain (FMA = 2): per stage the
# stencil product B X (5), the slope -B X + g (1 - X^2) W (5) and the next
# stage's arguments (4); four stages less the first one's arguments, plus the
# weighted combination (9)
ALG_VDP_CHAIN_FLOPS = 61
# the register kernel's form (FMA = 2): B x with split coefficients (8), three
# high-coefficient stencils of the offsets (4 each), the four slopes with
# their offsets and the low parts' sums (11, 14, 14, 10) and the two Kahan
# updates (10)
IMPL_VDP_CHAIN_FLOPS = 79

WORKLOADS = {
    "c1": dict(kind="chain", method="rk4", prec="f64",
               desc="paper's two-mass system eq. (3): m=2, C=2025, dt=1e-5, 1e5 RK4 steps, FP64, 1 instance"),
    "c2": dict(kind="chain", method="rk4", prec="f32",
               desc="two-mass ensemble eq. (2): 2^20 instances, s=2, 1e4 RK4 steps, FP32"),
    "c2v": dict(kind="chain", method="verlet", prec="f32",
                desc="two-mass ensemble eq. (2): 2^20 instances, s=2, 1e4 Verlet steps, FP32"),
    "c3": dict(kind="chain", method="rk4", prec="f32",
               desc="fixed-free spring chain: 4096 instances, s=1024, 1e5 RK4 steps, FP32"),
    "c3v": dict(kind="chain", method="verlet", prec="f32",
                desc="fixed-free spring chain: 4096 instances, s=1024, 1e5 Verlet steps, FP32"),
    "c4": dict(kind="dense", method="rk4", prec="f32",
               desc="dense eq. (1), s=256, one A shared by 8192 instances, 1e4 RK4 steps, FP32 state, FP16x3 MFMA"),
    "c4v": dict(kind="dense", method="verlet", prec="f32",
                desc="dense eq. (1), s=256, one A shared by 8192 instances, 1e4 Verlet steps, FP32 state, FP16x3 MFMA"),
    "c1p": dict(kind="chain", method="rk4", prec="f64", propagator=2,
                desc="paper's two-mass system eq. (3): m=2, C=2025, dt=1e-5, 1e5 RK4 steps, FP64, 1 instance, "
                     "per-step propagator (the 4x4 step matrix)"),
    "c2p": dict(kind="chain", method="rk4", prec="f32", propagator=2,
                desc="two-mass ensemble eq. (2): 2^20 instances, s=2, 1e4 RK4 steps, FP32, "
                     "per-step propagator (one 4x4 step matrix per instance)"),
    "c2j": dict(kind="chain", method="rk4", prec="f32", propagator=1,
                desc="two-mass ensemble eq. (2): 2^20 instances, s=2, 1e4 RK4 steps, frames every 100 steps "
                     "by powers of the step matrix (FP64 state, FP32 in/out)"),
    "c4j": dict(kind="dense", method="rk4", prec="f32", propagator=1,
                desc="dense eq. (1), s=256, one A shared by 8192 instances, 1e4 RK4 steps, frames every 1000 steps "
                     "by powers of the step matrix (FP64 matrix cores, FP32 in/out)"),
    "c3d": dict(kind="chain", method="rk4", prec="f32", driven=True,
                desc="fixed-free spring chain: 4096 instances, s=1024, 1e4 RK4 steps, FP32, Rayleigh damping "
                     "(alpha=0.05, beta=1e-5) and a harmonic force per chain"),
    "c3n": dict(kind="chain", method="rk4", prec="f32", vdp=True,
                desc="coupled Van der Pol chains: the C3 chains (4096 instances, s=1024) with mu=20, 1e4 RK4 "
                     "steps, FP32"),
    "c4d": dict(kind="dense", method="rk4", prec="f32", driven=True,
                desc="dense eq. (1), s=256, one A shared by 8192 instances, 1e4 RK4 steps, FP32, Rayleigh damping "
                     "(alpha=0.02, beta=1e-3) and a harmonic force per instance (FP16 split MFMA)"),
    "c5": dict(kind="serve", method="rk4", prec="f32",
               desc="served stream: chains and dense SPD systems, s LogU[2,2048], nsteps LogU[1e3,1e5], FP32"),
}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_1702_02207_amd import workloads
    if name in ("c1", "c1p"):
        return workloads.c1_paper_two_mass(out_stride=1000)
    if name.startswith("c2"):
        w = workloads.c2_two_dof_ensemble()
        w.out_stride = 100 if name == "c2j" else w.nsteps
        return w
    if name == "c3n":
        w, mu = workloads.c3_vdp_chain()
        w.vdp_mu = mu
        return w
    if name == "c3d":
        w, ex = workloads.c3_driven_chain()
        w.excitation = ex
        return w
    if name.startswith("c3"):
        w = workloads.c3_spring_chain()
        w.out_stride = w.nsteps
        return w
    if name == "c4d":
        w, ex = workloads.c4_driven_dense()
        w.excitation = ex
        return w
    if name.startswith("c4"):
        return workloads.c4_dense_shared()
    raise SystemExit(f"unknown workload {name}")


# kernel sources that decide the dominant kernel of each workload family
TRAFFIC_SOURCES = {"chain": ("chain.hip", "chain_run.h", "osc_internal.h"), "dense": ("dense_mfma.hip", "osc_internal.h"),
                   "driven": ("driven.hip", "driven_run.h", "osc_internal.h"), "vdp": ("vdp.hip", "vdp_run.h", "osc_internal.h")}


def src_hash(workload):
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1702_02207_amd", "csrc")
    kind = ("dense" if workload.startswith("c4") else "driven" if workload == "c3d" else
            "vdp" if workload == "c3n" else "chain")
    for f in TRAFFIC_SOURCES[kind]:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the dominant kernel from rocprofv3 --pmc runs
    recorded in profiles/traffic.json, valid only while the kernel sources are
    unchanged since the counters were taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json"))).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("csrc_hash") != src_hash(workload):
        return None
    return rec.get("bytes_per_launch")


def host_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))


def sample_instances(batch, n, seed=1702022075):
    """Instance 0, the last instance and n - 2 seeded others in between."""
    import numpy as np
    if n >= batch:
        return np.arange(batch)
    rng = np.random.Generator(np.random.PCG64(seed))
    mid = rng.choice(np.arange(1, batch - 1), size=max(n - 2, 0), replace=False)
    return np.unique(np.concatenate([[0, batch - 1], mid]))


def cpu_baseline(w, kind, method, prec, idx):
    """Time the FP64 oracle on the sampled instances (full step count)."""
    import numpy as np
    import oracle
    sub = w.subset(idx)
    x0, v0 = sub.x0, sub.v0
    if prec == "f32":
        x0 = x0.astype(np.float32).astype(np.float64)
        v0 = v0.astype(np.float32).astype(np.float64)
    threads = host_threads()
    t0 = time.perf_counter()
    if getattr(w, "vdp_mu", None) is not None:
        xf, vf, _, _ = oracle.chain_vdp(sub.m, sub.k, sub.dt, w.vdp_mu, x0, v0, w.nsteps, w.out_stride)
    elif getattr(w, "excitation", None) is not None:
        ex = w.excitation.subset(idx)
        if kind == "chain":
            xf, vf, _, _ = oracle.chain_driven(sub.m, sub.k, sub.dt, ex.alpha, ex.beta, ex.F, ex.omega, x0, v0,
                                               w.nsteps, w.out_stride)
        else:
            xf, vf, _, _ = oracle.dense_driven(sub.M, sub.K, sub.dt, ex.alpha, ex.beta, ex.F, ex.omega, x0, v0,
                                               w.nsteps, w.out_stride, shared=sub.shared)
    elif kind == "chain":
        xf, vf, _, _ = oracle.chain(method, sub.m, sub.k, sub.dt, x0, v0, w.nsteps, w.out_stride)
    else:
        xf, vf, _, _ = oracle.dense(method, sub.M, sub.K, sub.dt, x0, v0, w.nsteps, w.out_stride,
                                    shared=sub.shared)
    el = time.perf_counter() - t0
    rate = len(idx) * w.s * w.nsteps / el
    return dict(value=rate, unit="DOF-steps/s", cores=min(threads, len(idx)), kind="oracle",
                sample=f"{len(idx)} of {w.batch} instances (instance 0, the last and seeded others), "
                       f"all {w.nsteps} steps, FP64 C oracle (OpenMP over instances)",
                seconds=round(el, 3)), (xf, vf)


def jump_roofline(w, kind, seconds):
    """Frame jumps: the two-mass ensemble's one kernel moves its inputs, the
    frames and the final state (HBM-bound); dense shared systems are FP64
    matrix-core products (rocBLAS DGEMM): the powers of the step matrix by
    repeated squaring (A^2, then squarings and multiplications of 2s x 2s
    matrices) and one (batch x 2s) x (2s x 2s) product per frame; seconds is
    the device time of the whole call."""
    nf = w.nsteps // w.out_stride + 1 if w.out_stride else 0
    rest = w.nsteps - (nf - 1) * w.out_stride if nf else w.nsteps
    if kind == "chain":
        elem = 4
        per_inst = (w.s * 2 * 8 + 8) + 2 * w.s * elem + (nf + 1) * 2 * w.s * elem   # m, k, h; x0, v0; frames, end
        byts = per_inst * w.batch
        achieved = byts / seconds / 1e9
        return dict(bound="hbm", achieved=round(achieved, 1), peak=8000.0, unit="GB/s",
                    frac=round(achieved / 8000.0, 4), traffic=None, kernel="small_jump_kernel",
                    kernel_ms=round(seconds * 1e3, 4), bytes_per_launch=int(byts))
    n = 2 * w.s
    squarings = max(int(w.out_stride if nf > 1 else 0).bit_length(), int(rest).bit_length()) - 1
    gemms = max(squarings, 0) + max(bin(int(w.out_stride)).count("1") - 1, 0) * (nf > 1) \
        + max(bin(int(rest)).count("1") - 1, 0) * (rest > 0)
    flops = 2.0 * w.s ** 3 + gemms * 2.0 * n ** 3 + ((nf - 1) + (rest > 0)) * 2.0 * n * n * w.batch
    achieved = flops / seconds / 1e12
    return dict(bound="mfma", achieved=round(achieved, 2), peak=PEAK["fp64"], unit="TFLOP/s",
                frac=round(achieved / PEAK["fp64"], 4), traffic=None, kernel="rocBLAS DGEMM (FP64 matrix cores)",
                kernel_ms=round(seconds * 1e3, 4), flops_per_launch=flops, matrix_products=gemms)


def bench_batched(args, name, spec):
    import numpy as np
    import torch
    from paper_1702_02207_amd import osc
    kind, method, prec = spec["kind"], spec["method"], spec["prec"]
    dev = torch.device("cuda:0")
    _log(f"[bench] generating workload {name}")
    w = make_workload(name)
    tdt = torch.float32 if prec == "f32" else torch.float64
    if kind == "chain":
        P1, P2, P3 = (torch.as_tensor(a, device=dev) for a in (w.m, w.k, w.dt))
    else:
        P1, P2, P3 = (torch.as_tensor(a, device=dev) for a in (w.M, w.K, w.dt))
    x0 = torch.as_tensor(w.x0, dtype=tdt, device=dev)
    v0 = torch.as_tensor(w.v0, dtype=tdt, device=dev)
    nf = w.nsteps // w.out_stride + 1
    xf = torch.empty((nf, w.batch, w.s), dtype=tdt, device=dev)
    vf = torch.empty_like(xf)
    xe, ve = torch.empty_like(x0), torch.empty_like(v0)
    stream = torch.cuda.current_stream()
    kern_ms = []

    mode = spec.get("propagator", 0)

    def make_system():
        if kind == "chain":
            sysm = osc.System("chain", method, prec, P1, P2, P3, stream=stream).create()
        else:
            sysm = osc.System("dense", method, prec, P1, P2, P3, shared=True, batch=w.batch, stream=stream).create()
        if mode:
            sysm.set_config(osc.CFG_PROPAGATOR, mode)
        if spec.get("driven"):
            ex = w.excitation
            sysm.set_excitation(ex.alpha, ex.beta, ex.F, ex.omega)
        if spec.get("vdp"):
            sysm.set_van_der_pol(w.vdp_mu)
        return sysm

    def one_step(record):
        sysm = make_system()
        a = b = None
        if record:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
        sysm.integrate(x0, v0, w.nsteps, w.out_stride, out=(xf, vf, xe, ve))
        if record:
            b.record(stream)
        sysm.energy(xe, ve)
        sysm.sync()
        sysm.close()
        if record:
            kern_ms.append(a.elapsed_time(b))

    for i in range(args.warmup):
        _log(f"[bench] warmup {i + 1}/{args.warmup}")
        one_step(False)
    torch.cuda.synchronize()
    _log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dof_steps = w.batch * w.s * w.nsteps
    value = dof_steps * args.steps / el
    ms_per_step = el / args.steps * 1e3
    _log(f"[bench] {value:.4e} DOF-steps/s, {ms_per_step:.3f} ms/step")

    kavg = float(np.mean(kern_ms)) * 1e-3
    if mode == 1:
        roofline = jump_roofline(w, kind, kavg)
    elif spec.get("driven") and kind == "dense":
        # stage form: four stages of B X and B W; issued: the recursion's FP16
        # passes (B x 3, B w 3 with stiffness damping, three level products)
        fpd = 8 * 2 * w.s
        passes = 3 + (3 if w.excitation.beta else 2) + 2 + (1 if w.excitation.beta else 0)
        achieved = fpd * dof_steps / kavg / 1e12
        hw = passes * 2 * w.s * dof_steps / kavg / 1e12
        peak = PEAK["fp16_mfma"]
        roofline = dict(bound="mfma", achieved=round(achieved, 2), peak=peak, unit="TFLOP/s",
                        frac=round(achieved / peak, 4), traffic=measured_traffic(name),
                        kernel="dense_mfma_kernel (damped, driven)", kernel_ms=round(kavg * 1e3, 4),
                        flops_per_dof_step=fpd, hw_mfma_tflops=round(hw, 1), hw_mfma_frac=round(hw / peak, 4))
    elif spec.get("vdp"):
        fpd = ALG_VDP_CHAIN_FLOPS
        achieved = fpd * dof_steps / kavg / 1e12
        roofline = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK["fp32"], unit="TFLOP/s",
                        frac=round(achieved / PEAK["fp32"], 4), traffic=measured_traffic(name),
                        kernel="vdp_chain_kernel", kernel_ms=round(kavg * 1e3, 4), flops_per_dof_step=fpd,
                        impl_flops_per_dof_step=IMPL_VDP_CHAIN_FLOPS,
                        impl_frac=round(IMPL_VDP_CHAIN_FLOPS * dof_steps / kavg / 1e12 / PEAK["fp32"], 4))
    elif spec.get("driven"):
        fpd = ALG_DRIVEN_CHAIN_FLOPS
        achieved = fpd * dof_steps / kavg / 1e12
        roofline = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK["fp32"], unit="TFLOP/s",
                        frac=round(achieved / PEAK["fp32"], 4), traffic=measured_traffic(name),
                        kernel="driven_chain_kernel",
                        kernel_ms=round(kavg * 1e3, 4), flops_per_dof_step=fpd,
                        impl_flops_per_dof_step=IMPL_DRIVEN_CHAIN_FLOPS,
                        impl_frac=round(IMPL_DRIVEN_CHAIN_FLOPS * dof_steps / kavg / 1e12 / PEAK["fp32"], 4))
    elif kind == "chain":
        fpd = (ALG_CHAIN2_FLOPS if w.s == 2 else ALG_CHAIN_FLOPS)[method]
        impl = IMPL_PROP_STEP_FLOPS if mode == 2 else IMPL_CHAIN_FLOPS[(method, prec)]
        achieved = fpd * dof_steps / kavg / 1e12
        peak = PEAK["fp32"] if prec == "f32" else PEAK["fp64"]
        roofline = dict(bound="alu", achieved=round(achieved, 3), peak=peak, unit="TFLOP/s",
                        frac=round(achieved / peak, 4), traffic=measured_traffic(name),
                        kernel="prop_step_kernel" if mode == 2 else "chain_kernel",
                        kernel_ms=round(kavg * 1e3, 4), flops_per_dof_step=fpd,
                        impl_flops_per_dof_step=impl,
                        impl_frac=round(impl * dof_steps / kavg / 1e12 / peak, 4))
    else:
        fpd = DENSE_PRODUCTS[method] * 2 * w.s
        achieved = fpd * dof_steps / kavg / 1e12
        hw = DENSE_HW_TERMS[method] * 2 * w.s * dof_steps / kavg / 1e12
        peak = PEAK["fp16_mfma"]
        roofline = dict(bound="mfma", achieved=round(achieved, 2), peak=peak, unit="TFLOP/s",
                        frac=round(achieved / peak, 4), traffic=measured_traffic(name), kernel="dense_mfma_kernel",
                        kernel_ms=round(kavg * 1e3, 4), flops_per_dof_step=fpd,
                        hw_mfma_tflops=round(hw, 1), hw_mfma_frac=round(hw / peak, 4))

    out = {
        "metric": "DOF-steps/sec batched vs plain at stated err; p50/p99 solve latency",
        "value": value, "unit": "DOF-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": spec["desc"], "batch": w.batch, "s": w.s, "nsteps": w.nsteps,
                   "method": method, "out_stride": w.out_stride,
                   "mode": {0: "time stepping", 1: "frame jumps by powers of the step matrix",
                            2: "per-step propagator"}[mode]},
        "roofline": roofline,
    }

    if not args.no_plain and not spec.get("driven") and not spec.get("vdp"):
        pn = min(args.plain_instances, w.batch)
        psteps = args.plain_steps or w.nsteps
        sub = w.subset(np.arange(pn))
        _log(f"[bench] plain integrator: {pn} instances x {psteps} steps, one step per launch")
        if kind == "chain":
            ps = osc.System("chain", method, prec, sub.m, sub.k, sub.dt, stream=stream).create()
        else:
            ps = osc.System("dense", method, prec, sub.M, sub.K, sub.dt, shared=True, batch=pn,
                            stream=stream).create()
        px0 = torch.as_tensor(sub.x0, dtype=tdt, device=dev)
        pv0 = torch.as_tensor(sub.v0, dtype=tdt, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ps.integrate_plain(px0, pv0, psteps)
        ps.sync()
        tp = time.perf_counter() - t1
        ps.close()
        plain_rate = pn * w.s * psteps / tp
        out["plain"] = {"value": plain_rate, "unit": "DOF-steps/s", "instances": pn, "steps": psteps,
                        "entry_point": "osc_integrate_plain",
                        "us_per_launch": tp / (pn * max(psteps, 1)) * 1e6}
        out["speedup_vs_plain"] = value / plain_rate

    if not args.no_cpu_baseline:
        n = args.cpu_sample or CPU_SAMPLE.get(name, 16)
        idx = sample_instances(w.batch, n)
        _log(f"[bench] oracle on {len(idx)} instances")
        cb, (rxf, rvf) = cpu_baseline(w, kind, method, prec, idx)
        out["cpu_baseline"] = cb
        import oracle
        gx = xf[:, torch.as_tensor(idx, device=dev)].double().cpu().numpy()
        gv = vf[:, torch.as_tensor(idx, device=dev)].double().cpu().numpy()
        ex = oracle.rel_traj_err(gx, rxf)
        ev = oracle.rel_traj_err(gv, rvf)
        out["error"] = {"max_rel_err_x": float(ex.max()), "max_rel_err_v": float(ev.max()),
                        "p99_rel_err_x": float(np.percentile(ex, 99)),
                        "p99_rel_err_v": float(np.percentile(ev, 99)),
                        "tolerance": TOL[prec], "instances_checked": int(len(idx)),
                        "frames_checked": int(nf),
                        "within_tolerance": bool(max(ex.max(), ev.max()) < TOL[prec])}
    return out


def serve_pass(args, method="rk4", prec="f32"):
    """The served stream: a burst of every request at once measures the
    saturation rate, then Poisson arrivals at args.load times that rate."""
    import numpy as np
    from paper_1702_02207_amd import serve, workloads
    _log(f"[bench] serving: generating {args.requests} requests")
    reqs = workloads.c5_request_stream(n_requests=args.requests, qps=1.0)
    work = sum(r.system.s * r.system.nsteps for r in reqs)
    _log("[bench] serving: burst (saturation)")
    sat = serve.run_stream(reqs, None, method=method, prec=prec, hbm_budget=args.hbm_budget)
    sat_qps = len(reqs) / sat["makespan_s"]
    qps = args.qps or args.load * sat_qps
    _log(f"[bench] serving: Poisson arrivals at {qps:.2f} requests/s")
    arr = serve.poisson_arrivals(len(reqs), qps, seed=1702022074)
    run = serve.run_stream(reqs, arr, method=method, prec=prec, hbm_budget=args.hbm_budget)
    _log("[bench] serving: the same arrivals, dense frames by jumps where much cheaper")
    jr = serve.run_stream(reqs, arr, method=method, prec=prec, hbm_budget=args.hbm_budget, frame_jumps=True)

    # slowdown against the request served alone, on a seeded sample that
    # always holds the largest request of each kind
    rng = np.random.default_rng(1702022076)
    work_of = np.array([r.system.s * r.system.nsteps for r in reqs])
    largest = [int(np.argmax(np.where([r.kind == k for r in reqs], work_of, -1))) for k in ("chain", "dense")]
    sample = sorted(set(largest) | set(rng.choice(len(reqs), min(args.slowdown_sample, len(reqs)), replace=False).tolist()))
    _log(f"[bench] serving: {len(sample)} requests alone (slowdown reference)")
    alone = serve.alone_latencies(reqs, sample, method=method, prec=prec, hbm_budget=args.hbm_budget)

    def slowdown(res):
        sl = {"chain": [], "dense": []}
        for i in sample:
            if res["results"][i] is not None:
                sl[reqs[i].kind].append(res["results"][i]["latency_s"] / alone[i])
        out = {}
        for kind, v in sl.items():
            if v:
                v = np.array(v)
                out[kind] = {"requests": int(v.size), "median": float(np.median(v)), "max": float(v.max())}
        return out

    def per_kind(res):
        d = {}
        for kind in ("chain", "dense"):
            lat = np.array([x["latency_s"] for r, x in zip(reqs, res["results"]) if x is not None and r.kind == kind])
            if lat.size:
                d[kind] = {"requests": int(lat.size), "p50_latency_s": float(np.percentile(lat, 50)),
                           "p99_latency_s": float(np.percentile(lat, 99))}
        return d

    return {
        "workload": WORKLOADS["c5"]["desc"], "requests": len(reqs), "qps": qps, "load": args.load,
        "hbm_budget": args.hbm_budget, "total_dof_steps": int(work),
        "p50_latency_s": run["p50_latency_s"], "p99_latency_s": run["p99_latency_s"],
        "mean_latency_s": run["mean_latency_s"], "dof_steps_per_s": run["dof_steps_per_s"],
        "makespan_s": run["makespan_s"], "per_kind": per_kind(run), "failed": run["failed"],
        "slowdown_vs_alone": slowdown(run), "alone_sample": len(sample),
        "hbm_peak_bytes": run["hbm_peak_bytes"], "iterations": run["iterations"],
        "worker_setup_s": run["worker_setup_s"], "worker_iterate_s": run["worker_iterate_s"],
        "frame_jumps": {
            "note": "same stream and arrivals; dense requests whose frames cost much less by powers of the "
                    "one-step matrix (FP64) are served that way: their steps are represented, not computed",
            "requests_by_jumps": len(jr["by_frame_jumps"]),
            "dof_steps_by_jumps": int(sum(reqs[i].system.s * reqs[i].system.nsteps for i in jr["by_frame_jumps"])),
            "p50_latency_s": jr["p50_latency_s"], "p99_latency_s": jr["p99_latency_s"],
            "mean_latency_s": jr["mean_latency_s"], "makespan_s": jr["makespan_s"], "per_kind": per_kind(jr),
            "failed": jr["failed"], "worker_setup_s": jr["worker_setup_s"]},
        "saturation": {"requests_per_s": sat_qps, "dof_steps_per_s": sat["dof_steps_per_s"],
                       "p50_latency_s": sat["p50_latency_s"], "p99_latency_s": sat["p99_latency_s"],
                       "per_kind": per_kind(sat), "slowdown_vs_alone": slowdown(sat)},
    }


def realtime_pass(args):
    """The paper's two-mass system (eq. (3), FP64, RK4, dt = 1e-5) stepped in
    real time: one step per wall-clock period, launched per tick (osc_rt_run)
    or by a resident kernel (osc_rt_run_resident); the latency from each
    release to the result being ready, as seen by the host."""
    import torch
    from paper_1702_02207_amd import osc, workloads
    w = workloads.c1_paper_two_mass(nsteps=1, out_stride=1)
    x0 = torch.as_tensor(w.x0, dtype=torch.float64, device="cuda:0")
    v0 = torch.as_tensor(w.v0, dtype=torch.float64, device="cuda:0")
    sysm = osc.System("chain", "rk4", "f64", w.m, w.k, w.dt).create()
    out = {"workload": "paper's two-mass system eq. (3), FP64 RK4, one step per period",
           "ticks_per_period": args.rt_ticks, "periods": []}
    try:
        # "launch": one kernel launch per tick (osc_rt_run); "resident": one
        # kernel on the device for the whole run, released through host-mapped
        # memory (osc_rt_run_resident)
        for mode in ("launch", "resident"):
            for period in (20e-6, 100e-6, 1e-3):
                _log(f"[bench] real-time ({mode}): period {period * 1e6:.0f} us, {args.rt_ticks} ticks")
                with osc.Realtime(sysm, x0, v0, 1) as rt:
                    run = rt.run if mode == "launch" else rt.run_resident
                    _, _, _, st = run(period, args.rt_ticks, frames=False)
                out["periods"].append({"mode": mode, "period_s": period, "p50_latency_s": st["p50_s"],
                                       "p99_latency_s": st["p99_s"], "max_latency_s": st["max_s"],
                                       "jitter_s": st["jitter_s"], "missed": int(st["missed"]),
                                       "gpu_p50_s": st["gpu_p50_s"], "launch_p99_s": st["launch_p99_s"]})
        # the same pair with a Van der Pol element on each mass (mu = 10): the
        # nonlinear coupled oscillators of section 1, on the resident kernel
        sysm.set_van_der_pol(10.0)
        out["van_der_pol"] = {"workload": "the same pair with a Van der Pol element on each mass, mu = 10",
                              "periods": []}
        for period in (20e-6, 100e-6):
            _log(f"[bench] real-time (resident, Van der Pol): period {period * 1e6:.0f} us, {args.rt_ticks} ticks")
            with osc.Realtime(sysm, x0, v0, 1) as rt:
                _, _, _, st = rt.run_resident(period, args.rt_ticks, frames=False)
            out["van_der_pol"]["periods"].append({"mode": "resident", "period_s": period,
                                                   "p50_latency_s": st["p50_s"], "p99_latency_s": st["p99_s"],
                                                   "max_latency_s": st["max_s"], "jitter_s": st["jitter_s"],
                                                   "missed": int(st["missed"])})
    finally:
        sysm.close()
    return out


def bench_serve(args, spec):
    sv = serve_pass(args, spec["method"], spec["prec"])
    return {
        "metric": "DOF-steps/sec batched vs plain at stated err; p50/p99 solve latency",
        "value": sv["dof_steps_per_s"], "unit": "DOF-steps/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": sv["makespan_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": spec["prec"], "data": "synthetic",
        "config": {"workload": spec["desc"], "requests": sv["requests"], "qps": sv["qps"],
                   "hbm_budget": args.hbm_budget, "total_dof_steps": sv["total_dof_steps"]},
        "serving": sv,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--plain-instances", type=int, default=64)
    ap.add_argument("--plain-steps", type=int, default=0, help="0 = workload default")
    ap.add_argument("--cpu-sample", type=int, default=0, help="0 = workload default (CPU_SAMPLE)")
    ap.add_argument("--no-serve", action="store_true", help="leave the served-stream pass out of the line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-realtime", action="store_true", help="leave the real-time stepping pass out of the line")
    ap.add_argument("--rt-ticks", type=int, default=1000, help="real-time pass: periods per tested period length")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--requests", type=int, default=200, help="c5: requests in the stream")
    ap.add_argument("--qps", type=float, default=0.0, help="c5: arrival rate (0 = load x saturation)")
    ap.add_argument("--load", type=float, default=0.5, help="c5: fraction of the saturation rate")
    ap.add_argument("--hbm-budget", type=int, default=32 << 30, help="c5: server HBM budget in bytes")
    ap.add_argument("--slowdown-sample", type=int, default=16,
                    help="served stream: requests also run alone for their slowdown (plus the largest of each kind)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain elementwise copy of 1 GiB (reads 1 GiB, writes 1 GiB) "
                         "to calibrate the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent instances would shard across GPUs with no collective).", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 2.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": x.numel() * 4, "bytes_written": y.numel() * 4}))
        return
    spec = WORKLOADS[args.workload]
    if spec["kind"] == "serve":
        out = bench_serve(args, spec)
    else:
        out = bench_batched(args, args.workload, spec)
        if not args.no_serve:
            out["serving"] = serve_pass(args)
        if not args.no_realtime:
            out["realtime"] = realtime_pass(args)
    for r in (out.get("serving") or {}), (out.get("serving") or {}).get("saturation", {}):
        r.pop("results", None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
