#!/usr/bin/env python3
"""Throughput benchmark of the batched oscillator integrator on one MI355X.

Default workload: 2^20 independent two-mass systems (eq. (2)), m1, m2 ~
LogU[0.5, 5], C1, C2 ~ LogU[1e2, 1e4], x0, v0 ~ N(0, 1), dt = 0.01/omega_max,
10^4 classic RK4 steps with FP32 state (synthetic, seeded).

One timed step is one pass of the whole hot path over the batch, with every
input already resident in HBM: osc_create from device-resident FP64
parameters (coefficients h^2 k/m split into FP32 hi + lo, stability bound),
osc_integrate (all 10^4 steps, frames at n = 0 and n = nsteps), osc_energy
(FP64 energy of the final state), osc_sync and osc_destroy.

Printed JSON line (rank 0): value = DOF-steps/s = batch * s * nsteps / step
time.  Also reported: the plain per-instance GPU integrator (one step per
launch) on a sample and the speedup over it, the roofline of the dominant
kernel, the FP64 oracle timed on the host cores on a bounded sample, and the
max relative trajectory error of the sampled instances against that oracle.
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

PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32 vector (published)
PEAK_FP64_TFLOPS = 78.6
TOL = {"f32": 1e-5, "f64": 1e-10}

# Algorithmic FP32 flops per DOF-step of the integrator arithmetic at the
# target precision (FMA = 2 flops): RK4 four B-products (B x with split
# coefficients 8, three others 4 each), two update polynomials (6 each) and
# two compensated sums (4 each) = 40; Verlet leapfrog: B x split 8, two
# compensated sums 4 each = 16.
FLOPS_PER_DOF_STEP = {"rk4": 40, "verlet": 16}

WORKLOADS = {
    "c2": dict(desc="two-mass ensemble eq. (2): 2^20 instances, s=2, 1e4 RK4 steps, FP32",
               method="rk4", prec="f32"),
    "c2v": dict(desc="two-mass ensemble eq. (2): 2^20 instances, s=2, 1e4 Verlet steps, FP32",
                method="verlet", prec="f32"),
    "c3": dict(desc="fixed-free chain: 4096 instances, s=1024, 1e5 RK4 steps, FP32",
               method="rk4", prec="f32"),
    "c3v": dict(desc="fixed-free chain: 4096 instances, s=1024, 1e5 Verlet steps, FP32",
                method="verlet", prec="f32"),
}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_1702_02207_amd import workloads
    if name.startswith("c2"):
        w = workloads.c2_two_dof_ensemble()
        w.out_stride = w.nsteps
        return w
    if name.startswith("c3"):
        w = workloads.c3_spring_chain()
        w.out_stride = w.nsteps
        return w
    raise SystemExit(f"unknown workload {name}")


def src_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1702_02207_amd", "csrc"))):
        h.update(open(os.path.join(ROOT, "paper_1702_02207_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the dominant kernel from rocprofv3 --pmc runs
    recorded in profiles/traffic.json, valid only while the kernel sources
    are unchanged since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(p)).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("csrc_hash") != src_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(w, method, sample_n):
    """Time the FP64 oracle on the first sample_n instances (full step count)."""
    import numpy as np
    import oracle
    idx = np.arange(min(sample_n, w.batch))
    sub = w.subset(idx)
    x0 = sub.x0.astype(np.float32).astype(np.float64)
    v0 = sub.v0.astype(np.float32).astype(np.float64)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    t0 = time.perf_counter()
    xf, vf, xe, ve = oracle.chain(method, sub.m, sub.k, sub.dt, x0, v0, w.nsteps, w.out_stride)
    el = time.perf_counter() - t0
    rate = len(idx) * w.s * w.nsteps / el
    return dict(value=rate, unit="DOF-steps/s", cores=threads, kind="oracle",
                sample=f"first {len(idx)} of {w.batch} instances, all {w.nsteps} steps, FP64 C oracle",
                seconds=round(el, 3)), (idx, xf, vf)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--plain-instances", type=int, default=64)
    ap.add_argument("--plain-steps", type=int, default=0, help="0 = full step count")
    ap.add_argument("--cpu-sample", type=int, default=65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain elementwise copy of 1 GiB (reads 1 GiB, writes 1 GiB) "
                         "to calibrate the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent instances would shard across GPUs with no collective).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1702_02207_amd import osc

    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 2.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": x.numel() * 4, "bytes_written": y.numel() * 4}))
        return

    spec = WORKLOADS[args.workload]
    method, prec = spec["method"], spec["prec"]
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    _log(f"[bench] generating workload {args.workload}")
    w = make_workload(args.workload)
    tdt = torch.float32 if prec == "f32" else torch.float64
    # inputs resident in HBM before timing
    m_d = torch.as_tensor(w.m, device=dev)
    k_d = torch.as_tensor(w.k, device=dev)
    dt_d = torch.as_tensor(w.dt, device=dev)
    x0 = torch.as_tensor(w.x0, dtype=tdt, device=dev)
    v0 = torch.as_tensor(w.v0, dtype=tdt, device=dev)
    nf = w.nsteps // w.out_stride + 1
    xf = torch.empty((nf, w.batch, w.s), dtype=tdt, device=dev)
    vf = torch.empty_like(xf)
    xe = torch.empty_like(x0)
    ve = torch.empty_like(v0)
    E = torch.empty(w.batch, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    kern_ms = []

    def one_step(record):
        sysm = osc.System("chain", method, prec, m_d, k_d, dt_d, stream=stream).create()
        if record:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
        sysm.integrate(x0, v0, w.nsteps, w.out_stride, out=(xf, vf, xe, ve))
        if record:
            b.record(stream)
        osc_E = sysm.energy(xe, ve)
        sysm.sync()
        sysm.close()
        if record:
            kern_ms.append(a.elapsed_time(b))
        return osc_E

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

    # roofline of the dominant kernel (the integration launch)
    kavg = float(np.mean(kern_ms)) * 1e-3
    flops = FLOPS_PER_DOF_STEP[method] * dof_steps
    achieved = flops / kavg / 1e12
    peak = PEAK_FP32_TFLOPS if prec == "f32" else PEAK_FP64_TFLOPS
    traffic = measured_traffic(args.workload)
    roofline = dict(bound="alu", achieved=round(achieved, 2), peak=peak, unit="TFLOP/s",
                    frac=round(achieved / peak, 4), traffic=traffic,
                    kernel="chain_kernel", kernel_ms=round(kavg * 1e3, 4),
                    flops_per_dof_step=FLOPS_PER_DOF_STEP[method])

    out = {
        "metric": "DOF-steps/sec batched vs plain at stated err; p50/p99 solve latency",
        "value": value, "unit": "DOF-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": spec["desc"], "batch": w.batch, "s": w.s, "nsteps": w.nsteps,
                   "method": method, "out_stride": w.out_stride},
        "roofline": roofline,
    }

    # plain per-instance integrator (one step per launch) on a sample
    if not args.no_plain:
        pn = min(args.plain_instances, w.batch)
        psteps = args.plain_steps or w.nsteps
        sub = w.subset(np.arange(pn))
        _log(f"[bench] plain integrator: {pn} instances x {psteps} steps")
        ps = osc.System("chain", method, prec, sub.m, sub.k, sub.dt, stream=stream).create()
        px0 = torch.as_tensor(sub.x0, dtype=tdt, device=dev)
        pv0 = torch.as_tensor(sub.v0, dtype=tdt, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pxe, pve = ps.integrate_plain(px0, pv0, psteps)
        ps.sync()
        tp = time.perf_counter() - t1
        ps.close()
        plain_rate = pn * w.s * psteps / tp
        out["plain"] = {"value": plain_rate, "unit": "DOF-steps/s", "instances": pn, "steps": psteps,
                        "us_per_launch": tp / (pn * psteps) * 1e6}
        out["speedup_vs_plain"] = value / plain_rate
        if psteps == w.nsteps:
            d = (pxe.double() - xe[:pn].double()).abs().max().item()
            out["plain"]["max_abs_diff_vs_batched"] = d

    # CPU baseline: the oracle on a bounded sample; the same sample gives the error
    if not args.no_cpu_baseline:
        _log(f"[bench] oracle on {min(args.cpu_sample, w.batch)} instances")
        cb, (idx, rxf, rvf) = cpu_baseline(w, method, args.cpu_sample)
        out["cpu_baseline"] = cb
        import oracle
        gx = xf[:, :len(idx)].double().cpu().numpy()
        gv = vf[:, :len(idx)].double().cpu().numpy()
        ex = oracle.rel_traj_err(gx, rxf)
        ev = oracle.rel_traj_err(gv, rvf)
        out["error"] = {"max_rel_err_x": float(ex.max()), "max_rel_err_v": float(ev.max()),
                        "p99_rel_err_x": float(np.percentile(ex, 99)),
                        "p99_rel_err_v": float(np.percentile(ev, 99)),
                        "tolerance": TOL[prec], "instances_checked": int(len(idx)),
                        "within_tolerance": bool(max(ex.max(), ev.max()) < TOL[prec])}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
