"""Benchmark of the projection hot path on one MI355X.

Default workload: one Algorithm 3 step (step size, conjugate direction,
rho~, single-row projection, stop test) on the 256x128x128 single-constraint
case (n = 4,194,304, float32 streams), i.e. one pgdto_pgd_step launch per
step.  Inputs are synthetic (seeded), resident in HBM before timing; steps
rotate over several independent instances whose combined footprint exceeds
the 256 MB Infinity Cache, so every step reads its inputs from HBM.

Prints one JSON line (see the design doc for every field's definition).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="pgd_compliance",
                    choices=["pgd_compliance", "project_compliance", "multimaterial", "volcom"])
    ap.add_argument("--instances", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (HBM counter calibration)")
    return ap.parse_args()


# HBM traffic of the timed kernel, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of this script (summaries under profiles/), per launch and
# scaled by the same counters on a plain 1 GiB copy.  Reported only while the
# kernel source is the one that was measured (sha256 of the HIP file).
KERNEL_SRC = os.path.join(ROOT, "paper_2511_13905_amd", "csrc", "pgdto_kernels.hip")
MEASURED_TRAFFIC = {
    # profiles/k_solve_1d_f32_pgd_compliance_hbm_traffic.md
    "pgd_compliance": {"kernel_sha": "2633e7d790b0806e", "bytes_per_launch": 278090623,
                       "read": 191416134, "written": 86674490},
}


def kernel_sha():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(workload):
    m = MEASURED_TRAFFIC.get(workload)
    if not m or m["kernel_sha"] != kernel_sha():
        return None
    return m["bytes_per_launch"]


def copy_calibration():
    """A plain elementwise copy of 1 GiB (read 1 GiB, write 1 GiB), 5 times."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 5,
                                           "kernel": "elementwise mul by 1.0 (float32)"}}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described in DESIGN.md, not built)"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2511_13905_amd import inputs as I
    from paper_2511_13905_amd.api import Context, result_from_bytes, result_nbytes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    ctx = Context(0)
    stream = torch.cuda.current_stream(dev)

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    R = max(1, args.instances)
    insts = []
    wl = args.workload
    if wl == "pgd_compliance":
        for s in range(R):
            st = I.pgd_compliance_3d(s, t=60)
            insts.append(dict(A=T(st.problem.A), rho=T(st.rho), rho_prev=T(st.rho_prev), grad=T(st.grad),
                              grad_prev=T(st.grad_prev), d=T(st.d_prev), g=st.g, G=st.G, t=st.t,
                              x=torch.empty_like(T(st.rho)), st=st))
        n = insts[0]["rho"].numel()
        m = 1
        kind = "single"
        dtype = "f32"
        workload = "pgd_step, single linearized compliance row, 256x128x128 grid (n=4194304), float32 streams"
    else:
        gen = {"project_compliance": lambda s: I.compliance_3d(s),
               "multimaterial": lambda s: I.multi_material(s),
               "volcom": lambda s: I.volume_com(s)}[wl]
        for s in range(R):
            p = gen(s)
            insts.append(dict(p=p, y=T(p.y), A=T(p.A), x=torch.empty(p.n, dtype=torch.float32, device=dev)))
        p0 = insts[0]["p"]
        n, m, kind = p0.n, p0.m, p0.kind
        dtype = "f32"
        workload = {"project_compliance": "project, single compliance row, 256x128x128 (n=4194304), float32",
                    "multimaterial": "project, 4 independent volume blocks of 524288 (n=2097152), float32",
                    "volcom": "project, volume + centre-of-mass m=5 coupled, 192x96x96 (n=1769472), float32, "
                              "even seeds feasible / odd seeds infeasible"}[wl]

    is_pgd = wl == "pgd_compliance"
    nres = result_nbytes(pgd=is_pgd)
    res_bufs = [torch.zeros(nres, dtype=torch.uint8, device=dev) for _ in range(R)]

    def launch(i):
        it = insts[i % R]
        if is_pgd:
            ctx.pgd_step_async("single", it["A"], it["rho"], it["rho_prev"], it["grad"], it["grad_prev"], it["d"],
                               it["g"], it["G"], it["t"], I.LO, I.HI, res_bufs[i % R], x=it["x"])
        else:
            p = it["p"]
            ctx.project_async(p.kind, it["y"], it["A"], p.b, p.lo, p.hi, res_bufs[i % R], C=p.C,
                              offsets=p.offsets, x=it["x"])

    for i in range(args.warmup):
        launch(i)
    torch.cuda.synchronize()

    # per-launch kernel durations (HIP events on the launch stream)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    for i in range(args.steps):
        evs[i][0].record(stream)
        launch(i)
        evs[i][1].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    per = [a.elapsed_time(b) for a, b in evs]
    ms_step = total_ms / args.steps
    kern_ms = sum(per) / len(per)
    per_sorted = sorted(per)
    p50 = per_sorted[len(per) // 2]
    p99 = per_sorted[min(len(per) - 1, int(math.ceil(0.99 * len(per))) - 1)]

    # passes taken (algorithmic bytes follow the algorithm's own pass count)
    results = [result_from_bytes(b, pgd=is_pgd) for b in res_bufs]
    proj = [r["proj"] if is_pgd else r for r in results]
    passes = sum(r["passes"] for r in proj) / len(proj)
    errors = [r["error"] for r in proj]
    esz = 4
    if is_pgd:
        # pass R: rho, rho_prev, grad, grad_prev, a; pass D+0: rho, grad, d, a read, d, rho~ written;
        # each search pass: rho~, a; final: rho~, a, rho read, x written
        search_passes = passes - 3
        bytes_launch = n * esz * (5 + 6 + 2 * search_passes + 4)
        compulsory = n * esz * (6 + 2)
    else:
        rows = m if kind == "coupled" else 1
        per_pass = n * esz * (1 + rows)
        bytes_launch = passes * per_pass + n * esz          # final pass also writes x
        compulsory = n * esz * (1 + rows + 1)
    achieved = bytes_launch / (kern_ms * 1e-3)
    value = n / (ms_step * 1e-3)

    line = {
        "metric": "projected elements/s and % HBM roofline; p50/p99 batched projection latency",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": workload, "instances_rotated": R, "passes_per_launch": passes,
                   "latency_ms": {"p50": p50, "p99": p99}, "wall_s": wall, "device_errors": errors,
                   "kernel_sha": kernel_sha()},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK, "traffic": traffic_for(wl),
                     "bytes_per_launch": bytes_launch, "kernel_ms": kern_ms},
        "roofline_compulsory": {"bytes": compulsory, "achieved": compulsory / (kern_ms * 1e-3) / 1e9,
                                "unit": "GB/s", "frac": compulsory / (kern_ms * 1e-3) / HBM_PEAK},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, insts, args.cpu_seconds, n)
    ctx.close()
    print(json.dumps(line), flush=True)


def cpu_baseline(wl, insts, budget_s, n):
    """The CPU oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np
    import oracle
    from paper_2511_13905_amd import inputs as I
    done = 0
    t0 = time.perf_counter()
    while done < len(insts) and time.perf_counter() - t0 < budget_s:
        it = insts[done]
        if wl == "pgd_compliance":
            st = it["st"]
            oracle.pgd_step("single", st.rho, st.rho_prev, st.grad, st.grad_prev, st.d_prev, st.problem.A,
                            st.g, st.G, st.t, I.LO, I.HI, stream_dtype=np.float32)
        else:
            p = it["p"]
            oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C, p.offsets)
        done += 1
    el = time.perf_counter() - t0
    return {"value": done * n / el, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} full-size instance(s) of the same workload in {el:.1f} s (numpy float64, one thread)"}


if __name__ == "__main__":
    main()
