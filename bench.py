"""Benchmark of the projection hot path on one MI355X.

Default workload (one step = one launch): one Algorithm 3 step (step size,
conjugate direction, rho~, single-row projection, stop test) on each of 16
distinct instances of the 256x128x128 single-constraint case (n = 4,194,304
each, float32 streams), solved together by one pgdto_pgd_step_batch_async
launch.  The 16 instances (1.9 GB) are far larger than the 256 MB Infinity
Cache, so every pass reads its inputs from HBM.  Inputs are synthetic
(seeded) and resident in HBM before timing.

Prints one JSON line: the metric, throughput and latency of the timed steps,
the roofline of the batch kernel (algorithmic bytes per launch over the
launch time from HIP events on the launch stream, and the HBM traffic that
rocprofv3 counters measured for the same kernel source), the one-instance
launch (warm and after a 1 GB cache flush), the CPU oracle's rate on the
host (one thread and a process pool) and the error against it, and the
served-stream and server-route batch measurements.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
ESZ = 4                    # float32 streams


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="pgd_compliance",
                    choices=["pgd_compliance", "project_compliance", "multimaterial", "volcom"])
    ap.add_argument("--batch", type=int, default=16, help="distinct instances per launch")
    ap.add_argument("--slots", type=int, default=0, help="slots of the batch launch (0: pick by a short sweep)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-serve", action="store_true", help="skip the served-stream and server-route batch")
    ap.add_argument("--no-single", action="store_true", help="skip the one-instance launch measurements")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--serve-pool", type=int, default=128,
                    help="distinct request instances the served stream cycles through")
    ap.add_argument("--compact", action="store_true", help="turn the free-set compaction on")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="processes that generate the inputs (1 under a profiler)")
    ap.add_argument("--wide-m", default="32,64",
                    help="row counts of the many-row coupled leg (wide kernel), comma separated; empty: skip")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (HBM counter calibration)")
    ap.add_argument("--wide-only", action="store_true",
                    help="run only the many-row coupled leg (--wide-m): the command the wide kernel "
                         "profiles are taken with")
    ap.add_argument("--single-only", action="store_true",
                    help="run only the one-instance launches (no batch, server or wide legs): the command "
                         "the one-instance kernel profiles are taken with")
    return ap.parse_args()


# HBM traffic of the timed kernel, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of this script (summaries under profiles/), per launch and
# scaled by the same counters on a plain 1 GiB copy.  Reported only while the
# kernel sources are the ones that were measured (sha256 over the files).
CSRC = os.path.join(ROOT, "paper_2511_13905_amd", "csrc")
KERNEL_SRC = [os.path.join(CSRC, f) for f in ("pgdto_internal.h", "pgdto_device.h", "pgdto_kernels.hip")]
WIDE_SRC = [os.path.join(CSRC, f) for f in ("pgdto_internal.h", "pgdto_device.h", "pgdto_wide.hip")]
MEASURED_TRAFFIC = {
    # profiles/k_batch_f32_pgd_compliance_b16_hbm_traffic.md
    "pgd_compliance": {"kernel_sha": "2c988a558aedc463", "bytes_per_launch": 6713519145,
                       "read": 5885478935, "written": 828040210, "instances": 16},
}


# the same for one-instance launches (bench.py --single-only; profiles/k_solve_*_hbm_traffic.md),
# per launch, means over the timed launches of the workload's four instances
SINGLE_MEASURED_TRAFFIC = {
    "pgd_compliance": {"kernel_sha": "2c988a558aedc463", "bytes_per_launch": 196753538},
    "project_compliance": {"kernel_sha": "2c988a558aedc463", "bytes_per_launch": 56435242},
    "multimaterial": {"kernel_sha": "2c988a558aedc463", "bytes_per_launch": 31294599},
    "volcom": {"kernel_sha": "2c988a558aedc463", "bytes_per_launch": 518471577},
}


# the same for the wide coupled kernel's launches (one projection each), by row count
# (profiles/k_solve_wide_f32_many_rows_hbm_traffic.md)
WIDE_MEASURED_TRAFFIC = {
    64: {"kernel_sha": "02848ea381ddf98d", "bytes_per_launch": 20462464119, "read": 20312890035,
         "written": 149574085},
    32: {"kernel_sha": "02848ea381ddf98d", "bytes_per_launch": 6704075485, "read": 6664916198,
         "written": 39159287},
}


def kernel_sha(files=None):
    import hashlib
    h = hashlib.sha256()
    for path in files or KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(workload, instances):
    m = MEASURED_TRAFFIC.get(workload)
    if not m or m["kernel_sha"] != kernel_sha() or m["instances"] != instances:
        return None
    return m


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


# ---------------------------------------------------------------- inputs
def _gen_pgd(seed):
    from paper_2511_13905_amd import inputs as I
    return I.pgd_compliance_3d(seed, t=60)


def _gen_proj(wl_seed):
    from paper_2511_13905_amd import inputs as I
    wl, seed = wl_seed
    return {"project_compliance": I.compliance_3d, "multimaterial": I.multi_material,
            "volcom": I.volume_com}[wl](seed)


WIDE_SEED = 7


def _gen_wide(m):
    """The many-row coupled instance of the wide leg and its candidate rows
    (violated at lam = 0), from float64 dot products of the rounded arrays."""
    import numpy as np
    from paper_2511_13905_amd import inputs as I
    p = I.many_rows(WIDE_SEED, m=m)
    x0 = np.clip(p.y.astype(np.float64), p.lo, p.hi)
    h0 = np.array([float(np.dot(p.A[j].astype(np.float64), x0)) for j in range(m)]) - p.b
    return p, int(np.count_nonzero(h0 > 0.0))


def generate(fn, args, workers, side=None):
    """Seeded instances, generated in a process pool (before the GPU is
    touched); side(), if given, runs in this process meanwhile."""
    if workers <= 1 or len(args) <= 1:
        out = [fn(a) for a in args]
        return out, (side() if side else None)
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(workers, len(args))) as pool:
        res = pool.map_async(fn, args)
        extra = side() if side else None
        return res.get(), extra


def host_cpu():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


# ---------------------------------------------------------------- byte model
def compact_split(r):
    """(search passes over every element, kept pairs, passes over the kept
    pairs only) of one result: the free-set compaction pass reads every
    element and writes the kept (y, a) pairs; later search passes read only
    those pairs."""
    kept = max(0, r.get("n_compact", -1))
    pc = r.get("passes_compacted", 0) if r.get("n_compact", -1) >= 0 else 0
    return r["iters_search"] - pc, kept, pc


def pgd_bytes(n, r):
    """Algorithmic bytes of one pgd_step (float32 streams): pass R reads
    rho, rho_prev, grad, grad_prev, a; the zero pass reads rho, grad, d, a and
    writes d, rho~; each full search pass reads rho~, a (the compaction pass
    also writes the kept pairs, each later pass reads them); the final pass
    reads rho~, a, rho and writes x."""
    full, kept, pc = compact_split(r)
    return n * ESZ * (5 + 6 + 2 * full + 4) + kept * 2 * ESZ * (1 + pc)


def proj_bytes(n, rows, r):
    """Every full pass reads y and the rows (kept pairs as above for the
    1-D searches); the final pass also writes x."""
    full, kept, pc = compact_split(r)
    other = r["passes"] - r["iters_search"]          # zero pass, Stage 1, Newton, final ...
    return (other + full) * n * ESZ * (1 + rows) + n * ESZ + kept * 2 * ESZ * (1 + pc)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    cpu = host_cpu()
    workers = max(1, min(args.gen_workers, cpu["usable_cpus"]))
    wl = args.workload
    B = max(1, args.batch)
    t_gen = time.perf_counter()
    wide_ms = [int(v) for v in args.wide_m.split(",") if v.strip()]
    wide_gen = (lambda: [_gen_wide(m) for m in wide_ms]) if wide_ms else None
    if args.wide_only:
        states, wide_insts = [], (wide_gen() if wide_gen else [])
    elif wl == "pgd_compliance":
        states, wide_insts = generate(_gen_pgd, list(range(B)), workers, wide_gen)
    else:
        states, wide_insts = generate(_gen_proj, [(wl, s) for s in range(B)], workers, wide_gen)
    t_gen = time.perf_counter() - t_gen

    # the CPU oracle runs before the GPU is initialised (its process pool forks)
    cpu_line, refs = (None, [])
    if not args.no_cpu_baseline and not args.wide_only:
        cpu_line, refs = cpu_baseline(wl, states, args.cpu_seconds, workers, cpu)

    import numpy as np
    import torch
    from paper_2511_13905_amd import inputs as I
    from paper_2511_13905_amd.api import Context, aligned_rows, close_all, result_from_bytes, result_nbytes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    ctx = Context(0)
    stream = torch.cuda.current_stream(dev)

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    if args.wide_only:
        out = {"wide_rows": [wide_bench(ctx, p, ncand, args) for p, ncand in wide_insts]}
        close_all()
        torch.cuda.synchronize()
        print(json.dumps(out), flush=True)
        return

    is_pgd = wl == "pgd_compliance"
    if is_pgd:
        insts = [dict(kind="single", A=T(st.problem.A), rho=T(st.rho), rho_prev=T(st.rho_prev), grad=T(st.grad),
                      grad_prev=T(st.grad_prev), d=T(st.d_prev), g=st.g, G=st.G, t=st.t, lo=I.LO, hi=I.HI)
                 for st in states]
        for it in insts:
            it["x"] = torch.empty_like(it["rho"])
            it["work"] = torch.empty_like(it["rho"])     # free-set compaction scratch
        n, m, rows = insts[0]["rho"].numel(), 1, 1
        workload = (f"pgd_step on {B} distinct instances per launch, single linearized compliance row, "
                    "256x128x128 grid (n=4194304 each), float32 streams")
    else:
        insts = []
        for p in states:
            A = T(p.A)
            if p.kind != "independent":
                A = aligned_rows(A)
            insts.append(dict(p=p, y=T(p.y), A=A, x=torch.empty(p.n, dtype=torch.float32, device=dev)))
        p0 = states[0]
        n, m = p0.n, p0.m
        rows = m if p0.kind == "coupled" else 1
        workload = {"project_compliance": "project, single compliance row, 256x128x128 (n=4194304)",
                    "multimaterial": "project, 4 independent volume blocks of 524288 (n=2097152)",
                    "volcom": "project, volume + centre-of-mass m=5 coupled, 192x96x96 (n=1769472), "
                              "even seeds feasible / odd seeds infeasible"}[wl]
        workload = f"{workload} on {B} distinct instances per launch, float32"
    if args.single_only:
        out = {"workload": workload.replace(f" on {B} distinct instances per launch", "") + ", one-instance launches",
               "single_instance": single_bench(ctx, insts, is_pgd, n, rows, args), "kernel_sha": kernel_sha()}
        close_all()
        del insts
        torch.cuda.synchronize()
        print(json.dumps(out), flush=True)
        return
    nres = result_nbytes(pgd=is_pgd)
    res_buf = torch.zeros(nres * B, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    params = {"compact": 1 if args.compact else 0}

    def launch(slots):
        if is_pgd:
            ctx.pgd_step_batch_async(insts, res_buf, slots=slots, params=params)
        else:
            ctx.project_batch_async([(it["p"].kind, it["y"], it["A"], it["p"].b, it["p"].lo, it["p"].hi, it["p"].C,
                                      it["p"].offsets, it["x"]) for it in insts], res_buf, slots=slots, params=params)

    def timed(slots, k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            launch(slots)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    # slot count of the batch launch: a short sweep (each candidate warmed once)
    sweep = {}
    if args.slots > 0:
        slots = args.slots
    else:
        for s in (4, 8, 16):
            if s > B:
                continue
            timed(s, 1)
            sweep[str(s)] = timed(s, 3)
        slots = int(min(sweep, key=sweep.get)) if sweep else 0
    for _ in range(args.warmup):
        launch(slots)
    torch.cuda.synchronize()

    # per-launch kernel durations (HIP events on the launch stream)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for i in range(args.steps):
        evs[i][0].record(stream)
        launch(slots)
        evs[i][1].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = t0.elapsed_time(t1) / args.steps
    per = sorted(a.elapsed_time(b) for a, b in evs)
    kern_ms = sum(per) / len(per)
    grid, tiles = ctx.last_launch()

    results = [result_from_bytes(res_buf[i * nres:(i + 1) * nres], pgd=is_pgd) for i in range(B)]
    proj = [r["proj"] if is_pgd else r for r in results]
    passes = [r["passes"] for r in proj]
    errors = [r["error"] for r in proj]
    if is_pgd:
        bytes_launch = sum(pgd_bytes(n, r) for r in proj)
        compulsory = B * n * ESZ * (6 + 2)
    else:
        bytes_launch = sum(proj_bytes(st.n, rows, r) for st, r in zip(states, proj))
        compulsory = sum(st.n * ESZ * (rows + 2) for st in states)
    elems = B * n if is_pgd else sum(st.n for st in states)
    achieved = bytes_launch / (kern_ms * 1e-3)
    tr = traffic_for(wl, B)
    line = {
        "metric": "projected elements/s and % HBM roofline; p50/p99 batched projection latency",
        "value": elems / (ms_step * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "instances_per_launch": B, "elements_per_launch": elems,
                   "slots": slots, "slot_sweep_ms": sweep, "grid_workgroups": grid, "tiles_per_instance": tiles,
                   "passes_per_instance": {"mean": sum(passes) / B, "min": min(passes), "max": max(passes)},
                   "compaction": {"on": bool(args.compact),
                                  "kept_fraction_mean": sum(max(0, r["n_compact"]) for r in proj) / B / n,
                                  "passes_on_kept_mean": sum(r["passes_compacted"] for r in proj) / B},
                   "latency_ms": {"p50": per[len(per) // 2],
                                  "p99": per[min(len(per) - 1, int(math.ceil(0.99 * len(per))) - 1)]},
                   "wall_s": wall, "device_errors": sorted(set(errors)), "kernel_sha": kernel_sha(),
                   "input_generation_s": t_gen},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK, "traffic": tr["bytes_per_launch"] if tr else None,
                     "kernel": "k_batch", "bytes_per_launch": bytes_launch, "kernel_ms": kern_ms},
        "roofline_compulsory": {"bytes": compulsory, "achieved": compulsory / (kern_ms * 1e-3) / 1e9,
                                "unit": "GB/s", "frac": compulsory / (kern_ms * 1e-3) / HBM_PEAK},
    }
    if tr:
        line["roofline"]["traffic_read"] = tr["read"]
        line["roofline"]["traffic_written"] = tr["written"]
        line["roofline"]["traffic_frac"] = tr["bytes_per_launch"] / (kern_ms * 1e-3) / HBM_PEAK
    if not args.no_single:
        line["single_instance"] = single_bench(ctx, insts, is_pgd, n, rows, args)
    if not args.no_serve:
        line["serving"] = serve_bench(ctx, args)
        if wl == "project_compliance":
            line["server_batch"] = server_batch_bench(ctx, insts, args)
    if wide_insts:
        line["wide_rows"] = [wide_bench(ctx, p, ncand, args) for p, ncand in wide_insts]
    if cpu_line is not None:
        line["cpu_baseline"] = cpu_line
        line["oracle_error"] = oracle_error(ctx, wl, states, insts, refs)
    # explicit teardown: executors and contexts, then the device, before exit
    close_all()
    del insts, res_buf
    torch.cuda.synchronize()
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- many coupled rows
MFMA_F32_PEAK = 157.3e12      # dense matrix-core peak, float32 (MI355X)
MFMA_F64_PEAK = 78.6e12       # dense matrix-core peak, float64


def wide_work(n, m, r, ncand):
    """Algorithmic work of one wide-kernel solve.  Each Newton pass forms
    h (m sums) and the m (m + 1) / 2 Jacobian sums of eq. reg_jacobian
    (2 flops per element each, float32 matrix cores); each candidate-check
    pass (Stage-1 exit test) the nc x m sums a_k.x(lam_j e_j), nc <= 16
    candidates per pass (float64 matrix cores).  Every pass reads y and the
    m rows; the final pass writes x."""
    newton = r["iters_ls"]
    checks = max(0, r["passes"] - 2 - r["iters_search"] - newton)
    f32 = newton * n * m * (m + 1)
    f64 = sum(2 * n * m * min(16, ncand - 16 * i) for i in range(checks))
    nbytes = r["passes"] * n * ESZ * (m + 1) + n * ESZ
    return f32, f64, nbytes, checks


def wide_bench(ctx, p, ncand, args):
    """One-instance launches of the wide coupled kernel (m dense rows,
    256x128x128 elements): the launch time from HIP events on the launch
    stream, and the per-pass times of one more launch on a tracing context."""
    import torch
    from paper_2511_13905_amd.api import Context, aligned_rows, result_from_bytes, result_nbytes
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    y = torch.from_numpy(p.y).to(dev)
    A = aligned_rows(torch.from_numpy(p.A).to(dev))
    x = torch.empty_like(y)
    buf = torch.zeros(result_nbytes(), dtype=torch.uint8, device=dev)

    def launch(c):
        c.project_async("coupled", y, A, p.b, p.lo, p.hi, buf, C=p.C, x=x)

    for _ in range(2):
        launch(ctx)
    torch.cuda.synchronize()
    K = max(4, min(args.steps, 10))
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for i in range(K):
        evs[i][0].record(stream)
        launch(ctx)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in evs)
    mean_ms = sum(ms) / K
    r = result_from_bytes(buf)
    grid = list(ctx.last_launch())
    n, m = p.n, p.m
    f32, f64, nbytes, checks = wide_work(n, m, r, ncand)
    lam = r["lam"]
    planted = p.meta["planted_lambda"]
    lam_err = max(abs(a - b) for a, b in zip(lam, planted)) / max(abs(v) for v in planted)
    # per-pass times of one launch on a tracing context
    os.environ["PGDTO_TRACE"] = "1"
    try:
        tc = Context(0)
    finally:
        del os.environ["PGDTO_TRACE"]
    launch(tc)
    torch.cuda.synchronize()
    recs = tc.trace_passes()
    tc.close()
    by = {}
    for rec in recs:
        by.setdefault(rec["phase"], []).append(rec)
    phases = {k: {"passes": len(v), "loop_us": sum(q["loop_us"] for q in v) / len(v),
                  "pass_us": sum(q["pass_us"] for q in v) / len(v)} for k, v in by.items()}
    out = {"workload": f"project, {m} dense coupled rows (planted multiplier on every fourth row, seed "
                       f"{WIDE_SEED}), 256x128x128 (n={n}), float32 streams",
           "kernel": f"k_solve_wide<{(m + 15) // 16}>", "grid_tiles": grid, "launches": K,
           "kernel_ms": {"mean": mean_ms, "p50": ms[K // 2], "max": ms[-1]},
           "outcome": r["outcome"], "path": r["path"], "passes": r["passes"], "newton": r["iters_newton"],
           "newton_passes": r["iters_ls"], "stage1_passes": r["iters_search"], "check_passes": checks,
           "candidates": ncand, "lambda_rel_err_vs_planted": lam_err, "error": r["error"],
           "roofline": {"bound": "mfma", "achieved": f32 / (mean_ms * 1e-3) / 1e12, "peak": MFMA_F32_PEAK / 1e12,
                        "unit": "TFLOP/s", "frac": f32 / (mean_ms * 1e-3) / MFMA_F32_PEAK,
                        "flops_per_launch": f32, "dtype": "f32 (Jacobian sums A D A^T)",
                        "note": "whole launch: the zero, Stage-1, check and final passes add time, not f32 flops"},
           "check_f64": {"flops_per_launch": f64, "achieved": f64 / (mean_ms * 1e-3) / 1e12,
                         "peak": MFMA_F64_PEAK / 1e12, "unit": "TFLOP/s"},
           "hbm": {"bytes_per_launch": nbytes, "achieved": nbytes / (mean_ms * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
                   "unit": "GB/s", "frac": nbytes / (mean_ms * 1e-3) / HBM_PEAK, "traffic": None},
           "passes_traced": phases, "kernel_sha": kernel_sha(WIDE_SRC)}
    tr = WIDE_MEASURED_TRAFFIC.get(m)
    if tr and tr["kernel_sha"] == out["kernel_sha"] and p.meta.get("seed") == WIDE_SEED:
        out["hbm"]["traffic"] = tr["bytes_per_launch"]
        out["hbm"]["traffic_read"] = tr["read"]
        out["hbm"]["traffic_written"] = tr["written"]
    if "newton" in phases:
        t = phases["newton"]["loop_us"] * 1e-6
        tp = phases["newton"]["pass_us"] * 1e-6
        fl = n * m * (m + 1)
        by_pass = n * ESZ * (m + 1)
        out["newton_pass"] = {"flops": fl, "bytes": by_pass, "loop_us": t * 1e6, "pass_us": tp * 1e6,
                              "mfma_frac_loop": fl / t / MFMA_F32_PEAK, "mfma_frac_pass": fl / tp / MFMA_F32_PEAK,
                              "hbm_frac_loop": by_pass / t / HBM_PEAK, "hbm_frac_pass": by_pass / tp / HBM_PEAK}
    return out


# ---------------------------------------------------------------- one instance
def single_bench(ctx, insts, is_pgd, n, rows, args):
    """One-instance launches (pgdto_pgd_step_async / pgdto_project_async),
    four instances in turn: warm (back to back) and cold (each after a 1 GB
    streaming copy that evicts the Infinity Cache and L2)."""
    import torch
    from paper_2511_13905_amd import inputs as I
    from paper_2511_13905_amd.api import result_from_bytes, result_nbytes
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    R = min(4, len(insts))
    nres = result_nbytes(pgd=is_pgd)
    bufs = [torch.zeros(nres, dtype=torch.uint8, device=dev) for _ in range(R)]

    def launch(i):
        it = insts[i % R]
        if is_pgd:
            ctx.pgd_step_async("single", it["A"], it["rho"], it["rho_prev"], it["grad"], it["grad_prev"], it["d"],
                               it["g"], it["G"], it["t"], I.LO, I.HI, bufs[i % R], x=it["x"], work=it["work"],
                               params={"compact": 1 if args.compact else 0})
        else:
            p = it["p"]
            ctx.project_async(p.kind, it["y"], it["A"], p.b, p.lo, p.hi, bufs[i % R], C=p.C, offsets=p.offsets,
                              x=it["x"], params={"compact": 1 if args.compact else 0})

    for i in range(4):
        launch(i)
    torch.cuda.synchronize()
    K = max(8, args.steps)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for i in range(K):
        evs[i][0].record(stream)
        launch(i)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    warm = sorted(a.elapsed_time(b) for a, b in evs)
    res = [result_from_bytes(b, pgd=is_pgd) for b in bufs]
    passes = [(r["proj"] if is_pgd else r)["passes"] for r in res]
    # cold: a 1 GB copy before each launch
    flush_src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    flush_dst = torch.empty_like(flush_src)
    cold = []
    for i in range(8):
        flush_dst.copy_(flush_src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        launch(i)
        e1.record(stream)
        torch.cuda.synchronize()
        cold.append(e0.elapsed_time(e1))
    cold.sort()
    del flush_src, flush_dst
    mean_ms = sum(warm) / len(warm)
    mean_passes = sum(passes) / len(passes)
    pr = [(r["proj"] if is_pgd else r) for r in res]
    alg = sum(pgd_bytes(n, r) if is_pgd else proj_bytes(n, rows, r) for r in pr) / len(pr)
    # HBM bytes the counters measured per launch (register-resident passes read nothing)
    mt = SINGLE_MEASURED_TRAFFIC.get(args.workload)
    tr_gbps = mt["bytes_per_launch"] / (mean_ms * 1e-3) / 1e9 if mt and mt["kernel_sha"] == kernel_sha() else None
    return {"launch": "pgdto_pgd_step_async" if is_pgd else "pgdto_project_async",
            "instances_rotated": R, "passes_mean": mean_passes, "grid_tiles": list(ctx.last_launch()),
            "warm_ms": {"mean": mean_ms, "p50": warm[len(warm) // 2], "p99": warm[-1]},
            "cold_ms": {"p50": cold[len(cold) // 2], "max": cold[-1],
                        "flush": "1 GB device copy before each launch"},
            "elements_per_s": n / (mean_ms * 1e-3),
            "algorithmic_GBps": alg / (mean_ms * 1e-3) / 1e9,
            "algorithmic_frac": alg / (mean_ms * 1e-3) / HBM_PEAK,
            "traffic_GBps": tr_gbps,
            "traffic_frac": None if tr_gbps is None else tr_gbps * 1e9 / HBM_PEAK,
            "note": "one instance is latency-bound: its first tiles stay in registers across passes and "
                    "the per-pass grid synchronisation dominates; algorithmic bytes count those passes as "
                    "reads, traffic is what the HBM counters measured"}


# ---------------------------------------------------------------- serving
def _pctl(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))]


def _run_stream(ctx, structs, params, max_slots, arrivals, wg_per_slot=0):
    """Submit the pre-built requests at the given arrival offsets (s) through
    one pgdto_batch; returns per-request (submit, admit, done) ns and statuses."""
    import ctypes as C
    from paper_2511_13905_amd import _native as N
    from paper_2511_13905_amd.api import Batch
    L = N.lib()
    B = Batch(ctx, max_slots=max_slots, wg_per_slot=wg_per_slot)
    tickets = []
    t0 = time.perf_counter()
    for st, at in zip(structs, arrivals):
        while time.perf_counter() - t0 < at:
            pass
        t = C.c_uint64()
        rc = L.pgdto_batch_submit(B.h, C.byref(st), C.byref(params), C.byref(t))
        if rc != 0:
            raise RuntimeError(f"submit failed: {rc}")
        tickets.append(t.value)
    times, status = [], []
    r = N.Result()
    tm = (C.c_int64 * 3)()
    for t in tickets:
        rc = L.pgdto_batch_poll_timed(B.h, t, C.byref(r), tm, 1)
        status.append(rc)
        times.append((tm[0], tm[1], tm[2]))
    shape = B.shape()
    B.close()
    return times, status, shape


def _stream_stats(times, status, ns):
    lat = [(d - s) / 1e6 for s, a, d in times]
    svc = [(d - a) / 1e6 for s, a, d in times]
    wall = (max(d for _, _, d in times) - min(s for s, _, _ in times)) / 1e9
    return {"requests": len(times), "errors": sum(1 for x in status if x != 0), "wall_s": wall,
            "requests_per_s": len(times) / wall, "elements_per_s": sum(ns) / wall,
            "latency_ms": {"p50": _pctl(lat, 0.5), "p99": _pctl(lat, 0.99), "max": max(lat)},
            "service_ms": {"p50": _pctl(svc, 0.5), "p99": _pctl(svc, 0.99)}}


def serve_bench(ctx, args):
    """Served stream: requests of n log-uniform in [4096, 2097152], kind uniform
    over 1 row / 4 independent blocks / 5 coupled rows, float32.  The first
    `pool` requests of the stream are generated; request i uses instance
    i mod pool (inputs shared, outputs distinct).  Measures the plain
    one-at-a-time path and the persistent multi-slot executor, saturated (all
    requests at t = 0) and with Poisson arrivals at 0.7x and 2x the plain
    path's saturated rate."""
    import numpy as np
    import torch
    from paper_2511_13905_amd import inputs as I
    from paper_2511_13905_amd.api import make_params, problem_struct, aligned_rows, _Keep
    stream = I.serve_stream(0, args.serve_requests)
    P = min(args.serve_pool, len(stream))
    pool = [I.serve_request(s, n, kind) for (s, kind, n) in stream[:P]]
    dev = []
    for p in pool:
        A = torch.from_numpy(np.ascontiguousarray(p.A)).to("cuda:0")
        if p.kind != "independent":
            A = aligned_rows(A)
        dev.append((torch.from_numpy(np.ascontiguousarray(p.y)).to("cuda:0"), A))
    keep = _Keep()
    structs, ns, xs = [], [], []
    for i in range(len(stream)):
        p = pool[i % P]
        y, A = dev[i % P]
        x = torch.empty(p.n, dtype=torch.float32, device="cuda:0")
        st, _, _ = problem_struct(p.kind, y, A, p.b, p.lo, p.hi, p.C, p.offsets, x, None, keep, copy_ok=False)
        structs.append(st)
        ns.append(p.n)
        xs.append(x)
    torch.cuda.synchronize()
    params = make_params()
    rng = np.random.default_rng(1)
    out = {"workload": f"{len(stream)} requests, n log-uniform [4096, 2097152] (mean {np.mean(ns):.0f}), "
                       f"kinds 1 row / 4 independent / 5 coupled, float32, {P} distinct instances",
           "bytes_in_requests": int(sum(4 * p.n * ((1 if p.kind == 'independent' else p.m) + 2) for p in pool))}
    zero = [0.0] * len(stream)
    t, s, _ = _run_stream(ctx, structs, params, 1, zero)
    out["plain_saturated"] = _stream_stats(t, s, ns)
    t, s, shape = _run_stream(ctx, structs, params, 0, zero)
    out["server_saturated"] = _stream_stats(t, s, ns)
    out["server_shape"] = {"slots": shape[0], "wg_per_slot": shape[1]}
    # the throughput-oriented shape: the executor autotuner on the served mix
    from paper_2511_13905_amd.api import TUNE_SLOTS, batch_autotune
    (ts, tw), cand = batch_autotune(
        ctx, [(p.kind, y, A, p.b, p.lo, p.hi, p.C, p.offsets, x) for p, (y, A), x in zip(pool, dev, xs[:P])],
        count=512, params=params)
    t, s, shape = _run_stream(ctx, structs, params, ts, zero, tw)
    out["server_saturated_tuned"] = _stream_stats(t, s, ns)
    out["server_saturated_tuned"]["shape"] = {"slots": shape[0], "wg_per_slot": shape[1]}
    out["server_saturated_tuned"]["autotune_wall_ms"] = dict(zip([str(v) for v in TUNE_SLOTS], cand))
    r_plain = out["plain_saturated"]["requests_per_s"]
    for name, f in (("0.7x", 0.7), ("2x", 2.0)):
        rate = f * r_plain
        arr = np.cumsum(rng.exponential(1.0 / rate, len(stream))).tolist()
        res = {"rate_per_s": rate}
        t, s, _ = _run_stream(ctx, structs, params, 1, arr)
        res["plain"] = _stream_stats(t, s, ns)
        t, s, _ = _run_stream(ctx, structs, params, 0, arr)
        res["server"] = _stream_stats(t, s, ns)
        out[f"poisson_{name}_plain_rate"] = res
    del xs
    return out


def server_batch_bench(ctx, insts, args):
    """The persistent executor (server route) on 64 projections of the
    256x128x128 single-row problem, all submitted at once: 4 device copies of
    each of the 16 distinct instances, so no two requests read the same
    memory; algorithmic bytes of every pass over the wall time."""
    import torch
    from paper_2511_13905_amd.api import make_params, problem_struct, _Keep
    keep = _Keep()
    structs, hold, ns, per = [], [], [], []
    params = make_params()
    passes = {}
    for i in range(64):
        it = insts[i % len(insts)]
        p = it["p"]
        y, A = it["y"].clone(), it["A"].clone()
        x = torch.empty_like(y)
        hold.append((y, A, x))
        st, _, _ = problem_struct(p.kind, y, A, p.b, p.lo, p.hi, p.C, None, x, None, keep, copy_ok=False)
        structs.append(st)
        ns.append(p.n)
        if i < len(insts):
            _, r = ctx.project(p.kind, it["y"], it["A"], p.b, p.lo, p.hi, p.C)
            passes[i] = r
        per.append(proj_bytes(p.n, 1, passes[i % len(insts)]))
    torch.cuda.synchronize()
    alg = sum(per)
    out = {"workload": "64 x project, 256x128x128 single row (n=4194304), float32, 16 distinct instances in "
                       "4 device copies each, all submitted at once"}
    for name, slots in (("shape_8x32", 8), ("shape_32x8", 32)):
        _run_stream(ctx, structs[:16], params, slots, [0.0] * 16)
        best = None
        for _ in range(2):
            times, status, shape = _run_stream(ctx, structs, params, slots, [0.0] * 64)
            wall = (max(d for _, _, d in times) - min(s for s, _, _ in times)) / 1e9
            if best is None or wall < best[0]:
                best = (wall, status, shape)
        wall, status, shape = best
        out[name] = {"errors": sum(1 for x in status if x != 0), "wall_s": wall, "projections_per_s": 64 / wall,
                     "elements_per_s": sum(ns) / wall, "algorithmic_GBps": alg / wall / 1e9,
                     "hbm_frac": alg / wall / HBM_PEAK, "server_shape": {"slots": shape[0], "wg_per_slot": shape[1]}}
    del hold
    return out


# ---------------------------------------------------------------- CPU oracle
_POOL_STATES = None


def _oracle_one(wl, st):
    import numpy as np
    import oracle
    from paper_2511_13905_amd import inputs as I
    if wl == "pgd_compliance":
        return oracle.pgd_step("single", st.rho, st.rho_prev, st.grad, st.grad_prev, st.d_prev, st.problem.A, st.g,
                               st.G, st.t, I.LO, I.HI, stream_dtype=np.float32)
    return oracle.project(st.kind, st.y, st.A, st.b, st.lo, st.hi, st.C, st.offsets)


def _pool_task(args):
    wl, i = args
    t = time.perf_counter()
    _oracle_one(wl, _POOL_STATES[i])
    return time.perf_counter() - t


def cpu_baseline(wl, states, budget_s, workers, cpu):
    """The CPU oracle, as it stands, on bounded samples of the same workload:
    one thread on as many instances as fit the budget, then a process pool of
    `workers` processes over every instance of the batch."""
    global _POOL_STATES
    n_el = lambda st: st.rho.size if wl == "pgd_compliance" else st.n
    refs = []
    t0 = time.perf_counter()
    while len(refs) < len(states) and (not refs or time.perf_counter() - t0 < budget_s):
        refs.append(_oracle_one(wl, states[len(refs)]))
    el1 = time.perf_counter() - t0
    single = {"value": sum(n_el(states[i]) for i in range(len(refs))) / el1, "unit": "elements/s", "cores": 1,
              "sample": f"{len(refs)} full-size instance(s), one thread, {el1:.1f} s"}
    out = {"value": single["value"], "unit": "elements/s", "cores": 1, "kind": "oracle",
           "sample": single["sample"] + " (numpy float64)", "cpu": cpu, "single_thread": single}
    if workers > 1 and len(states) > 1:
        import multiprocessing as mp
        _POOL_STATES = states
        P = min(workers, len(states))
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(P) as pool:
            secs = pool.map(_pool_task, [(wl, i) for i in range(len(states))])
        elp = time.perf_counter() - t0
        _POOL_STATES = None
        tot = sum(n_el(st) for st in states)
        out.update({"value": tot / elp, "cores": P,
                    "sample": f"all {len(states)} instances of the launch, {P} worker processes "
                              f"(numpy float64, one thread each), {elp:.1f} s wall, "
                              f"{sum(secs) / len(secs):.2f} s per instance"})
        out["pool"] = {"value": tot / elp, "unit": "elements/s", "cores": P, "wall_s": elp}
    return out, refs


def oracle_error(ctx, wl, states, insts, refs):
    """Error of the GPU result against the float64 oracle on the instances the
    CPU baseline solved on one thread (each solved once more on the GPU from its
    original inputs, outside the timed region): x relative to |x|, the
    constraint residual relative to |b_j| (to the row scale sigma_j = sum |a_j|
    max(|lo|, |hi|) where b_j is zero up to rounding, as in the parity tests),
    the multiplier relative to itself, free-set disagreements outside the
    1e-6 band around the bounds, and whether the stated bound covered the
    multiplier error."""
    import numpy as np
    import torch
    from paper_2511_13905_amd import inputs as I
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    xe, re_, le, mism, covered = 0.0, 0.0, 0.0, 0, True
    for st, it, ref in zip(states, insts, refs):
        mask = None
        if wl == "pgd_compliance":
            nn = st.rho.size
            mask = torch.zeros((nn + 31) // 32, dtype=torch.int32, device="cuda:0")
            x, out = ctx.pgd_step("single", it["A"], it["rho"], it["rho_prev"], it["grad"], it["grad_prev"],
                                  dev(st.d_prev), st.g, st.G, st.t, I.LO, I.HI)
            r, o, b = out["proj"], ref["proj"], ref["b"]
            rows = np.atleast_2d(st.problem.A).astype(np.float64)
            free = None
        else:
            p = st
            mask = torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0")
            x, r = ctx.project(p.kind, it["y"], it["A"], p.b, p.lo, p.hi, p.C, offsets=p.offsets, free_mask=mask)
            o, b = ref, p.b
            rows = p.dense_rows()
            torch.cuda.synchronize()
            bits = np.unpackbits(mask.cpu().numpy().view(np.uint8), bitorder="little")[:p.n].astype(bool)
            free = bits
        sig = np.abs(rows).sum(axis=1) * max(abs(I.LO), abs(I.HI))
        torch.cuda.synchronize()
        xv = x.cpu().numpy().astype(np.float64)
        xe = max(xe, float(np.max(np.abs(xv - o.x) / np.maximum(np.abs(o.x), 1e-300))))
        z = o.z
        far = np.minimum(np.abs(z - I.LO), np.abs(z - I.HI)) > 1e-6
        if free is None:
            free = (xv != np.float32(I.LO)) & (xv != np.float32(I.HI))
        mism += int(np.count_nonzero((free != ((z >= I.LO) & (z <= I.HI))) & far))
        for j in range(len(o.resid)):
            bj = abs(float(b[j]))
            scale = bj if bj > 1e-9 * sig[j] else sig[j]
            re_ = max(re_, float(abs(r["resid"][j] - o.resid[j]) / max(scale, 1e-300)))
            err = abs(r["lam"][j] - o.lam[j])
            covered = covered and bool(err <= r["lambda_err"][j])
            if o.lam[j] != 0.0:
                le = max(le, float(err / abs(o.lam[j])))
    return {"instances": len(refs), "x_rel_max": xe, "resid_rel_max": re_, "lam_rel_max": le,
            "free_mismatch_outside_band": mism, "stated_lambda_bound_covers_error": covered,
            "tolerance": {"x_rel": 1e-5, "resid_rel": 1e-6, "free_band": 1e-6}}


if __name__ == "__main__":
    main()
