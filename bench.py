"""Throughput of the fused stencil sweep on one MI355X, beside the plain sweep
and the FP64 CPU oracle.

Workload: 3D 7-point star (r = 1), 512^3 grid, FP32 storage and arithmetic,
zero halo, T = 64 steps, seeded normalised weights and a U[-1, 1) field.
One timed step = one whole sweep (stencil_run, T = 64, with the library's
measured default fused depth k, tile variant and z-chunk, or the autotuned
ones with --autotune) followed by the FP64 checksum reduction of u_T, inputs
resident in HBM.  The plain one-step-per-launch sweep (k = 1) is
timed the same way for the speedup.  The line also carries the roofline of
the dominant kernel (HIP-event launch timing; counted HBM traffic while the
kernel sources match the recorded profile), the same grid in FP64, the
other workloads at their defaults (other_configs: 2D 8192^2 periodic, the
batched 256-grid workload, the 256^3 adjoint, 1D FP64) and the FP64 CPU
oracle timed on a bounded sample (cpu_baseline).

Prints one JSON line.  Usage:
  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                  [--no-configs] [--no-f64] [--stencil 3d7p|3d13p|3d27p]
                  [--method fused|tessellate] [--inplace]
  python bench.py --workload batched|table1|configs|adjoint
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GStencil/s + % HBM roofline, fused vs plain sweep, 3D7P 512^3 FP32"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_stream3d_7p_512.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("stream_kernel.hpp", "device_common.hpp", "variants.hpp", "launch.hpp"):
        with open(os.path.join(ROOT, "paper_2103_08825_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def time_sweep(plan, x, y, T, steps, warmup, with_reduce=True):
    """Returns (ms per step, ms of the sweeps alone per step) with HIP events on
    torch's current stream, the stream the library launches on."""
    import torch
    from paper_2103_08825_amd import reduce
    for _ in range(warmup):
        plan.run(x, T, out=y)
        if with_reduce:
            reduce(y)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b, c in ev:
        a.record()
        plan.run(x, T, out=y)
        b.record()
        if with_reduce:
            reduce(y)
        c.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    total = sum(a.elapsed_time(c) for a, b, c in ev) / steps
    sweep = sum(a.elapsed_time(b) for a, b, c in ev) / steps
    return total, sweep, wall


def cpu_model() -> str:
    """The host CPU's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(u0_f64, coeffs, r, kind, bc, T, budget_s=12.0, budget_1t_s=6.0):
    """The oracle as it stands on the host cores (all of them, then one thread),
    each over a bounded number of steps of the same grid."""
    import oracle
    threads = oracle.max_threads()
    _, s1 = oracle.run(u0_f64, coeffs, 1, r=r, kind=kind, bc=bc, return_seconds=True)
    steps = max(1, min(T, int(budget_s / max(s1, 1e-3))))
    _, secs = oracle.run(u0_f64, coeffs, steps, r=r, kind=kind, bc=bc, return_seconds=True)
    pts = u0_f64.size * steps
    grid = "x".join(str(s) for s in u0_f64.shape)
    # one thread: a shorter run of the same grid, scaled per point-step
    _, s1t = oracle.run(u0_f64, coeffs, 1, r=r, kind=kind, bc=bc, nthreads=1, return_seconds=True)
    steps1 = max(1, min(T, int(budget_1t_s / max(s1t, 1e-3))))
    if steps1 > 1:
        _, s1t = oracle.run(u0_f64, coeffs, steps1, r=r, kind=kind, bc=bc, nthreads=1, return_seconds=True)
    return {"value": pts / secs / 1e9, "unit": "GStencil/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "full %s grid, %d of the %d steps (FP64 loop nest, OpenMP over the grid)"
                      % (grid, steps, T),
            "seconds": secs,
            "single_thread": {"value": u0_f64.size * steps1 / s1t / 1e9, "unit": "GStencil/s",
                              "cores": 1, "seconds": s1t,
                              "sample": "full %s grid, %d of the %d steps on one thread "
                                        "(a shorter T, rate per point-step)" % (grid, steps1, T)}}


def copy_bandwidth(x, y, reps=10):
    """Read + write bandwidth of a device-to-device copy of the field (GB/s): the
    practical ceiling of an HBM-bound kernel on this part."""
    import torch
    for _ in range(2):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * x.numel() * x.element_size() * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def launch_probe(plan, buf, k, n):
    """Mean duration of one fused launch (k steps, one pass) over n launches,
    each bracketed by HIP events on torch's current stream; the launches
    ping-pong between `buf` and a second field."""
    import torch
    other = torch.empty_like(buf)
    bufs = [buf, other]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    plan.run(bufs[0], k, out=bufs[1])
    torch.cuda.synchronize()
    for i in range(n):
        ev[i][0].record()
        plan.run(bufs[i % 2], k, out=bufs[(i + 1) % 2])
        ev[i][1].record()
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in ev) / n
    del other
    return ms


def batched_rate(steps, compare):
    """256 independent 2D FP32 grids (sides log-uniform in [64, 2048], 5-point star
    or 9-point box, T uniform in [10, 200], zero halo): one graph-captured
    persistent launch whose item depth (per stencil) and rows per item the
    library's item tuner chose by timing this batch's own replays (the untuned
    defaults are timed beside it), optionally against 256
    separate plain sweeps (k = 1, one launch per step) and 256 separate fused
    sweeps.  Returns a record; hbm_frac_alg is one read and one write of every
    grid per pass over the replay time, against 8 TB/s."""
    import torch
    from paper_2103_08825_amd import Plan, workloads as W
    from paper_2103_08825_amd.batched import Batch
    grids = W.batched_grids(seed=0)
    xs = [torch.from_numpy(W.batched_field(0, g)).float().cuda() for g in grids]
    ys = [torch.empty_like(x) for x in xs]
    Ts = [g.T for g in grids]
    work = float(sum(x.numel() * T for x, T in zip(xs, Ts)))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    fused = [Plan(g.shape, 1, g.kind, g.coeffs, W.BC_ZERO, "f32") for g in grids]
    t0 = time.time()
    default = Batch(fused, xs, ys, Ts)
    log("batch build %.1fs, items/workgroups %s" % (time.time() - t0, default.info()))
    ms_default = timed(default.launch, max(3, steps))
    default.status()
    default_choice = default.choice()
    default.close()
    t0 = time.time()
    batch = Batch(fused, xs, ys, Ts, tune_items=True)
    tune_s = time.time() - t0
    depths, rows = batch.choice()
    log("item tuner %.2fs: depths (5P, 9P) %s, rows %d" % (tune_s, depths[:2], rows))
    ms_batch = timed(batch.launch, max(3, steps))
    batch.status()
    # algorithmic bytes: every pass of a grid reads and writes it once (order-1
    # grids: depths[0] steps per pass for the 5-point star, depths[1] for the box)
    alg = float(sum(2 * 4 * x.numel() * (-(-T // depths[g.kind])) for x, T, g in zip(xs, Ts, grids)))
    rec = {"value": work / (ms_batch * 1e-3) / 1e9, "unit": "GStencil/s", "ms": ms_batch,
           "hbm_frac_alg": alg / (ms_batch * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "points": int(sum(x.numel() for x in xs)), "point_steps": int(work),
           "items": batch.info()[0], "workgroups": batch.info()[1],
           "tuned": {"depth_5p": depths[0], "depth_9p": depths[1], "rows": rows, "tune_s": tune_s},
           "untuned": {"ms": ms_default, "value": work / (ms_default * 1e-3) / 1e9,
                       "depth_5p": default_choice[0][0], "depth_9p": default_choice[0][1],
                       "rows": default_choice[1]}}
    log("batched: %.3f ms per replay, %.1f GStencil/s (untuned %.3f ms, %.1f)"
        % (ms_batch, rec["value"], ms_default, rec["untuned"]["value"]))
    if compare:
        ms_fused = timed(lambda: [p.run(x, T, out=y) for p, x, y, T in zip(fused, xs, ys, Ts)], 2)
        plain = [Plan(g.shape, 1, g.kind, g.coeffs, W.BC_ZERO, "f32", method="plain") for g in grids]
        ms_plain = timed(lambda: [p.run(x, T, out=y) for p, x, y, T in zip(plain, xs, ys, Ts)], 2)
        rec["separate_plain"] = {"ms": ms_plain, "value": work / (ms_plain * 1e-3) / 1e9, "launches": int(sum(Ts))}
        rec["separate_fused"] = {"ms": ms_fused, "value": work / (ms_fused * 1e-3) / 1e9}
        rec["speedup_vs_plain"] = ms_plain / ms_batch
        rec["speedup_vs_separate_fused"] = ms_fused / ms_batch
        for p in plain:
            p.close()
    batch.close()
    for p in fused:
        p.close()
    return rec


def bench_batched(a):
    """The batched 256-grid workload as one JSON line."""
    r = batched_rate(a.steps, not a.no_compare)
    rec = {"metric": "GStencil/s, batched uneven 2D workload", "unit": "GStencil/s",
           "value": r["value"], "ms_per_step": r["ms"], "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic", "vs_baseline": None,
           "config": {"workload": "256 2D grids, sides log-uniform [64,2048], 5P star or 9P box, "
                                  "T in [10,200], zero halo", "points": r["points"],
                      "point_steps": r["point_steps"], "items": r["items"], "workgroups": r["workgroups"]},
           "batched": r}
    print(json.dumps(rec), flush=True)
    return 0


def other_configs():
    """The other workloads of the hot path at the library's defaults, for the
    headline line: 2D 5P/9P 8192^2 FP32 periodic (T=100), the batched 256-grid
    workload, the adjoint of the 3D 7P 256^3 FP32 periodic sweep (T=100,
    checkpoints every 10) and the 1D 3P 262,144-point FP64 sweep (T=200)."""
    import torch
    from paper_2103_08825_amd import Plan, workloads as W
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}

    def sweep(case, dt):
        tdt = {"f64": torch.float64, "f32": torch.float32}[dt]
        x = torch.from_numpy(case.u0).to(tdt).cuda()
        y = torch.empty_like(x)
        plan = Plan(case.shape, case.r, case.kind, case.coeffs, case.bc, dt)
        plan.run(x, case.T, out=y)
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(3):
            e0.record()
            plan.run(x, case.T, out=y)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        info = plan.info()
        k = info["fused_k"]
        pts = float(np.prod(case.shape))
        plan.close()
        return {"value": pts * case.T / best / 1e6, "unit": "GStencil/s", "ms": best, "k": k,
                "variant": info["variant"], "hbm_frac_alg": 2.0 * x.element_size() * pts * (-(-case.T // k))
                / (best * 1e-3) / 1e9 / HBM_PEAK_GBS}

    for kind, nm in ((W.STAR, "2d5p_8192_f32_periodic"), (W.BOX, "2d9p_8192_f32_periodic")):
        out[nm] = sweep(W.case_2d(kind), "f32")
        log("%s: %.1f GStencil/s (k=%d)" % (nm, out[nm]["value"], out[nm]["k"]))
    out["1d3p_262144_f64"] = sweep(W.case_1d3p(), "f64")
    out["batched_256_2d_f32"] = batched_rate(3, False)
    out["adjoint_3d7p_256_f32_periodic"] = adjoint_rates(2)
    return out


def bench_table1(a):
    """The six problems of the paper's evaluation table in FP64 (zero halo, T=1000):
    the library's default fused sweep and the plain one-step sweep of each, as one
    JSON line; `value` is total point-steps over total fused time."""
    import torch
    from paper_2103_08825_amd import Plan, workloads as W
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    rows, tot_work, tot_ms = {}, 0.0, 0.0
    for name, shape, r, kind in W.TABLE1:
        case = W.case_table1(name)
        x = torch.from_numpy(case.u0).cuda()
        y = torch.empty_like(x)
        work = float(np.prod(shape)) * case.T
        fused = Plan(shape, r, kind, case.coeffs, case.bc, "f64")
        ms_f = timed(lambda: fused.run(x, case.T, out=y), max(1, a.steps // 2))
        plain = Plan(shape, r, kind, case.coeffs, case.bc, "f64", method="plain")
        ms_p = timed(lambda: plain.run(x, case.T, out=y), 1)
        info = fused.info()
        rows[name] = {"shape": list(shape), "npts": case.npts, "T": case.T,
                      "fused": {"GStencil/s": work / ms_f / 1e6, "ms": ms_f, "k": info["fused_k"],
                                "method": info["method"], "variant": info["variant"],
                                "tile": list(info["tile"])},
                      "plain": {"GStencil/s": work / ms_p / 1e6, "ms": ms_p}}
        log("%-9s %-16s fused k=%d %8.1f GStencil/s (%.2f ms)   plain %7.1f GStencil/s (%.2f ms)"
            % (name, "x".join(map(str, shape)), info["fused_k"], work / ms_f / 1e6, ms_f, work / ms_p / 1e6, ms_p))
        tot_work += work
        tot_ms += ms_f
        fused.close()
        plain.close()
        del x, y
    rec = {"metric": "GStencil/s, the paper's Table 1 problems (FP64, T=1000, zero halo)",
           "unit": "GStencil/s", "value": tot_work / tot_ms / 1e6, "ms_per_step": tot_ms, "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic", "vs_baseline": None,
           "config": {"workload": "1D3P/1D5P 10240000, 2D5P/2D9P 3000^2, 3D7P/3D27P 128^3; T=1000 each"},
           "problems": rows}
    print(json.dumps(rec), flush=True)
    return 0


def adjoint_rates(reps):
    """The adjoint of the 3D 7-point periodic FP32 sweep (256^3, T=100, checkpoints
    every 10 steps): time of the forward sweep and of stencil_adjoint."""
    import torch
    from paper_2103_08825_amd import Plan, workloads as W
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    case = W.case_adjoint()
    x = torch.from_numpy(case.u0).float().cuda()
    tgt = torch.from_numpy(case.target).float().cuda()
    plan = Plan(case.shape, 1, W.STAR, case.coeffs, W.BC_PERIODIC, "f32")
    uT = plan.run(x, case.T)
    g = (uT - tgt).contiguous()
    ms_f = timed(lambda: plan.run(x, case.T, out=uT))
    ms_a = timed(lambda: plan.adjoint(x, g, case.T, 10))
    pts = float(np.prod(case.shape))
    plan.close()
    log("adjoint 256^3 T=100: forward %.2f ms, adjoint %.2f ms" % (ms_f, ms_a))
    return {"forward_ms": ms_f, "adjoint_ms": ms_a, "T": case.T, "checkpoint_every": 10,
            "adjoint GStencil/s": pts * case.T / ms_a / 1e6,
            "forward+adjoint GStencil/s": pts * case.T / (ms_f + ms_a) / 1e6}


def bench_adjoint(a):
    """One JSON line for the adjoint workload alone."""
    r = adjoint_rates(max(2, a.steps // 2))
    rec = {"metric": "point-steps/s of the adjoint sweep (dL/du0 and dL/dc)", "unit": "GStencil/s",
           "value": r["adjoint GStencil/s"], "ms_per_step": r["adjoint_ms"], "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic", "vs_baseline": None,
           "config": {"workload": "3D 7-point star 256^3 FP32, periodic, T=100, checkpoints every 10"},
           "adjoint": r}
    print(json.dumps(rec), flush=True)
    return 0


def bench_configs(a):
    """Every workload of the hot path, fused and plain, as one JSON line: the 1D
    3-point FP64 sweep (262,144 points, T=200), the 2D 5-point and 9-point FP32
    periodic sweeps (8192^2, T=100), the 3D 7-, 13- and 27-point sweeps (512^3,
    T=64) in FP32, BF16 and FP16, and the adjoint of the 3D 7-point periodic
    sweep (256^3 FP32, T=100, checkpoints every 10).  Rates are useful
    point-steps per second; hbm_frac is the algorithmic traffic (one read and
    one write of the field per launch) over 8 TB/s."""
    import torch
    from paper_2103_08825_amd import Plan, workloads as W
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}

    def timed(fn, reps):
        # back-to-back calls between one pair of events, so the host-side work of
        # a call overlaps the previous call's kernels (steady-state throughput)
        fn()
        torch.cuda.synchronize()
        n = max(2, reps)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    def sweep(case, dt, method, reps):
        x = torch.from_numpy(case.u0).to(tdt[dt]).cuda()
        y = torch.empty_like(x)
        plan = Plan(case.shape, case.r, case.kind, case.coeffs, case.bc, dt, method=method)
        ms = timed(lambda: plan.run(x, case.T, out=y), reps)
        info = plan.info()
        k = info["fused_k"]
        launches = -(-case.T // k)
        pts = float(np.prod(case.shape))
        rec = {"GStencil/s": pts * case.T / ms / 1e6, "ms": ms, "k": k, "variant": info["variant"],
               "tile": list(info["tile"]),
               "hbm_frac": 2.0 * x.element_size() * pts * launches / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        plan.close()
        return rec

    out = {}

    def entry(name, case, dt, reps=2):
        f = sweep(case, dt, "auto", reps)
        p = sweep(case, dt, "plain", 1)
        out[name] = {"fused": f, "plain": p, "speedup": p["ms"] / f["ms"]}
        log("%-22s fused %8.1f GStencil/s (k=%d, %.2f ms, hbm %.2f)   plain %7.1f (%.2f ms, hbm %.2f)"
            % (name, f["GStencil/s"], f["k"], f["ms"], f["hbm_frac"], p["GStencil/s"], p["ms"], p["hbm_frac"]))

    entry("1d3p_262144_f64", W.case_1d3p(), "f64")
    # the same launch-bound sweep replayed from a recorded HIP graph
    case = W.case_1d3p()
    x = torch.from_numpy(case.u0).cuda()
    y = torch.empty_like(x)
    for method in ("plain", "auto"):
        plan = Plan(case.shape, 1, W.STAR, case.coeffs, W.BC_ZERO, "f64", method=method, graph=True)
        ms = timed(lambda: plan.run(x, case.T, out=y), 3)
        key = "plain" if method == "plain" else "fused"
        out["1d3p_262144_f64"][key + "_graph"] = {"GStencil/s": x.numel() * case.T / ms / 1e6, "ms": ms}
        log("1d3p graph replay (%s): %.3f ms, %.1f GStencil/s" % (key, ms, x.numel() * case.T / ms / 1e6))
        plan.close()
    del x, y
    for kind, nm in ((W.STAR, "2d5p"), (W.BOX, "2d9p")):
        entry(nm + "_8192_f32_periodic", W.case_2d(kind), "f32")
    for nm in ("3d7p", "3d13p", "3d27p"):
        case = W.case_3d(nm)
        for dt in ("f32", "bf16", "f16"):
            entry("%s_512_%s" % (nm, dt), case, dt)
        del case
    out["adjoint_3d7p_256_f32_periodic"] = adjoint_rates(max(2, a.steps // 2))
    rec = {"metric": "GStencil/s per workload (fused and plain)", "unit": "GStencil/s",
           "value": out["3d7p_512_f32"]["fused"]["GStencil/s"], "n_gpus": 1, "higher_is_better": True,
           "dtype": "mixed", "data": "synthetic", "vs_baseline": None,
           "config": {"workload": "1D3P 262144 FP64 T=200; 2D 5P/9P 8192^2 FP32 periodic T=100; "
                                  "3D 7P/13P/27P 512^3 FP32/BF16/FP16 T=64; adjoint 3D7P 256^3 FP32 T=100"},
           "workloads": out}
    print(json.dumps(rec), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--T", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 sub-record")
    ap.add_argument("--autotune", action="store_true",
                    help="time every compiled (variant, k, chunk) first instead of the "
                         "library's measured default")
    ap.add_argument("--fused-k", type=int, default=0)
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--workload", choices=["3d7p", "batched", "table1", "configs", "adjoint"], default="3d7p",
                    help="3d7p (default): the headline sweep; batched: 256 uneven 2D grids "
                         "in one graph-captured persistent launch vs separate sweeps; table1: "
                         "the paper's six evaluation problems in FP64; configs: every "
                         "workload, fused and plain, and the adjoint; adjoint: the adjoint alone")
    ap.add_argument("--stencil", choices=["3d7p", "3d13p", "3d27p"], default="3d7p",
                    help="headline sweep's stencil (default: the 3D 7-point star)")
    ap.add_argument("--method", choices=["fused", "tessellate"], default="fused",
                    help="headline sweep: the overlapped fused sweep (default) or the "
                         "tessellated one")
    ap.add_argument("--inplace", action="store_true",
                    help="headline sweep: update the field in place (no ping-pong field)")
    ap.add_argument("--no-configs", action="store_true",
                    help="headline line without the other workloads' sub-record")
    ap.add_argument("--no-compare", action="store_true",
                    help="batched: time the batch only, not the 256 separate sweeps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy the FP32 field (2 x 512 MiB moved per copy) --steps times; "
                         "used to scale the HBM byte counters")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print("bench.py measures one GPU: the sweep of one grid runs on one device; "
              "--gpus %d is not supported (multi-GPU slab decomposition is design-only)" % a.gpus,
              file=sys.stderr)
        return 2

    import torch
    from paper_2103_08825_amd import Plan, workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    n, T = a.n, a.T
    if a.copy_calibration:
        x = torch.rand((n, n, n), device="cuda", dtype=torch.float32)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.steps
        nbytes = 2 * x.numel() * 4
        print(json.dumps({"copy_bytes": nbytes, "ms": ms, "GBps": nbytes / (ms * 1e-3) / 1e9}),
              flush=True)
        return 0
    if a.workload == "batched":
        return bench_batched(a)
    if a.workload == "table1":
        return bench_table1(a)
    if a.workload == "configs":
        return bench_configs(a)
    if a.workload == "adjoint":
        return bench_adjoint(a)
    case = W.case_3d(a.stencil, seed=0, n=n, T=T)
    sname = {"3d7p": "3D 7-point star r=1", "3d13p": "3D 13-point star r=2", "3d27p": "3D 27-point box r=1"}[a.stencil]
    log("inputs: %s %s T=%d" % (case.name, case.shape, T))
    x = torch.from_numpy(case.u0).to(torch.float32).cuda()
    y = torch.empty_like(x)

    points = float(np.prod(case.shape))
    # the plain comparator first: its sweeps also bring the clocks to their
    # sustained state before the fused sweeps are timed
    plain_rec = None
    if not a.no_plain:
        plain = Plan(case.shape, case.r, case.kind, case.coeffs, case.bc, "f32", method="plain")
        if a.autotune:
            plain.autotune()
        pms, pms_sweep, _ = time_sweep(plain, x, y, T, max(2, a.steps // 2), 1)
        plain_rec = {"value": points * T / (pms * 1e-3) / 1e9, "ms_per_step": pms,
                     "kernel_ms_per_launch": pms_sweep / T,
                     "hbm_frac": (2 * 4 * points / (pms_sweep / T * 1e-3) / 1e9) / HBM_PEAK_GBS,
                     "config": plain.info()}
        log("plain: %.3f ms/step, %.1f GStencil/s" % (pms, plain_rec["value"]))
        plain.close()

    fused = Plan(case.shape, case.r, case.kind, case.coeffs, case.bc, "f32", method=a.method,
                 fused_k=a.fused_k, variant=a.variant, chunk=a.chunk, inplace=a.inplace)
    if a.autotune:
        t0 = time.time()
        fused.autotune()
        log("autotune (fused) %.1fs -> %s" % (time.time() - t0, fused.info()))
    info = fused.info()
    log("fused plan: %s" % info)
    k = info["fused_k"]
    ms, ms_sweep, wall = time_sweep(fused, x, y, T, a.steps, a.warmup)
    gst = points * T / (ms * 1e-3) / 1e9
    log("fused: %.3f ms/step (sweep %.3f ms), %.1f GStencil/s" % (ms, ms_sweep, gst))
    probe_ms = launch_probe(fused, y, k, 2 * ((T + k - 1) // k))
    log("fused k=%d launch: %.4f ms (HIP events around each of %d launches)" % (k, probe_ms, 2 * ((T + k - 1) // k)))
    copy_gbs = copy_bandwidth(x, y)
    log("device copy of the field: %.0f GB/s" % copy_gbs)

    # roofline of the dominant kernel (the fused pass): algorithmic bytes per launch
    # = one read and one write of the field, over the launch duration measured with
    # events around single launches right after the timed sweeps (the sweep time
    # shared out in proportion to the steps each launch advances agrees within a
    # few per cent: launch_ms_from_sweep)
    launch_ms = probe_ms
    alg_bytes = 2.0 * 4 * points
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        with open(PROFILE_TRAFFIC) as f:
            prof = json.load(f)
        if (a.stencil == "3d7p" and prof.get("source_hash") == kernel_source_hash() and prof.get("k") == k and
                prof.get("variant") == info["variant"] and prof.get("chunk") == info["tile"][2]):
            traffic = prof.get("bytes_per_launch")
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "stream_kernel<float,3,R=%d,%s,K=%d> variant %d%s" % (
                case.r, "box" if case.kind else "star", k, info["variant"], {"fused": "", "tessellate": ", tessellated (stages A and B per pass)"}[a.method]
                + (", in place (plus the fix-up kernel)" if a.inplace else "")),
            "launch_ms": launch_ms, "launch_ms_from_sweep": ms_sweep * k / T,
            "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs}

    # the same kernel seen from the vector ALU: useful FMAs (7 per point-step, k steps
    # per launch) against the FP32 vector peak without packed math (256 CU x 64 lanes
    # x 2 FLOP x 2.4 GHz = 78.6 TFLOP/s; the build keeps packed FP32 off)
    useful_flops = 2.0 * case.npts * k * points
    roof_alu = {"bound": "alu", "achieved": useful_flops / (launch_ms * 1e-3) / 1e12, "peak": 78.6,
                "unit": "TFLOP/s",
                "frac": useful_flops / (launch_ms * 1e-3) / 1e12 / 78.6,
                "note": "useful FMAs only; the recomputed tile halo and the chunk fill add "
                        "issued VALU work (see profiles/stream3d_7p_512_f32_sq_counters.md)"}

    # the paper's own precision (FP64) on the same grid and steps, library defaults
    f64_rec = None
    if not a.no_f64:
        x64 = torch.from_numpy(case.u0).cuda()
        y64 = torch.empty_like(x64)
        p64 = Plan(case.shape, case.r, case.kind, case.coeffs, case.bc, "f64")
        ms64, sw64, _ = time_sweep(p64, x64, y64, T, max(2, a.steps // 2), 1, with_reduce=False)
        i64 = p64.info()
        f64_rec = {"value": points * T / (ms64 * 1e-3) / 1e9, "unit": "GStencil/s", "ms_per_step": ms64,
                   "fused_k": i64["fused_k"], "variant": i64["variant"], "tile": i64["tile"],
                   "hbm_frac_alg": 2.0 * 8 * points * (-(-T // i64["fused_k"])) / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log("fp64: %.3f ms/step, %.1f GStencil/s (k=%d)" % (ms64, f64_rec["value"], i64["fused_k"]))
        p64.close()
        del x64, y64

    configs = None
    if not a.no_configs and a.method == "fused" and not a.inplace and a.stencil == "3d7p":
        # free the headline fields before the other workloads allocate theirs
        del y
        configs = other_configs()
        y = None

    cpu = None
    if not a.no_cpu_baseline:
        log("cpu baseline ...")
        c32 = case.coeffs.astype(np.float32).astype(np.float64)
        u32 = x.double().cpu().numpy()
        cpu = cpu_baseline(u32, c32, case.r, case.kind, case.bc, T)
        log("cpu: %.3f GStencil/s on %d threads, %.3f on one (%s)"
            % (cpu["value"], cpu["cores"], cpu["single_thread"]["value"], cpu["cpu_model"]))

    rec = {
        "metric": METRIC, "value": gst, "unit": "GStencil/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%s, %d^3 grid, FP32, zero halo, T=%d" % (sname, n, T),
                   "fused_k": k, "variant": info["variant"], "tile": info["tile"],
                   "points": int(points), "T": T},
        "sweep_ms_per_step": ms_sweep, "wall_ms_per_step": wall,
        "plain": plain_rec,
        "speedup_vs_plain": (plain_rec["ms_per_step"] / ms) if plain_rec else None,
        "roofline": roof, "roofline_alu": roof_alu, "cpu_baseline": cpu,
        "fp64": f64_rec,
        "other_configs": configs,
    }
    print(json.dumps(rec), flush=True)
    fused.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
