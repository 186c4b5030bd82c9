#!/usr/bin/env python
"""Throughput of the truncated-kernel FFT convolution on one MI355X.

Headline workload (default): 3D Helmholtz, k = 20, N = 256 points per side
(512^3 zero-padded complex FFTs), FP32 complex bulk with FP64-built tables,
density a seeded sum of 8 plane-wave-modulated Gaussians
(workloads.helmholtz3d_k20_n256).  A step is one vg_apply: zero padding,
forward FFT, multiplication by the kernel's 2N-box spectrum, inverse FFT and
cropping (Section 4), on a density already resident in HBM.  The plan (FP64
precompute of the kernel table) is built once beforehand and its device time
is reported separately, like the paper's T_precomp.

Prints one JSON line.
  value        grid points per second = N^3 * steps / time of the timed steps.
  roofline     the pass with the most algorithmic bytes (the fused pass P3):
               its bytes per launch over its average launch time, measured with
               HIP events on the apply stream around that pass in every 5th
               timed step, against 8 TB/s (`frac`); beside it the same launch
               time from the committed rocprofv3 kernel trace (`trace`), the
               pass's instruction-issue bound from its committed counters
               (`valu`: VALU instructions over one wave64 VALU instruction per
               CU per clock, 256 CUs at 2.4 GHz), the HBM bytes the counters
               measured (`traffic`), and every pass of the step.
  cpu_baseline the FP64 oracle's apply on the host cores, same workload.
  fp64_gpu     the FP64 GPU path (complex128 end to end) on the same density.

Order.  The GPU's clock dips for roughly the first 25 ms of heavy load after
an idle spell (the fused pass runs 290 us settled, up to 370 us inside the
dip; measured with a kernel trace), so the FP64 path is timed first and the
FP32 warmup and timed steps follow it without a pause; the other
configurations settle the clock for 40 ms before their timed calls.
  configs      the other measured configurations: 3D Laplace N=32 (FP64),
               3D Helmholtz k=20 N=128, 2D Laplace and Helmholtz k=200
               N=4096, the 64-density mixed batch, and 3D Helmholtz k=150
               N=512 potential plus gradient; each with its time, grid
               points/s, all-pass HBM fraction and rel L2 / rel max error
               against the oracle (N=512: against the FP64 GPU path).
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

HBM_PEAK_GBS = 8000.0
# one wave64 VALU instruction per CU per clock (non-packed FP32): 256 CUs x 2.4 GHz
VALU_WAVE_INSTS_PER_S = 256 * 2.4e9
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "traffic_helmholtz3d_k20_n256.json")
TRACE_FILE = os.path.join(PROFILES, "kernel_trace_helmholtz3d_k20_n256.json")
COUNTER_FILE = os.path.join(PROFILES, "counters_p3_fused_helmholtz3d_k20_n256.json")
KERNEL_SOURCES = ["fft_fast_impl.h", "fft_fast_512.hip", "butterfly.h", "common.h", "fft_pass.hip"]
KERNEL_NAMES = {"laplace": "Laplace", "helmholtz": "Helmholtz"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1604_03155_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_profile(path):
    """A committed rocprofv3 summary (JSON) and whether it was taken on the
    current kernel sources; (None, False) when missing."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, False
    return t, t.get("source_hash") == kernel_source_hash()


def rel_errors(got, ref):
    import numpy as np
    d = np.abs(got - ref)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref)), float(d.max() / np.abs(ref).max())


def settle(fn, ms=40.0):
    """Call fn() for at least `ms` of wall time (at least 3 calls), so that the
    GPU clock has left its post-idle dip."""
    import torch
    t0 = time.perf_counter()
    n = 0
    while n < 3 or 1e3 * (time.perf_counter() - t0) < ms:
        fn()
        n += 1
        if n % 4 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()


def time_calls(fn, steps, warmup, settle_ms=0.0):
    """ms per call of fn() over `steps` calls after `warmup` calls (and, with
    settle_ms, the clock settled first), by events on the current stream (the
    stream the library launches on)."""
    import torch
    if settle_ms > 0:
        settle(fn, settle_ms)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / steps


def step_bytes(vg, fn):
    """Algorithmic HBM bytes of one call of fn() (sum over its passes, from the
    library's per-pass byte model)."""
    import torch
    torch.cuda.synchronize()
    vg.profiler_enable(True)
    fn()
    torch.cuda.synchronize()
    vg.profiler_enable(False)
    return sum(p["bytes_per_launch"] * p["launches"] for p in vg.profiler_collect())


def single_config(vg, name, steps, warmup, with_gradient=False):
    """One named workload: FP32 time, pts/s, all-pass fraction, accuracy
    against the FP64 oracle (potential; and gradient when asked)."""
    import numpy as np
    import torch
    from oracle import operator as op
    from workloads import evaluate_grid, workload
    prm, src = workload(name)
    d, N, kernel, k = prm["d"], prm["N"], prm["kernel"], prm["k"]
    f = evaluate_grid(src, N)
    plan = vg.Plan(d, N, kernel, k, precision="fp32")
    x = torch.from_numpy(f).to(torch.complex64).cuda()
    out, ws = torch.empty_like(x), plan.new_workspace()
    fn = lambda: plan.apply(x, out=out, workspace=ws)  # noqa: E731
    ms = time_calls(fn, steps, warmup, settle_ms=40.0)
    nbytes = step_bytes(vg, fn)
    r = {"ms": round(ms, 4), "grid_pts_per_s": N ** d / (ms * 1e-3),
         "all_passes_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
         "plan_ms": round(plan.info["precompute_ms"], 2)}
    tp = time.perf_counter()
    o = op.Plan(d, N, kernel, k)
    fn()
    torch.cuda.synchronize()
    r["rel_l2"], r["rel_max"] = rel_errors(out.cpu().numpy().astype(np.complex128), o.apply(f))
    if with_gradient:
        _, grad = plan.gradient(x)
        torch.cuda.synchronize()
        e = [rel_errors(grad[j].cpu().numpy().astype(np.complex128), g) for j, g in enumerate(o.gradient(f))]
        r["grad_rel_l2"], r["grad_rel_max"] = max(a for a, _ in e), max(b for _, b in e)
    r["reference"] = "FP64 oracle, full grid"
    log(f"[bench] {name}: {ms:.3f} ms, rel L2 {r['rel_l2']:.2e}, rel max {r['rel_max']:.2e} "
        f"(oracle {time.perf_counter() - tp:.1f} s)")
    return r


def laplace3d_n32_fp64(vg, steps, warmup):
    import torch
    from oracle import operator as op
    from workloads import evaluate_grid, workload
    prm, src = workload("laplace3d_n32")
    N = prm["N"]
    f = evaluate_grid(src, N)
    plan = vg.Plan(3, N, "laplace", precision="fp64")
    x = torch.from_numpy(f).cuda()
    out, ws = torch.empty_like(x), plan.new_workspace()
    ms = time_calls(lambda: plan.apply(x, out=out, workspace=ws), steps, warmup, settle_ms=40.0)
    l2, mx = rel_errors(out.cpu().numpy(), op.Plan(3, N, "laplace").apply(f))
    log(f"[bench] laplace3d_n32 fp64: {ms:.4f} ms, rel L2 {l2:.2e}")
    return {"precision": "fp64", "ms": round(ms, 4), "grid_pts_per_s": N ** 3 / (ms * 1e-3), "rel_l2": l2,
            "rel_max": mx, "reference": "FP64 oracle, full grid"}


def batch_config(vg, steps, warmup, sample):
    """The 64-density mixed batch in one vg_apply_batched call (graph replay)."""
    import numpy as np
    import torch
    from oracle import operator as op
    from workloads import batch_workload, evaluate_grid
    items = batch_workload()
    plans = [vg.Plan(3, p["N"], p["kernel"], p["k"], precision="fp32") for p, _ in items]
    fs_host = [evaluate_grid(src, p["N"]) for p, src in items]
    fs = [torch.from_numpy(f).to(torch.complex64).cuda() for f in fs_host]
    outs = [torch.empty_like(f) for f in fs]
    ws = torch.empty(vg.batched_workspace_size(plans), dtype=torch.uint8, device="cuda")
    fn = lambda: vg.apply_batched(plans, fs, outs, workspace=ws)  # noqa: E731
    ms = time_calls(fn, steps, warmup, settle_ms=40.0)
    nbytes = step_bytes(vg, fn)
    pts = sum(p["N"] ** 3 for p, _ in items)
    wss = [p.new_workspace() for p in plans]
    singles = lambda: [p.apply(f, out=o, workspace=w) for p, f, o, w in zip(plans, fs, outs, wss)]  # noqa: E731
    ms_single = time_calls(singles, max(3, steps // 4), 1, settle_ms=40.0)
    fn()
    torch.cuda.synchronize()
    # oracle on a sample: the first density of every (N, kernel) class
    seen, errs = set(), []
    for i, (p, _) in enumerate(items):
        key = (p["N"], p["kernel"])
        if key in seen or len(errs) >= sample:
            continue
        seen.add(key)
        ref = op.Plan(3, p["N"], p["kernel"], p["k"]).apply(fs_host[i])
        errs.append(rel_errors(outs[i].cpu().numpy().astype(np.complex128), ref))
    r = {"densities": len(items), "grid_points": pts, "ms": round(ms, 4), "grid_pts_per_s": pts / (ms * 1e-3),
         "all_passes_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
         "single_applies_ms": round(ms_single, 4), "batched_speedup": round(ms_single / ms, 3),
         "oracle_sample": len(errs), "max_rel_l2": max(e[0] for e in errs), "max_rel_max": max(e[1] for e in errs),
         "reference": f"FP64 oracle on {len(errs)} densities (one per N and kernel)"}
    log(f"[bench] batch of {len(items)}: {ms:.3f} ms ({ms_single:.3f} ms as single applies), "
        f"max rel L2 {r['max_rel_l2']:.2e} over {len(errs)}")
    return r


def large_gradient_config(vg, steps, warmup):
    """3D Helmholtz k=150, N=512: potential plus gradient, FP32 against the FP64
    GPU path (the FP64 path is held to the oracle at 1e-12 at N <= 256)."""
    import torch
    from workloads import evaluate_grid, workload
    prm, src = workload("helmholtz3d_k150_n512")
    N, k = prm["N"], prm["k"]
    f = evaluate_grid(src, N)
    p32 = vg.Plan(3, N, "helmholtz", k, precision="fp32")
    x = torch.from_numpy(f).to(torch.complex64).cuda()
    phi, grad = torch.empty_like(x), torch.empty((3,) + x.shape, dtype=x.dtype, device="cuda")
    ws = p32.new_workspace(gradient=True)
    fn = lambda: p32.gradient(x, phi=phi, grad=grad, workspace=ws)  # noqa: E731
    ms = time_calls(fn, steps, warmup, settle_ms=40.0)
    nbytes = step_bytes(vg, fn)
    ws2 = p32.new_workspace()
    ms_apply = time_calls(lambda: p32.apply(x, out=phi, workspace=ws2), steps, warmup, settle_ms=40.0)
    fn()
    torch.cuda.synchronize()
    del fn, ws, ws2
    torch.cuda.empty_cache()
    p64 = vg.Plan(3, N, "helmholtz", k, precision="fp64")
    phi64, grad64 = p64.gradient(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()

    def err(a, b):
        diff = a.to(torch.complex128) - b
        return ((torch.linalg.vector_norm(diff) / torch.linalg.vector_norm(b)).item(),
                (diff.abs().max() / b.abs().max()).item())

    (l2, mx), (gl2, gmx) = err(phi, phi64), err(grad, grad64)
    log(f"[bench] helmholtz3d_k150_n512 phi+grad: {ms:.3f} ms (apply {ms_apply:.3f} ms), "
        f"rel L2 {l2:.2e} / {gl2:.2e}")
    return {"ms_phi_and_grad": round(ms, 4), "ms_apply": round(ms_apply, 4), "grid_pts_per_s": N ** 3 / (ms * 1e-3),
            "all_passes_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "rel_l2": l2, "rel_max": mx, "grad_rel_l2": gl2, "grad_rel_max": gmx,
            "reference": "FP64 GPU path, full grid"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="helmholtz3d_k20_n256")
    ap.add_argument("--cpu-sample", type=int, default=2,
                    help="oracle applies timed for cpu_baseline (0: skip); one full-size apply takes about "
                         "5-10 s on 16 host threads")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=10,
                    help="timed applies of the FP64 GPU path on the same density (0: skip)")
    ap.add_argument("--configs", default="all",
                    help="other configurations to measure: all, none, or a comma list of c1,c2,c3,c4,c5")
    ap.add_argument("--hbm-copy-mib", type=int, default=0,
                    help="after timing, run one streaming copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs one plan per GPU; a multi-GPU decomposition is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1604_03155_amd as vg
    from workloads import evaluate_grid, workload

    params, src = workload(args.workload)
    d, N, kernel, k = params["d"], params["N"], params["kernel"], params["k"]
    V = N ** d
    log(f"[bench] workload {args.workload}: d={d} N={N} {kernel} k={k}")
    f64 = evaluate_grid(src, N)
    x = torch.from_numpy(f64).to(torch.complex64).cuda()

    plan = vg.Plan(d, N, kernel, k, precision="fp32")
    plan_ms = plan.info["precompute_ms"]
    ws = plan.new_workspace()
    out = torch.empty_like(x)

    # the plain FP64 single-density GPU path on the same density, for the
    # FP32 speedup at the stated accuracy; timed first (see Order above)
    fp64 = None
    if args.fp64_steps > 0:
        plan64 = vg.Plan(d, N, kernel, k, precision="fp64")
        x64 = torch.from_numpy(f64).cuda()
        out64 = torch.empty_like(x64)
        ws64 = plan64.new_workspace()
        ms64 = time_calls(lambda: plan64.apply(x64, out=out64, workspace=ws64), args.fp64_steps, 1, settle_ms=40.0)
        fp64 = {"ms_per_step": round(ms64, 4), "value": V / (ms64 * 1e-3), "steps": args.fp64_steps}

    for _ in range(args.warmup):
        plan.apply(x, out=out, workspace=ws)
    torch.cuda.synchronize()
    log(f"[bench] plan {plan_ms:.1f} ms; warmup done; timing {args.steps} steps")

    # timed region: HIP events on the plan's stream around the dominant pass
    # (the one with the most algorithmic bytes) of every SAMPLE-th step and
    # nowhere else (an event record between two kernels costs several
    # microseconds of stream time)
    SAMPLE = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        sampled = i % SAMPLE == 0
        if sampled:
            vg.profiler_enable(True, dominant_only=True)
        plan.apply(x, out=out, workspace=ws)
        if sampled:
            vg.profiler_enable(False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_rec = vg.profiler_collect()
    seconds = t1 - t0
    ms_per_step = 1e3 * seconds / args.steps
    value = V * args.steps / seconds
    log(f"[bench] {ms_per_step:.3f} ms/step, {value:.3e} grid pts/s")
    if fp64 is not None:
        fp64["fp32_speedup"] = round(fp64["ms_per_step"] / ms_per_step, 3)
        log(f"[bench] FP64 GPU path {fp64['ms_per_step']:.3f} ms/step; FP32 speedup {fp64['fp32_speedup']:.2f}x")

    # per-pass breakdown: the same steps again with an event between every
    # pair of passes (outside the timed region; the extra events lengthen it)
    vg.profiler_enable(True)
    for _ in range(args.steps):
        plan.apply(x, out=out, workspace=ws)
    torch.cuda.synchronize()
    vg.profiler_enable(False)
    passes = vg.profiler_collect()
    if fp64 is not None:
        del plan64, ws64

    if args.hbm_copy_mib > 0:
        nb = args.hbm_copy_mib << 20
        src_b = torch.empty(nb, dtype=torch.uint8, device="cuda")
        dst_b = torch.empty(nb, dtype=torch.uint8, device="cuda")
        vg.hbm_copy(dst_b, src_b)
        torch.cuda.synchronize()
        del src_b, dst_b

    def rows(recs):
        out_rows = []
        for p in recs:
            avg = p["total_ms"] / max(1, p["launches"])
            gbs = p["bytes_per_launch"] / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
            out_rows.append(dict(name=p["name"], avg_ms=round(avg, 5), bytes=p["bytes_per_launch"],
                                 gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4)))
        return out_rows

    pass_rows = rows(passes)
    dom = rows(dom_rec)[0]
    total_bytes = sum(r["bytes"] for r in pass_rows)
    roofline = {
        "bound": "hbm",
        "achieved": dom["gbs"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(dom["gbs"] / HBM_PEAK_GBS, 4),
        "traffic": None,
        "kernel": dom["name"],
        "bytes_per_launch": dom["bytes"],
        "avg_launch_ms": dom["avg_ms"],
        "launches_timed": dom_rec[0]["launches"],
        "timing": f"frac uses HIP events around every {SAMPLE}th launch of the kernel in the timed region",
        # algorithmic bytes of all passes of a step over the timed step time
        "all_passes_frac": round(total_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "passes": pass_rows,
        "passes_note": "per-pass times from a second run of the same steps with an event between passes",
    }
    if args.workload == "helmholtz3d_k20_n256":
        tr, tr_cur = load_profile(TRAFFIC_FILE)
        if tr and tr_cur and dom["name"] in tr.get("passes", {}):
            roofline["traffic"] = float(tr["passes"][dom["name"]]["bytes_per_launch"])
        kt, kt_cur = load_profile(TRACE_FILE)
        if kt and dom["name"] in kt.get("passes", {}):
            avg_us = float(kt["passes"][dom["name"]]["avg_us"])
            gbs = dom["bytes"] / (avg_us * 1e-6) / 1e9
            roofline["trace"] = {"avg_ms": round(avg_us * 1e-3, 5), "achieved": round(gbs, 1),
                                 "frac": round(gbs / HBM_PEAK_GBS, 4), "source": os.path.relpath(TRACE_FILE, ROOT),
                                 "current_sources": kt_cur}
        ct, ct_cur = load_profile(COUNTER_FILE)
        if ct and "SQ_INSTS_VALU" in ct.get("per_dispatch", {}):
            insts = float(ct["per_dispatch"]["SQ_INSTS_VALU"])
            min_ms = 1e3 * insts / VALU_WAVE_INSTS_PER_S
            roofline["valu"] = {
                "bound": "alu", "insts_per_launch": insts,
                "peak": "one wave64 VALU instruction per CU per clock, 256 CUs x 2.4 GHz (non-packed FP32)",
                "min_ms": round(min_ms, 5), "frac": round(min_ms / dom["avg_ms"], 4),
                "source": os.path.relpath(COUNTER_FILE, ROOT), "current_sources": ct_cur}

    kname = KERNEL_NAMES.get(kernel, kernel.capitalize())
    result = {
        "metric": f"grid pts/s, {d}D {kname} N={N}^{d} at rel L2<=1e-5 vs FP64; % HBM peak",
        "value": value,
        "unit": "grid pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "d": d, "N": N, "kernel": kernel, "k": k,
                   "padded_fft": f"{2 * N}^{d} C2C", "precision": "fp32 bulk, fp64-built tables",
                   "parallelism": "single GPU"},
        "plan_ms": round(plan_ms, 3),
        "roofline": roofline,
    }
    if fp64 is not None:
        result["fp64_gpu"] = fp64

    if not args.no_parity or args.cpu_sample > 0:
        from oracle import fft as offt
        from oracle import operator as op
        tp = time.perf_counter()
        oplan = op.Plan(d, N, kernel, k)
        log(f"[bench] oracle plan {time.perf_counter() - tp:.1f} s")
        ref = None
        if not args.no_parity:
            ref = oplan.apply(f64)
            result["rel_l2"], result["rel_max"] = rel_errors(out.cpu().numpy().astype(np.complex128), ref)
            log(f"[bench] rel L2 vs FP64 oracle {result['rel_l2']:.2e}, rel max {result['rel_max']:.2e}")
            if fp64 is not None:
                fp64["rel_l2"], fp64["rel_max"] = rel_errors(out64.cpu().numpy(), ref)
                log(f"[bench] FP64 GPU path rel L2 vs oracle {fp64['rel_l2']:.2e}")
        if args.cpu_sample > 0:
            threads = offt.threads()
            tc = time.perf_counter()
            for _ in range(args.cpu_sample):
                oplan.apply(f64)
            cpu_s = (time.perf_counter() - tc) / args.cpu_sample
            result["cpu_baseline"] = {
                "value": V / cpu_s, "unit": "grid pts/s", "cores": threads, "kind": "oracle",
                "sample": f"{args.cpu_sample} full-size FP64 oracle applies of {args.workload} "
                          f"({2 * N}^{d} oracle FFTs, {threads} OpenMP threads); plan excluded",
            }
            log(f"[bench] oracle apply {cpu_s:.2f} s on {threads} threads")
        del oplan, ref

    want = {"c1", "c2", "c3", "c4", "c5"} if args.configs == "all" else (
        set() if args.configs == "none" else set(args.configs.split(",")))
    if want:
        del ws, out
        torch.cuda.empty_cache()
        cfg = {}
        if "c1" in want:
            cfg["laplace3d_n32"] = laplace3d_n32_fp64(vg, 20, 3)
        if "c2" in want:
            cfg["helmholtz3d_k20_n128"] = single_config(vg, "helmholtz3d_k20_n128", 20, 3)
        if "c3" in want:
            for name in ("laplace2d_n4096", "helmholtz2d_k200_n4096"):
                cfg[name] = single_config(vg, name, 20, 3, with_gradient=True)
                torch.cuda.empty_cache()
        if "c4" in want:
            cfg["batch64_3d_n48_128"] = batch_config(vg, 20, 3, sample=8)
            torch.cuda.empty_cache()
        if "c5" in want:
            cfg["helmholtz3d_k150_n512_phi_grad"] = large_gradient_config(vg, 5, 2)
            torch.cuda.empty_cache()
        result["configs"] = cfg
    # the paper's own timing for the closest workload, as context (another
    # machine and another workload, hence not vs_baseline)
    result["paper_context"] = {
        "source": "Section 5.3, Table 7: Lippmann-Schwinger solve of a smoothed cube, 3D N = 250 (500^3 padded)",
        "seconds_per_matvec_upper_bound": 3.78,
        "note": "solve time over matvec count; one matvec is one forward and one inverse padded FFT convolution",
        "hardware": "two 8-core Intel Xeon E5-2450",
        "precision": "not stated",
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
