"""Benchmark: fwd+grad QAOA evaluations per second at n=28, p=8 (MaxCut, random 3-regular).

One step = one full evaluation of the hot path: cost-table-driven phase multiplies, X-mixer
rotations, <C> reduction and the reverse sweep for d<C>/d(beta, gamma), on one MI355X. The
table is built before timing (step (a) runs once per instance); every amplitude is resident
in HBM when the timed region starts.

Prints ONE JSON line on stdout (progress goes to stderr):
  value            FP32-state evaluations per second (whole job, one GPU)
  roofline         dominant kernel: algorithmic bytes per launch / mean launch time (HIP
                   events on the launch stream, during the timed region) vs 8 TB/s
  cpu_baseline     the FP64 CPU oracle on a bounded sample of the same workload
  fp64             the same kernels with a complex128 state (the plain FP64 GPU path)
  error            FP32 result vs the oracle's stored FP64 values
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "fwd+grad QAOA evals/sec & HBM GB/s at n=28 p=8, FP32 vs FP64, err<=1e-5"
# Algorithmic traffic of one fwd+grad evaluation at one pass per layer (bytes per amplitude):
# forward 16p (read+write complex64), reverse 32p (two vectors), table (2p+2) x 1 byte.
def eval_bytes_per_amp(p: int) -> int:
    return 16 * p + 32 * p + (2 * p + 2)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(q, P, M, angles, prec, steps, warmup, torch):
    for _ in range(warmup):
        q.expect_grad(P, M, angles, precision=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        e, g = q.expect_grad(P, M, angles, precision=prec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0), e, g


def copy_roof(torch, nbytes=2 << 30, reps=5):
    """Measured device-to-device copy rate (read + write) of a 2 GiB buffer: the achievable
    HBM rate for a streaming kernel, and the calibration kernel of the traffic counters."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"GBps": 2 * nbytes / (ms * 1e-3) / 1e9, "bytes_read": nbytes, "bytes_written": nbytes, "ms": ms}


def cpu_baseline(W, seconds_hint=True):
    """FP64 oracle, fwd + adjoint with p=1 at the full n (one of the p layers), scaled by p."""
    import numpy as np
    import oracle
    g = W.graphs[0]
    table = oracle.graph_table(g)
    a1 = np.array([W.angles[0][0], W.angles[0][W.p]])
    t0 = time.perf_counter()
    oracle.grad(g.n, table, a1)
    dt = time.perf_counter() - t0
    per_eval = dt * W.p
    return {"value": 1.0 / per_eval, "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one fwd+adjoint evaluation with p=1 at n={g.n} (1 of the {W.p} layers), "
                      f"{dt:.1f} s, scaled x{W.p} to one p={W.p} evaluation"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="maxcut3reg_n28_p8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the QAOA state of this workload is evaluated on a single "
              "MI355X (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    import paper_2312_06451_amd as q
    from paper_2312_06451_amd import _lib

    roof_copy = copy_roof(torch)
    log(f"copy roof: {roof_copy['GBps']:.0f} GB/s")
    W = workloads.workload(args.workload)
    g = W.graphs[0]
    angles = W.angles[0]
    n, p = g.n, W.p
    ctx = q.Context(0)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    log(f"workload {args.workload}: n={n} p={p} edges={g.m}")

    # ---- FP32 state (timed, with per-kernel events)
    _lib.qaoa_profile_enable(ctx.handle, False)
    for _ in range(args.warmup):
        q.expect_grad(P, M, angles, precision=q.QAOA_FP32)
    _lib.qaoa_profile_enable(ctx.handle, True)
    dt32, e32, g32 = time_steps(q, P, M, angles, q.QAOA_FP32, args.steps, 0, torch)
    prof = {k: _lib.qaoa_profile_read(ctx.handle, v) for k, v in _lib.KERNEL_CLASSES.items()}
    _lib.qaoa_profile_enable(ctx.handle, False)
    evals32 = args.steps / dt32
    log(f"FP32: {dt32 / args.steps * 1e3:.2f} ms/eval, {evals32:.2f} evals/s; kernels {prof}")

    # ---- FP64 state (the plain FP64 GPU path: same kernels, complex128)
    fp64 = None
    if not args.no_fp64:
        s64 = max(2, args.steps // 4)
        dt64, e64, g64 = time_steps(q, P, M, angles, q.QAOA_FP64, s64, 1, torch)
        fp64 = {"value": s64 / dt64, "unit": "evals/s", "ms_per_step": dt64 / s64 * 1e3, "steps": s64}
        log(f"FP64: {dt64 / s64 * 1e3:.2f} ms/eval")

    # ---- error vs the oracle's stored FP64 values
    err = None
    gpath = os.path.join(ROOT, "tests", "golden", args.workload + ".json")
    if os.path.exists(gpath):
        G = json.load(open(gpath))
        s = G["sets"][0]
        if np.allclose(s["angles"], angles, rtol=0, atol=0):
            ref_e, ref_g = s["expect"], np.array(s["grad"])
            err = {"expect_rel": abs(e32 - ref_e) / abs(ref_e),
                   "grad_inf_rel": float(np.max(np.abs(g32 - ref_g)) / np.max(np.abs(ref_g))),
                   "reference": "FP64 CPU oracle (stored)"}
            if fp64 is not None:
                err["fp64_expect_rel"] = abs(e64 - ref_e) / abs(ref_e)
                err["fp64_grad_inf_rel"] = float(np.max(np.abs(g64 - ref_g)) / np.max(np.abs(ref_g)))

    # ---- HBM traffic per launch from the committed rocprofv3 counter summary, valid only
    # while the kernel source is the one the counters were taken with
    traffic = {}
    tpath = os.path.join(ROOT, "profiles", f"pmc_traffic_k_pass_{args.workload}.md")
    if os.path.exists(tpath):
        import hashlib
        txt = open(tpath).read()
        ksrc = os.path.join(ROOT, "paper_2312_06451_amd", "csrc", "qaoa_kernels.hip")
        cur = hashlib.sha256(open(ksrc, "rb").read()).hexdigest()
        if f"kernel_source_sha256 = {cur}" in txt:
            for line in txt.splitlines():
                if line.startswith("traffic_bytes_per_launch "):
                    k, v = line[len("traffic_bytes_per_launch "):].split("=")
                    traffic[k.strip()] = float(v)

    # ---- roofline of the dominant kernel class
    dom = max(("fwd_pass", "rev_pass"), key=lambda k: prof[k]["ms"])
    d = prof[dom]
    mean_ms = d["ms"] / max(d["launches"], 1)
    bytes_per_launch = d["bytes"] / max(d["launches"], 1)
    achieved = bytes_per_launch / (mean_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic.get(dom),
            "kernel": "k_pass<float,13,2,uint8>" if dom == "rev_pass" else "k_pass<float,13,1,uint8>",
            "class": dom, "launches": d["launches"], "mean_ms": round(mean_ms, 4),
            "bytes_per_launch": bytes_per_launch}
    all_pass_ms = prof["fwd_pass"]["ms"] + prof["rev_pass"]["ms"]
    all_pass_bytes = prof["fwd_pass"]["bytes"] + prof["rev_pass"]["bytes"]
    path = {"algorithmic_bytes_per_eval": eval_bytes_per_amp(p) * 2.0 ** n,
            "algorithmic_GBps": eval_bytes_per_amp(p) * 2.0 ** n * evals32 / 1e9,
            "moved_bytes_per_eval": all_pass_bytes / args.steps,
            "pass_kernels_GBps": all_pass_bytes / (all_pass_ms * 1e-3) / 1e9 if all_pass_ms else None}
    path["algorithmic_frac"] = path["algorithmic_GBps"] / HBM_PEAK_GBS

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle) ...")
        cpu = cpu_baseline(W)
        log(f"CPU: {cpu}")

    out = {
        "metric": METRIC, "value": round(evals32, 3), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt32 / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "p": p, "graph": "random 3-regular, pairing model",
                   "mixer": "transverse field", "mode": "fwd+grad", "state": "complex64, FP64 sums",
                   "parallelism": "single GPU"},
        "roofline": roof, "path": path, "copy_roof": roof_copy, "fp64": fp64,
        "speedup_vs_fp64": (evals32 / fp64["value"]) if fp64 else None,
        "error": err, "cpu_baseline": cpu,
        "kernels": prof,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
