"""Benchmark: fwd+grad QAOA evaluations per second at n=28, p=8 (MaxCut, random 3-regular).

One step = one full evaluation of the hot path: cost-table-driven phase multiplies, X-mixer
rotations, <C> reduction and the reverse sweep for d<C>/d(beta, gamma), on one MI355X. The
table is built before timing (step (a) runs once per instance); every amplitude is resident
in HBM when the timed region starts.

Other workloads (--workload):
  maxcut3reg_n10_p3        n=10, p=3, one angle set (latency of the whole-state kernel)
  batched_er_n12to20_p10   8 weighted G(n,1/2) instances x 256 angle sets, p=10; one step is
                           one batched call (2048 evaluations)
  bisection_g16_k8_p6      clique mixer on Hamming weight 8 of 16 (12870 states), 512 angle
                           sets, p=6; one step is one batched call (512 evaluations)
  maxcut3reg_n32_p16       n=32, p=16 (32 GiB complex64 vectors)
  grover_maxcut3reg_n40_p16  Grover mixer: one step = the table-free degeneracy count over all
                           2^40 states plus one batched fwd+grad over 512 angle sets (p=16);
                           value in states/s
  angles_er_n12_p10        angle finding: one step = iterative basinhopping rounds 1..10 for 50
                           G(12,1/2) MaxCut instances at once; value in evals/s inside the loop
  xorders_maxcut3reg_n24_p4  mixer of all 1- and 2-body X products (tile passes with the basis
                           change as Y rotations), n=24, p=4, 16 angle sets per batched call
  multiangle_maxcut3reg_n24_p4  per-qubit multi-angle X mixer (tile passes, per-qubit diagonal),
                           n=24, p=4, 16 angle sets per batched call

Prints ONE JSON line on stdout (progress goes to stderr):
  value            FP32-state evaluations per second (whole job, one GPU)
  roofline         dominant kernel class: algorithmic bytes (the method's one-pass-per-round
                   traffic) or flops per launch / mean launch time (HIP events on the launch
                   stream, during the timed region) vs the MI355X peak (8 TB/s HBM; 2.5 PFLOP/s
                   dense FP16 MFMA; 157.3 TFLOP/s FP32); the bytes the tile plan moves beside it
  copy_roof        the library's streaming copy kernel over 2 GiB (the practical HBM roof)
  cpu_baseline     the FP64 CPU oracle on a bounded sample of the same workload
  fp64             the same kernels with a complex128 state (the plain FP64 GPU path)
  error            FP32 result vs FP64 oracle values
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
MFMA_F16_PEAK_TFS = 2500.0
FP32_VECTOR_PEAK_TFS = 157.3
# 32-bit integer VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
INT32_VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# LDS atomics: one wave64 ds_add_u32 per 4 clocks per CU (16 lane-ops per clock, bank-conflict free)
LDS_ATOMIC_PEAK_TOPS = 256 * 16 * 2.4e9 / 1e12
METRIC = "fwd+grad QAOA evals/sec & HBM GB/s at n=28 p=8, FP32 vs FP64, err<=1e-5"


def eval_bytes_per_amp(p: int) -> int:
    """Algorithmic traffic of one fwd+grad evaluation at one pass per layer (bytes per
    amplitude): forward 16p (read + write complex64), reverse 32p (two vectors), table
    (2p + 2) x 1 byte."""
    return 16 * p + 32 * p + (2 * p + 2)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def copy_roof(torch, q, _lib, nbytes=2 << 30, reps=20, warm=20):
    """Measured rate (read + write) of the library's own streaming copy kernel
    (``qaoa_stream_copy``: 16-byte non-temporal loads and stores, each byte read and written
    once) over a 2 GiB buffer, timed with HIP events on the stream it is launched on: the HBM
    rate a streaming kernel reaches on this device, and the calibration kernel of the traffic
    counters."""
    ctx = q.Context(0)
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    st = int(torch.cuda.current_stream().cuda_stream)
    for _ in range(warm):                                # clocks settle before the timed copies
        _lib.qaoa_stream_copy(ctx.handle, a.data_ptr(), b.data_ptr(), nbytes, st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        _lib.qaoa_stream_copy(ctx.handle, a.data_ptr(), b.data_ptr(), nbytes, st)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(a, b))
    del a, b
    torch.cuda.empty_cache()
    ctx.close()
    return {"kernel": "k_stream_copy (qaoa_stream_copy)", "GBps": 2 * nbytes / (ms * 1e-3) / 1e9,
            "frac_of_peak": 2 * nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes_read": nbytes,
            "bytes_written": nbytes, "ms": ms, "copy_exact": ok}


class Runner:
    """One workload on one context: single evaluations or one batched call per step."""

    def __init__(self, q, W):
        import torch
        from paper_2312_06451_amd.autograd import qaoa_expectation
        self.q, self.W = q, W
        self.torch, self.qaoa_expectation = torch, qaoa_expectation
        self.ctx = q.Context(0)
        k = W.hamming_k
        self.problems = [q.Problem.from_graph(self.ctx, g, hamming_k=k) for g in W.graphs]
        if W.mixer == "clique":
            self.mixers = [q.Mixer.clique(self.ctx, g.n, k) for g in W.graphs]
        elif W.mixer == "x_orders":
            self.mixers = [q.Mixer.x_orders(self.ctx, g.n, W.extra["orders"]) for g in W.graphs]
        elif W.mixer == "x_multiangle":
            self.mixers = [q.Mixer.x_multiangle(self.ctx, g.n) for g in W.graphs]
        else:
            self.mixers = [q.Mixer.x(self.ctx, g.n) for g in W.graphs]
        self.batched = len(W.graphs) > 1 or W.angles.shape[0] > 1
        self.evals_per_step = len(W.graphs) * (W.angles.shape[0] if self.batched else 1)

    def step(self, prec, grad):
        q, W = self.q, self.W
        if self.batched:
            if grad:
                return q.expect_grad_batched(self.problems, self.mixers, W.angles, precision=prec)
            return q.expect_batched(self.problems, self.mixers, W.angles, precision=prec), None
        if grad:
            # the torch.autograd.Function path: forward <C>, then backward() for the gradient
            ang = self.torch.tensor(W.angles[0], dtype=self.torch.float64, requires_grad=True)
            e = self.qaoa_expectation(ang, self.problems[0], self.mixers[0], prec)
            e.backward()
            return float(e), ang.grad.numpy()
        return q.expect(self.problems[0], self.mixers[0], W.angles[0], precision=prec), None

    def time(self, prec, grad, steps, warmup, torch):
        for _ in range(warmup):
            self.step(prec, grad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = self.step(prec, grad)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out


def cpu_baseline(W, sample):
    """The FP64 oracle on a bounded sample of the workload; returns (record, sample results)."""
    import numpy as np
    import oracle
    k = W.hamming_k
    if W.name == "maxcut3reg_n28_p8":
        # one fwd+adjoint evaluation with p=1 at the full n (one of the p layers), scaled by p
        g = W.graphs[0]
        table = oracle.graph_table(g)
        a1 = np.array([W.angles[0][0], W.angles[0][W.p]])
        t0 = time.perf_counter()
        oracle.grad(g.n, table, a1)
        dt = time.perf_counter() - t0
        return {"value": 1.0 / (dt * W.p), "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"one fwd+adjoint evaluation with p=1 at n={g.n} (1 of the {W.p} layers), "
                          f"{dt:.1f} s, scaled x{W.p} to one p={W.p} evaluation"}, {}
    if W.name == "maxcut3reg_n32_p16":
        return None, {}
    if W.mixer in ("x_orders", "x_multiangle"):
        # one fwd+adjoint evaluation with p=1 on a 3-regular graph of n - 2 vertices, scaled by 4 n / (n - 2)
        # (transform or per-qubit rotation work per amplitude grows with n) and by p
        from oracle import xmixers as X
        n = W.graphs[0].n
        gs = workloads_mod().random_regular_graph(n - 2, 3, 8124)
        table = oracle.graph_table(gs)
        t0 = time.perf_counter()
        if W.mixer == "x_orders":
            d = X.diag_orders(n - 2, W.extra["orders"])
            X.grad(n - 2, table, np.array([W.angles[0][0], W.angles[0][W.p]]), d=d)
        else:
            X.grad(n - 2, table, np.concatenate([W.angles[0][:n - 2], [W.angles[0][W.p * n]]]), multiangle=True)
        dt = time.perf_counter() - t0
        scale = 4.0 * n / (n - 2) * W.p
        return {"value": 1.0 / (dt * scale), "unit": "evals/s", "cores": 1, "kind": "oracle",
                "sample": f"one fwd+adjoint evaluation with p=1 at n={n - 2} (numpy, one thread), {dt:.1f} s, "
                          f"scaled x{scale:.2f} (4 n/(n-2) for the size, x{W.p} for the layers) to one n={n}, "
                          f"p={W.p} evaluation"}, {}
    tables = [oracle.graph_table(g, k) for g in W.graphs]
    res = {}
    t0 = time.perf_counter()
    count = 0
    grad = W.name != "maxcut3reg_n10_p3"
    for (i, s) in sample:
        g = W.graphs[i]
        if grad:
            res[(i, s)] = oracle.grad(g.n, tables[i], W.angles[s], k=k)
        else:
            res[(i, s)] = oracle.expect(g.n, tables[i], W.angles[s], k=k)
        count += 1
    dt = time.perf_counter() - t0
    # the sample's evaluations have the workload's mix of sizes when the sample covers every
    # instance equally
    return {"value": count / dt, "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{count} {'fwd+adjoint' if grad else 'forward'} evaluations "
                      f"({len(set(i for i, _ in sample))} instance(s)), {dt:.1f} s"}, res


def sample_for(W):
    if W.name == "maxcut3reg_n10_p3":
        return [(0, 0)] * 200
    if W.name == "batched_er_n12to20_p10":
        return [(i, s) for i in range(len(W.graphs)) for s in range(2)]
    if W.name == "bisection_g16_k8_p6":
        return [(0, 0)]
    return []


def traffic_from_profile(workload, cls):
    """HBM bytes per launch of the pass kernels from the committed rocprofv3 counter summary,
    valid only while the kernel source is the one the counters were taken with."""
    tpath = os.path.join(ROOT, "profiles", f"pmc_traffic_k_pass_{workload}.md")
    if not os.path.exists(tpath):
        return None
    txt = open(tpath).read()
    csrc = os.path.join(ROOT, "paper_2312_06451_amd", "csrc")
    h = hashlib.sha256()
    # the pass kernel and its launchers
    for f in ("qaoa_tile.h", "qaoa_kernels.hip", "qaoa_xpass.hip", "qaoa_swz_f32.hip", "qaoa_swz_f64.hip"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    if f"kernel_source_sha256 = {h.hexdigest()}" not in txt:
        return None
    for line in txt.splitlines():
        if line.startswith("traffic_bytes_per_launch "):
            k, v = line[len("traffic_bytes_per_launch "):].split("=")
            if k.strip() == cls:
                return float(v)
    return None


KERNEL_NAMES = {"xmix": "k_pass<float,13,1|3|4,uint8,1..4> (tile passes with Y rotations: basis change and "
                        "diagonals of X-product mixers)",
                "fwd_pass": "k_pass<float,13,1,uint8,0> (tile pass, one vector)",
                "rev_pass": "k_pass<float,13,2|3|4,uint8,0> (tile pass, state and adjoint vector)",
                "small": "k_whole / k_small<float> (whole state in one workgroup)",
                "dense": "k_split_gemm_bal<mode> + k_split_gemm_fix<mode> (hand-written split-FP16 MFMA eigenbasis product, XCD-balanced K-split schedule, fused epilogue)"}


def algorithmic_bytes(R, steps):
    """SURVEY-model algorithmic HBM bytes of the timed region per kernel class: every round
    moves each vector it touches once (one pass per round, the lower bound of the method), and
    reads the cost table once per phase. Per amplitude, angle set and fwd+grad evaluation of a
    tile-path instance (n above the whole-state kernels' 13 qubits): forward side
    16p + (p + 1) tb, reverse side (state and adjoint vector) 32p + (p + 1) tb, tb = bytes per
    table entry; for the X-product mixers each round is two half-rounds (diagonal + basis
    change), so both sides double their vector bytes (one class covers both)."""
    W, p = R.W, R.W.p
    sets = W.angles.shape[0] if R.batched else 1
    out = {"fwd_pass": 0.0, "rev_pass": 0.0, "xmix": 0.0}
    for P in R.problems:
        if P.n <= 13:
            continue
        tb = 1 if P.max_value <= 255 else 2
        amps = float(sets) * 2.0 ** P.n * steps
        if W.mixer in ("x_orders", "x_multiangle"):
            out["xmix"] += amps * (2 * 16 * p + 2 * 32 * p + 2 * (p + 1) * tb)
        else:
            out["fwd_pass"] += amps * (16 * p + (p + 1) * tb)
            out["rev_pass"] += amps * (32 * p + (p + 1) * tb)
    return out


def roofline(prof, workload, alg_bytes):
    """Dominant kernel class of the timed region against its roof. HBM classes: `achieved` =
    the class's algorithmic bytes (``algorithmic_bytes``) per launch / mean launch time (HIP
    events on the launch stream), so `frac` is the fraction of the 8 TB/s peak at which the
    method's lower-bound traffic would move; `moved_*` is the same time against the bytes the
    tile plan actually moves (two passes per round at n = 28). MFMA class: algorithmic flops
    of one FP32-accurate real product (2 N^2 x columns) per launch; the split form issues three
    FP16 products per launch (`mfma_issued_*`)."""
    cls = max(("fwd_pass", "rev_pass", "small", "dense", "xmix"), key=lambda k: prof[k]["ms"])
    d = prof[cls]
    L = max(d["launches"], 1)
    mean_ms = d["ms"] / L
    base = {"kernel": KERNEL_NAMES[cls], "class": cls, "launches": d["launches"], "mean_ms": round(mean_ms, 4)}
    if cls in ("fwd_pass", "rev_pass", "xmix"):
        apl = alg_bytes[cls] / L
        a = apl / (mean_ms * 1e-3) / 1e9
        mpl = d["bytes"] / L
        m = mpl / (mean_ms * 1e-3) / 1e9
        return dict({"bound": "hbm", "achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(a / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(workload, cls),
                     "bytes_per_launch": apl, "bytes_model": "one pass per round (16p / 32p B per amplitude "
                     "+ (p + 1) table reads per sweep)",
                     "moved_bytes_per_launch": mpl, "moved_GBps": round(m, 1),
                     "moved_frac": round(m / HBM_PEAK_GBS, 4)}, **base)
    if cls == "dense":
        fpl = d["flops"] / L
        a = fpl / (mean_ms * 1e-3) / 1e12
        return dict({"bound": "mfma", "achieved": round(a, 1), "peak": MFMA_F16_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": round(a / MFMA_F16_PEAK_TFS, 4), "traffic": None, "flops_per_launch": fpl,
                     "mfma_issued_TFLOPs": round(3 * a, 1), "mfma_issued_frac": round(3 * a / MFMA_F16_PEAK_TFS, 4),
                     "counters": mfma_from_profile(workload)},
                    **base)
    return dict({"bound": "alu", "achieved": None, "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
                 "frac": None, "traffic": None}, **base)


def mfma_from_profile(workload):
    """MFMA busy fraction and issued MFMA flops of the split product from the committed
    rocprofv3 counter summary (SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x SIMDs)), valid only
    while the product kernel's source is the one the counters were taken with."""
    tpath = os.path.join(ROOT, "profiles", f"pmc_mfma_k_split_gemm_{workload}.md")
    if not os.path.exists(tpath):
        return None
    txt = open(tpath).read()
    src = os.path.join(ROOT, "paper_2312_06451_amd", "csrc", "qaoa_gemm.hip")
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if f"kernel_source_sha256 = {cur}" not in txt:
        return None
    out = {}
    for line in txt.splitlines():
        for key in ("mfma_busy_frac", "lds_bank_conflicts_per_dispatch", "wait_inst_frac"):
            if line.startswith(key + " = "):
                out[key] = float(line.split("=")[1])
    return out or None


def valu_per_state_from_profile(workload):
    """VALU lane-instructions per counted state from the committed rocprofv3 SQ_INSTS_VALU
    summary, valid only while the counting kernel's source is the one it was taken with."""
    tpath = os.path.join(ROOT, "profiles", f"pmc_valu_k_enum_full_{workload}.md")
    if not os.path.exists(tpath):
        return None
    txt = open(tpath).read()
    src = os.path.join(ROOT, "paper_2312_06451_amd", "csrc", "qaoa_grover.hip")
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if f"kernel_source_sha256 = {cur}" not in txt:
        return None
    for line in txt.splitlines():
        if line.startswith("valu_lane_instructions_per_state = "):
            return float(line.split("=")[1])
    return None


def main_grover(args, W, q, _lib, torch, np):
    """Grover mixer: table-free degeneracy count + batched fwd+grad on the cost classes."""
    import oracle
    g = W.graphs[0]
    n, p = g.n, W.p
    steps = args.steps if args.steps is not None else 5
    warmup = args.warmup
    ctx = q.Context(0)
    h = ctx.handle
    M = q.Mixer.grover(ctx, n)
    log(f"workload {W.name}: {W.description}")

    def step():
        P = q.Problem.degeneracies_of_graph(ctx, g)
        E, G = q.expect_grad_batched([P], [M], W.angles)
        vals, cnt = P.degeneracies()
        P.close()
        return E, G, vals, cnt

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    _lib.qaoa_profile_enable(h, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        E, G, vals, cnt = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = {k: _lib.qaoa_profile_read(h, v) for k, v in _lib.KERNEL_CLASSES.items()}
    _lib.qaoa_profile_enable(h, False)
    N = 2 ** n
    cs, gv = prof["count_states"], prof["grover"]
    count_rate = cs["flops"] / (cs["ms"] * 1e-3)
    eval_rate = gv["launches"] and W.angles.shape[0] * gv["launches"] / (gv["ms"] * 1e-3)
    log(f"step {dt / steps * 1e3:.1f} ms; count {count_rate / 1e12:.3f} Tstates/s; class rounds {eval_rate:.0f} evals/s")
    # exactness: over all 2^n strings the edges' cut indicators are pairwise independent fair
    # bits, so sum m_c = 2^n, sum c m_c = W 2^(n-1), sum (2c - W)^2 m_c = 2^n sum w^2
    c = [int(v) for v in vals]
    m = [int(x) for x in cnt]
    Wt = int(g.w.sum())
    exact = (sum(m) == N and sum(ci * mi for ci, mi in zip(c, m)) == Wt * N // 2
             and sum((2 * ci - Wt) ** 2 * mi for ci, mi in zip(c, m)) == N * int((g.w.astype(np.int64) ** 2).sum()))
    vps = valu_per_state_from_profile(W.name)
    # one LDS histogram increment per counted state (algorithmic): the count is bound by the
    # LDS atomic issue rate; the VALU side is reported beside it from the committed counters
    roof = {"bound": "lds", "achieved": round(count_rate / 1e12, 3), "peak": round(LDS_ATOMIC_PEAK_TOPS, 3),
            "unit": "T LDS-atomic lane-ops/s (one histogram increment per state)",
            "frac": round(count_rate / 1e12 / LDS_ATOMIC_PEAK_TOPS, 4),
            "traffic": None, "kernel": "k_enum_full (Gray-code walk, private LDS histogram)",
            "class": "count_states", "launches": cs["launches"], "mean_ms": round(cs["ms"] / max(1, cs["launches"]), 3),
            "states_per_launch": cs["flops"] / max(1, cs["launches"]), "valu_per_state": vps,
            "valu_tops": None if vps is None else round(count_rate * vps / 1e12, 2),
            "valu_frac": None if vps is None else round(count_rate * vps / 1e12 / INT32_VALU_PEAK_TOPS, 4)}
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's table of a 3-regular graph on 28 vertices (same family, 2^28 states) and its
        # histogram, scaled to states/s
        gs = workloads_mod().workload("maxcut3reg_n28_p8").graphs[0]
        t1 = time.perf_counter()
        tab = oracle.graph_table(gs)
        np.bincount(tab)
        d1 = time.perf_counter() - t1
        cpu = {"value": 2 ** 28 / d1, "unit": "states/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"degeneracies of a random 3-regular graph on 28 vertices: oracle table + histogram, "
                         f"{d1:.1f} s"}
    out = {
        "metric": f"Grover-QAOA table-free degeneracy count + fwd+grad, states/sec ({W.name})",
        "value": round(steps * N / dt, 1), "unit": "states/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(dt / steps * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 (count), f64 (class rounds)", "data": "synthetic",
        "config": {"workload": W.name, "description": W.description, "n": n, "p": p,
                   "angle_sets": int(W.angles.shape[0]), "mixer": "grover", "mode": "count + fwd+grad",
                   "parallelism": "single GPU"},
        "roofline": roof,
        "path": {"count_states_per_s": count_rate, "classes": len(c), "grover_evals_per_s": eval_rate,
                 "count_share_of_step": cs["ms"] / (dt * 1e3)},
        "error": {"degeneracy_identities_exact": bool(exact),
                  "reference": "sum, mean and variance identities of the MaxCut cost over all 2^n states"},
        "cpu_baseline": cpu, "kernels": prof,
    }
    print(json.dumps(out), flush=True)


def main_angles(args, W, q, _lib, torch, np):
    """Angle-finding study: iterative basinhopping rounds 1..p for every instance at once, one
    paired fwd+grad launch per optimiser step for all instances and chains."""
    import oracle
    from oracle import angles as A
    ctx = q.Context(0)
    h = ctx.handle
    probs = [q.Problem.from_graph(ctx, g) for g in W.graphs]
    mixers = [q.Mixer.x(ctx, g.n) for g in W.graphs]
    opts = dict(W.extra)
    steps = args.steps if args.steps is not None else 1
    warmup = min(args.warmup, 1)
    log(f"workload {W.name}: {W.description}")
    for _ in range(warmup):
        q.find_angles_multi(probs, mixers, W.p, **opts)
    torch.cuda.synchronize()
    _lib.qaoa_profile_enable(h, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        res = q.find_angles_multi(probs, mixers, W.p, **opts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = {k: _lib.qaoa_profile_read(h, v) for k, v in _lib.KERNEL_CLASSES.items()}
    _lib.qaoa_profile_enable(h, False)
    sm = prof["small"]
    N = 2 ** W.graphs[0].n
    evals = sm["bytes"] / N          # one byte of table per amplitude and evaluation (uint8 tables)
    rate = evals / dt
    mean_ms = sm["ms"] / max(1, sm["launches"])
    achieved = sm["flops"] / (sm["ms"] * 1e-3) / 1e12
    log(f"study {dt / steps:.2f} s; {evals / steps:.0f} evaluations/study, {rate:.0f} evals/s; "
        f"{sm['launches'] / steps:.0f} launches/study, mean {mean_ms * 1e3:.1f} us, kernel share "
        f"{sm['ms'] / (dt * 1e3):.3f}")
    # validity: every round's value is the oracle's <C> at the returned angles; rounds never get worse
    worst, mono = 0.0, True
    for (ang, vals), g in zip(res, W.graphs):
        t = oracle.graph_table(g)
        mono = mono and bool(np.all(np.diff(vals) >= -1e-6 * t.max()))
        for r in (1, W.p):
            E, Nr = oracle.expect(g.n, t, ang[r - 1])
            worst = max(worst, abs(E / Nr - vals[r - 1]) / t.max())
    roof = {"bound": "alu", "achieved": round(achieved, 2), "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VECTOR_PEAK_TFS, 4), "traffic": None,
            "kernel": KERNEL_NAMES["small"], "class": "small", "launches": sm["launches"],
            "mean_ms": round(mean_ms, 4), "flops_per_launch": sm["flops"] / max(1, sm["launches"])}
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's own search (same options) on the first instance, rounds 1..3
        g = W.graphs[0]
        t = oracle.graph_table(g)
        calls = [0]

        def fun_for(r):
            f = A.Objective(g.n, t)

            def counted(x):
                calls[0] += 1
                return f(x)
            return counted
        t1 = time.perf_counter()
        A.find_angles(fun_for, 3, **opts)
        d1 = time.perf_counter() - t1
        cpu = {"value": calls[0] / d1, "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"the oracle's find_angles (same options) on 1 of the {len(W.graphs)} instances, "
                         f"rounds 1..3: {calls[0]} fwd+adjoint evaluations in {d1:.1f} s (cheaper p than the "
                         f"study's 1..{W.p} mix)"}
    mean_values = np.mean([v for _, v in res], axis=0)
    out = {
        "metric": f"fwd+grad QAOA evals/sec inside the angle-finding loop ({W.name})",
        "value": round(rate, 1), "unit": "evals/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(dt / steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": W.name, "description": W.description, "instances": len(W.graphs),
                   "n": W.graphs[0].n, "p_max": W.p, "mixer": "x", "mode": "find_angles (basinhopping rounds)",
                   "options": opts, "state": "complex64, FP64 sums", "parallelism": "single GPU"},
        "roofline": roof,
        "path": {"studies_per_s": steps / dt, "instances_per_s": steps * len(W.graphs) / dt,
                 "evaluations_per_study": evals / steps, "launches_per_study": sm["launches"] / steps,
                 "kernel_share_of_wall": sm["ms"] / (dt * 1e3), "mean_value_per_round": mean_values.tolist()},
        "error": {"value_vs_oracle_max_rel": worst, "rounds_monotone": mono,
                  "reference": "FP64 oracle <C> at the returned angles (rounds 1 and p of every instance)"},
        "cpu_baseline": cpu, "kernels": prof,
    }
    print(json.dumps(out), flush=True)


def workloads_mod():
    import workloads
    return workloads


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="maxcut3reg_n28_p8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-fwd-only", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="fixed tile-pass plan rule instead of the library's measured plan choice")
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

    W = workloads.workload(args.workload)
    if W.mixer == "grover":
        return main_grover(args, W, q, _lib, torch, np)
    if W.name == "angles_er_n12_p10":
        return main_angles(args, W, q, _lib, torch, np)
    steps = args.steps if args.steps is not None else {"maxcut3reg_n10_p3": 200, "maxcut3reg_n32_p16": 2}.get(W.name, 20)
    warmup = min(args.warmup, 1) if W.name == "maxcut3reg_n32_p16" else args.warmup
    grad = W.name != "maxcut3reg_n10_p3"

    roof_copy = copy_roof(torch, q, _lib)
    log(f"copy roof: {roof_copy['GBps']:.0f} GB/s")
    R = Runner(q, W)
    h = R.ctx.handle
    if not args.no_autotune:
        R.ctx.set_autotune(True)   # plans measured on first use (in the warm-up), then fixed
    log(f"workload {W.name}: {W.description}")

    # ---- FP32 state (timed, with per-kernel events)
    _lib.qaoa_profile_enable(h, False)
    for _ in range(warmup):
        R.step(q.QAOA_FP32, grad)
    graph_timing = None
    if R.batched and W.mixer == "x":
        # batched transverse-field calls replay a captured HIP graph, which per-launch events
        # cannot bracket: the whole-job value is timed without them, the kernel classes in a
        # second, event-timed region of the same length
        dtg, outg = R.time(q.QAOA_FP32, grad, steps, 0, torch)
        graph_timing = {"ms_per_step": dtg / steps * 1e3, "evals_per_s": steps * R.evals_per_step / dtg}
        log(f"FP32 (graph replays): {dtg / steps * 1e3:.3f} ms/step")
    _lib.qaoa_profile_enable(h, True)
    dt32, out32 = R.time(q.QAOA_FP32, grad, steps, 0, torch)
    prof = {k: _lib.qaoa_profile_read(h, v) for k, v in _lib.KERNEL_CLASSES.items()}
    _lib.qaoa_profile_enable(h, False)
    evals32 = steps * R.evals_per_step / dt32
    log(f"FP32: {dt32 / steps * 1e3:.3f} ms/step, {evals32:.2f} evals/s; kernels {prof}")
    event_timing = None
    if graph_timing is not None:
        event_timing = {"ms_per_step": dt32 / steps * 1e3, "evals_per_s": evals32}
        dt32, out32, evals32 = dtg, outg, graph_timing["evals_per_s"]

    # ---- forward only (the cost of the gradient relative to one evaluation)
    fwd = None
    if grad and not args.no_fwd_only:
        sf = max(1, steps // 2)
        dtf, _ = R.time(q.QAOA_FP32, False, sf, 1, torch)
        fwd = {"ms_per_step": dtf / sf * 1e3, "grad_over_fwd": (dt32 / steps) / (dtf / sf)}
        log(f"forward only: {fwd}")

    # ---- FP64 state (the plain FP64 GPU path: same kernels, complex128 / DGEMM)
    fp64 = None
    if not args.no_fp64:
        s64 = max(1, steps // 4)
        dt64, out64 = R.time(q.QAOA_FP64, grad, s64, 1, torch)
        fp64 = {"value": s64 * R.evals_per_step / dt64, "unit": "evals/s", "ms_per_step": dt64 / s64 * 1e3,
                "steps": s64}
        log(f"FP64: {dt64 / s64 * 1e3:.3f} ms/step")

    def pick(out, i, s):
        e, g = out
        if R.batched:
            return float(np.asarray(e)[i, s]), (None if g is None else np.asarray(g)[i, s])
        return float(e), (None if g is None else np.asarray(g))

    # ---- CPU oracle on a bounded sample; its results also give the error of the GPU path
    cpu, ref = None, {}
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle) ...")
        cpu, ref = cpu_baseline(W, sample_for(W))
        log(f"CPU: {cpu}")

    # ---- error vs FP64 oracle values (stored ones for the single-set workloads)
    gpath = os.path.join(ROOT, "tests", "golden", W.name + ".json")
    if os.path.exists(gpath):
        G = json.load(open(gpath))
        for s, rec in enumerate(G["sets"]):
            if s < W.angles.shape[0] and np.array_equal(np.array(rec["angles"]), W.angles[s]):
                ref[(0, s)] = (rec["expect"], 1.0, np.array(rec["grad"]))
    err = None
    if ref:
        ee, ge, ee64, ge64 = [], [], [], []
        for (i, s), r in ref.items():
            if grad:
                E0, N0, g0 = r
                e, gr = pick(out32, i, s)
                ee.append(abs(e - E0 / N0) / abs(E0 / N0))
                ge.append(float(np.max(np.abs(gr - g0 / N0)) / np.max(np.abs(g0 / N0))))
                if fp64:
                    e6, g6 = pick(out64, i, s)
                    ee64.append(abs(e6 - E0 / N0) / abs(E0 / N0))
                    ge64.append(float(np.max(np.abs(g6 - g0 / N0)) / np.max(np.abs(g0 / N0))))
            else:
                E0, N0 = r[0], r[1]
                e, _ = pick(out32, i, s)
                ee.append(abs(e - E0 / N0) / abs(E0 / N0))
                if fp64:
                    ee64.append(abs(pick(out64, i, s)[0] - E0 / N0) / abs(E0 / N0))
        err = {"expect_rel": max(ee), "grad_inf_rel": max(ge) if ge else None,
               "fp64_expect_rel": max(ee64) if ee64 else None, "fp64_grad_inf_rel": max(ge64) if ge64 else None,
               "reference": f"FP64 CPU oracle, {len(ref)} evaluation(s)"}

    roof = roofline(prof, W.name, algorithmic_bytes(R, steps))
    path = None
    if W.mixer == "x" and len(W.graphs) == 1:
        g = W.graphs[0]
        all_pass_ms = prof["fwd_pass"]["ms"] + prof["rev_pass"]["ms"]
        all_pass_bytes = prof["fwd_pass"]["bytes"] + prof["rev_pass"]["bytes"]
        path = {"algorithmic_bytes_per_eval": eval_bytes_per_amp(W.p) * 2.0 ** g.n,
                "algorithmic_GBps": eval_bytes_per_amp(W.p) * 2.0 ** g.n * evals32 / 1e9,
                "moved_bytes_per_eval": all_pass_bytes / steps if all_pass_ms else None,
                "pass_kernels_GBps": all_pass_bytes / (all_pass_ms * 1e-3) / 1e9 if all_pass_ms else None}
        path["algorithmic_frac"] = path["algorithmic_GBps"] / HBM_PEAK_GBS
    if W.mixer == "clique":
        d = prof["dense"]
        path = {"products_per_step": d["launches"] / steps,
                "algorithmic_TFLOPs_per_step": d["flops"] / steps / 1e12,
                "dense_share_of_step": d["ms"] / (dt32 * 1e3)}

    cfg = {"workload": W.name, "description": W.description, "p": W.p,
           "instances": len(W.graphs), "n": [g.n for g in W.graphs] if len(W.graphs) > 1 else W.graphs[0].n,
           "angle_sets": int(W.angles.shape[0]), "mixer": W.mixer, "mode": "fwd+grad" if grad else "fwd",
           "state": "complex64, FP64 sums", "parallelism": "single GPU"}
    if W.hamming_k >= 0:
        cfg["hamming_k"] = W.hamming_k
    out = {
        "metric": METRIC if W.name == "maxcut3reg_n28_p8" else f"{cfg['mode']} QAOA evals/sec ({W.name})",
        "value": round(evals32, 3), "unit": "evals/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(dt32 / steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": cfg,
        "roofline": roof, "path": path, "copy_roof": roof_copy, "fp64": fp64,
        "plans": R.ctx.plans().splitlines()[1:],
        "event_timed_region": event_timing,
        "speedup_vs_fp64": (evals32 / fp64["value"]) if fp64 else None, "forward_only": fwd,
        "error": err, "cpu_baseline": cpu, "kernels": prof,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
