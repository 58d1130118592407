#!/usr/bin/env python3
"""Throughput of hybrid-dealiased complex convolution on one MI355X.

Workload (default): 1D complex convolution, A = 2 inputs, B = 1 output,
L = 2^20, M = 2^21 (padding ratio 1/2), complex64 entries uniform in the unit
disk from a fixed seed; hybrid dealiasing as planned by libhdconv.  A step is
one hdconv_execute over inputs resident in HBM.

Printed as ONE JSON line: outputs/s (value), the roofline of the dominant
kernel (algorithmic bytes per launch / its average HIP-event duration, against
the 8 TB/s HBM peak), comparison legs on the same GPU (explicit padding, FP64,
L = 1,500,000), and the FP64 CPU oracle timed on the host cores as a baseline.
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

METRIC = "conv outputs/s + %HBM roofline: hybrid vs explicit pad, FP32 vs FP64 (err≤1e-5)"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["hd_k_fused.hip", "hd_k_multi.hip", "hd_k_outer.hip", "hd_kcommon.hpp", "hd_fft.hpp",
                  "hd_common.hpp", "hd_engine.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2303_17510_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    if name == "c2":
        return {"workload": "1D complex conv, A=2, B=1, L=2^20, M=2^21, complex64, unit disk, hybrid",
                "L": [1 << 20], "M": [1 << 21], "A": 2, "dtype": "c64", "config_id": 1}
    if name == "c2_1p5m":
        return {"workload": "1D complex conv, A=2, B=1, L=1500000, M=2999999, complex64, unit disk, hybrid",
                "L": [1500000], "M": [2999999], "A": 2, "dtype": "c64", "config_id": 1}
    if name == "c4":
        return {"workload": "2D complex conv, A=2, B=1, 2048x2048, M=4096x4096, complex64, Gaussian, hybrid",
                "L": [2048, 2048], "M": [4096, 4096], "A": 2, "dtype": "c64", "config_id": 3, "dist": "gauss"}
    if name == "c5_3d":
        return {"workload": "3D complex conv, A=2, B=1, 256^3, M=512^3, complex64, unit disk, hybrid",
                "L": [256] * 3, "M": [512] * 3, "A": 2, "dtype": "c64", "config_id": 4}
    if name == "c2_centered":
        return {"workload": "1D centered complex conv, A=2, B=1, L=2^20, M=3*2^19, complex64, unit disk, hybrid",
                "L": [1 << 20], "M": [3 << 19], "A": 2, "dtype": "c64", "config_id": 1, "centered": True}
    if name == "c4_centered":
        return {"workload": "2D centered complex conv, A=2, B=1, 2048x2048, M=3072x3072, complex64, Gaussian, hybrid",
                "L": [2048, 2048], "M": [3072, 3072], "A": 2, "dtype": "c64", "config_id": 3, "dist": "gauss",
                "centered": True}
    if name == "c2_hermitian":
        return {"workload": "1D Hermitian complex conv, A=2, B=1, L=2^20 (2^19 stored), M=3*2^19, complex64, "
                            "unit disk, hybrid",
                "L": [1 << 20], "M": [3 << 19], "A": 2, "dtype": "c64", "config_id": 1, "hermitian": True}
    if name == "c4_hermitian":
        return {"workload": "2D Hermitian complex conv, A=2, B=1, 2047x2048 (2047x1024 stored), M=3072x3072, "
                            "complex64, Gaussian, hybrid",
                "L": [2047, 2048], "M": [3072, 3072], "A": 2, "dtype": "c64", "config_id": 3, "dist": "gauss",
                "hermitian": True}
    if name == "basdevant2d_hermitian":
        return {"workload": "2D Hermitian quadratic conv (Basdevant: u^2-v^2, uv), A=2, B=2, 2047x2048 "
                            "(2047x1024 stored), M=3072x3072, complex64, Gaussian, hybrid",
                "L": [2047, 2048], "M": [3072, 3072], "A": 2, "dtype": "c64", "config_id": 3, "dist": "gauss",
                "hermitian": True, "B": 2, "coef": BASDEVANT_2D}
    if name == "basdevant3d":
        return {"workload": "3D quadratic conv (Basdevant: u^2-w^2, v^2-w^2, uv, uw, vw), A=3, B=5, 256^3, "
                            "M=512^3, complex64, unit disk, hybrid",
                "L": [256] * 3, "M": [512] * 3, "A": 3, "dtype": "c64", "config_id": 4, "B": 5,
                "coef": BASDEVANT_3D}
    if name == "mhd3d":
        return {"workload": "3D quadratic conv (MHD, Elsasser form: z+_0 z-_0 - z+_2 z-_2, z+_1 z-_1 - z+_2 z-_2, "
                            "z+_i z-_j for i != j), A=6, B=8, 256^3, M=512^3, complex64, unit disk, hybrid",
                "L": [256] * 3, "M": [512] * 3, "A": 6, "dtype": "c64", "config_id": 4, "B": 8,
                "coef": mhd_coefficients()}
    raise SystemExit("unknown workload " + name)


def mhd_coefficients():
    """Elsasser form of the 3D MHD nonlinearity: inputs z+ (0, 1, 2), z- (3, 4, 5)."""
    def out(terms):
        c = [[0.0] * 6 for _ in range(6)]
        for (i, j), w in terms.items():
            c[min(i, j)][max(i, j)] += w
        return c
    coef = [out({(0, 3): 1, (2, 5): -1}), out({(1, 4): 1, (2, 5): -1})]
    coef += [out({(i, 3 + j): 1}) for i in range(3) for j in range(3) if i != j]
    return coef


# Basdevant forms of the Navier-Stokes nonlinearity (coefficients c[b][i][j], i <= j)
BASDEVANT_2D = [[[1, 0], [0, -1]], [[0, 1], [0, 0]]]
BASDEVANT_3D = [[[1, 0, 0], [0, 0, 0], [0, 0, -1]], [[0, 0, 0], [0, 1, 0], [0, 0, -1]],
                [[0, 1, 0], [0, 0, 0], [0, 0, 0]], [[0, 0, 1], [0, 0, 0], [0, 0, 0]],
                [[0, 0, 0], [0, 0, 1], [0, 0, 0]]]


def make_inputs(wl, dtype):
    import numpy as np
    import torch
    from paper_2303_17510_amd import synth
    npdt = np.complex64 if dtype == "c64" else np.complex128
    shape = tuple(wl["L"][:-1]) + ((wl["L"][-1] + 1) // 2,) if wl.get("hermitian") else tuple(wl["L"])
    if wl.get("copies", 1) > 1:
        shape = (wl["copies"],) + shape
    xs = synth.inputs(wl["config_id"], wl["A"], shape, wl.get("dist", "disk"), dtype=npdt)
    return xs, [torch.from_numpy(x).cuda() for x in xs]


def time_plan(plan, dev, steps, warmup):
    """ms per execute over `steps` back-to-back executes, plus per-launch event stats."""
    import torch
    out = torch.empty_like(dev[0]) if plan.B == 1 else [torch.empty_like(dev[0]) for _ in range(plan.B)]
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.execute(dev, out)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        plan.execute(dev, out)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    # per-kernel durations: events recorded by the library on the same stream
    plan.profile_begin(steps)
    for _ in range(steps):
        plan.execute(dev, out)
    torch.cuda.synchronize()
    stats = plan.profile_end()
    return ms, stats, out


def dominant(stats):
    agg = {}
    for s in stats:
        a = agg.setdefault(s["name"], {"total_ms": 0.0, "launches": 0, "bytes": 0.0, "slots": 0})
        a["total_ms"] += s["total_ms"]
        a["launches"] += s["launches"]
        a["bytes"] += s["bytes_per_launch"] * s["launches"]
        a["slots"] += 1
    name = max(agg, key=lambda k: agg[k]["total_ms"])
    a = agg[name]
    avg_ms = a["total_ms"] / a["launches"]
    bpl = a["bytes"] / a["launches"]
    return name, avg_ms, bpl, agg


def read_traffic(kernel: str, wlname: str, khash: str):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter summary."""
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.txt" % (kernel, wlname))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_src") != khash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def leg(wl, dtype, method, steps, warmup, tuner="heuristic", m=None, **plan_kw):
    import math
    from paper_2303_17510_amd import Plan
    xs, dev = make_inputs(wl, dtype)
    t0 = time.perf_counter()
    kw = dict(plan_kw)
    if m:
        kw["m"] = m
    if wl.get("centered"):
        kw["centered"] = True
    if wl.get("hermitian"):
        kw["hermitian"] = True
    if wl.get("B", 1) > 1:
        kw.update(B=wl["B"], mult="quadratic", coef=wl["coef"])
    if wl.get("copies", 1) > 1:
        kw["copies"] = wl["copies"]
    with Plan(tuple(wl["L"]), tuple(wl["M"]), A=wl["A"], dtype=dtype, method=method, tuner=tuner, **kw) as p:
        plan_s = time.perf_counter() - t0
        info = p.info()
        ms, stats, out = time_plan(p, dev, steps, warmup)
    name, avg_ms, bpl, agg = dominant(stats)
    # outputs of the convolution (a Hermitian result of length L has L entries, half stored), all B arrays
    n_out = wl.get("B", 1) * wl.get("copies", 1)
    for l in wl["L"]:
        n_out *= l
    r = {"stats": stats, "info": info, "dtype": dtype, "method": method, "tuner": tuner, "plan_s": plan_s,
         "candidates": info.get("tuned_candidates"), "timed_candidates": info.get("timed_candidates"), "ms": ms,
         "outputs_per_s": n_out / (ms * 1e-3),
         "ns_per_NlogN": ms * 1e6 / (n_out * math.log2(max(2, n_out))),
         "plan": [(d["variant"], d["m"], d["p"], d["n"], d["q"]) for d in info["dims"]],
         "traffic_by_design_GBps": info["traffic_bytes"] / (ms * 1e-3) / 1e9,
         "compulsory_frac": info["compulsory_bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
         "dominant": {"kernel": name, "avg_ms": avg_ms,
                      "frac": bpl / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
         "kernels": {k: {"avg_ms": v["total_ms"] / v["launches"],
                         "GBps": (v["bytes"] / v["launches"]) / (v["total_ms"] / v["launches"] * 1e-3) / 1e9}
                     for k, v in agg.items()}}
    return r, xs, out


def batched_leg(steps, warmup, dtype="c64", count=4096, tuner="heuristic", Ls=None, config_id=2):
    """Independent convolutions in one graph launch: by default 4096 with L
    log-uniform in [64, 65536] and M = 2L."""
    import numpy as np
    import torch
    from paper_2303_17510_amd import BatchPlan, synth
    if Ls is None:
        Ls = [int(v) for v in synth.batched_lengths(count=count)]
    count = len(Ls)
    tot = sum(Ls)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    big = [torch.from_numpy(synth.unit_disk((tot,), synth.seed_for(config_id, a)).astype(npdt)).cuda()
           for a in range(2)]
    out_big = torch.empty_like(big[0])
    offs = np.concatenate([[0], np.cumsum(Ls)])
    ins = [[big[a][offs[i]:offs[i + 1]] for a in range(2)] for i in range(count)]
    outs = [out_big[offs[i]:offs[i + 1]] for i in range(count)]
    t0 = time.perf_counter()
    with BatchPlan(Ls, dtype=dtype, tuner=tuner) as bp:
        plan_s = time.perf_counter() - t0
        groups = bp.groups()
        bound = bp.bind(ins, outs)   # pointer tables built once, outside the timed region
        for _ in range(max(2, warmup)):   # the second execute captures the graph
            bound.execute()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(steps):
            bound.execute()
        t1.record()
        torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    w = 8 if dtype == "c64" else 16
    return {"dtype": dtype, "method": "hybrid, batched graph", "tuner": tuner, "plan_s": plan_s,
            "convolutions": count, "outputs": tot, "ms": ms, "outputs_per_s": tot / (ms * 1e-3),
            "compulsory_frac": 3 * w * tot / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "groups": [(g["variant"], g["m"], g["p"], g["q"], g["count"]) for g in groups]}


def explicit_best(wl, dtype, steps, warmup):
    """Explicit padding with the fastest split N' = p m among a few m (the
    baseline gets its own small search, as the hybrid plan gets the tuner)."""
    best = None
    for m in (None, 2048, 4096, 8192):
        try:
            r, _, o = leg(wl, dtype, "explicit", steps, warmup, m=m)
        except Exception:
            continue
        if best is None or r["ms"] < best[0]["ms"]:
            best = (r, o)
    return best


def kernel_flops(name, info, A=2):
    """Algorithmic floating-point operations of one launch of a 1D plan's
    kernel: 5 N log2 N per N-point complex FFT, 6 per complex multiply."""
    import math
    if len(info["dims"]) != 1:
        return None
    d = info["dims"][0]
    m, p, D, q = d["m"], d["p"], d["D"], d["q"]
    fft = lambda n: 5.0 * n * math.log2(n) if n > 1 else 0.0  # noqa: E731
    if name == "rows_conv":
        return D * p * ((A + 1) * fft(m) + 6.0 * m * (A + 1 + A - 1))
    if name == "cols_fwd":
        return A * D * m * (fft(p) + 6.0 * p)
    if name == "cols_bwd":
        return D * m * (fft(p) + 6.0 * p) + 2.0 * D * p * m
    if name == "fused1d":
        return q * ((A + 1) * fft(m) + 6.0 * m * (p * A + p + A - 1))
    return None


def copy_baseline(nbytes, reps=50):
    """GB/s of a plain device copy moving the same bytes (half read, half
    written) as one launch of the dominant kernel: the practical ceiling for
    a kernel of that size, beside the 8 TB/s peak."""
    import torch
    n = max(1, int(nbytes // 8))
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    return 8.0 * n / (ms * 1e-3) / 1e9


def cpu_baseline(wl, xs_by_dtype, outs_by_dtype, budget_s):
    """Time the FP64 oracle (explicit FFT convolution) on the workload; errors of the GPU results."""
    import oracle
    from paper_2303_17510_amd import synth
    res = {}
    errs = {}
    n_out = 1
    for l in wl["L"]:
        n_out *= l
    runs, t_total = 0, 0.0
    for dtype, xs in xs_by_dtype.items():
        ins = [synth.as_oracle(x) for x in xs]
        t0 = time.perf_counter()
        ref = oracle.conv_explicit(ins)
        dt = time.perf_counter() - t0
        runs += 1
        t_total += dt
        for key, out in outs_by_dtype.get(dtype, {}).items():
            errs[key] = oracle.rel_l2(out.cpu().numpy(), ref)
    # more runs on the first input set until the time budget is used
    xs = next(iter(xs_by_dtype.values()))
    ins = [synth.as_oracle(x) for x in xs]
    while t_total < budget_s:
        t0 = time.perf_counter()
        oracle.conv_explicit(ins)
        t_total += time.perf_counter() - t0
        runs += 1
    cores = oracle.num_threads()
    # one run on a single thread too (the paper's T = 1 setting)
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.conv_explicit(ins)
    t1 = time.perf_counter() - t0
    oracle.set_num_threads(cores)
    res = {"value": n_out * runs / t_total, "unit": "outputs/s", "cores": cores, "kind": "oracle",
           "sample": "%d full runs of the workload through the FP64 oracle's explicitly padded FFT "
                     "convolution (own radix-2 FFT, OpenMP), %.1f s total" % (runs, t_total),
           "single_thread_value": n_out / t1}
    return res, errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=["c2", "c2_1p5m", "c4", "c5_3d", "c2_centered",
                                                         "c4_centered", "c2_hermitian", "c4_hermitian"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-compare", action="store_true", help="skip explicit / FP64 / other-size legs")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hybrid-dealiasing path runs on a single MI355X "
              "(several GPUs would each take a share of the residues or of a batch); run without --gpus "
              "or with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_calib_mib:
        n = args.copy_calib_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    wl = workload(args.workload)
    khash = kernel_hash()
    log("workload:", wl["workload"])
    main_leg, xs32, out32 = leg(wl, wl["dtype"], "hybrid", args.steps, args.warmup)
    main_prof = main_leg.pop("stats")
    main_info = main_leg.pop("info")
    log("hybrid c64: %.4f ms, %.3e outputs/s, dominant %s" % (main_leg["ms"], main_leg["outputs_per_s"],
                                                               main_leg["dominant"]))
    compare = {}
    outs = {"c64": {"hybrid_c64": out32}}
    xs_by = {"c64": xs32}
    if not args.no_compare:
        sc = max(10, args.steps // 4)

        def run(name, fn):
            """One comparison leg; a failing leg is reported, not fatal."""
            try:
                return fn()
            except Exception as e:  # noqa: BLE001
                log("compare leg %s failed: %s" % (name, e))
                compare[name] = {"error": str(e)}
                return None

        def put(name, fn):
            r = run(name, fn)
            if r is not None:
                compare[name] = r[0] if isinstance(r, tuple) else r
            return r

        r = put("explicit_c64", lambda: explicit_best(wl, "c64", sc, 5))
        if r:
            outs["c64"]["explicit_c64"] = r[1]
        r = put("hybrid_c128", lambda: leg(wl, "c128", "hybrid", sc, 5))
        if r:
            outs["c128"] = {"hybrid_c128": r[2]}
            xs_by["c128"] = r[1]
        r = put("explicit_c128", lambda: explicit_best(wl, "c128", sc, 5))
        if r and "c128" in outs:
            outs["c128"]["explicit_c128"] = r[1]
        put("hybrid_c64_tuned", lambda: leg(wl, "c64", "hybrid", sc, 5, tuner="exhaustive"))
        put("hybrid_c128_tuned", lambda: leg(wl, "c128", "hybrid", sc, 5, tuner="exhaustive"))
        from paper_2303_17510_amd import tune as _tune
        have_model = os.path.exists(_tune.TRAINED_MODEL)
        if have_model:
            put("hybrid_c64_model", lambda: leg(wl, "c64", "hybrid", sc, 5, tuner="model"))
        if args.workload == "c2":
            w15 = workload("c2_1p5m")
            for dt in ("c64", "c128"):
                put("L1500000_hybrid_%s" % dt, lambda: leg(w15, dt, "hybrid", sc, 5))
                put("L1500000_hybrid_%s_tuned" % dt, lambda: leg(w15, dt, "hybrid", sc, 5, tuner="exhaustive"))
                put("L1500000_explicit_%s" % dt, lambda: explicit_best(w15, dt, sc, 5))
            sb = max(10, args.steps // 10)
            put("batched_4096_c64", lambda: batched_leg(sb, 3))
            put("batched_4096_c64_tuned", lambda: batched_leg(sb, 3, tuner="exhaustive"))
            if have_model:
                put("L1500000_hybrid_c64_model", lambda: leg(w15, "c64", "hybrid", sc, 5, tuner="model"))
                put("batched_4096_c64_model", lambda: batched_leg(sb, 3, tuner="model"))
            put("C1_8192_copies_c128", lambda: batched_leg(sb, 3, dtype="c128", Ls=[1024] * 8192, config_id=0))
            # C1 itself: one L = 1024 convolution (latency-bound: a single workgroup), and
            # the same problem as 8192 copies of one plan (the problem descriptor's copies)
            w1 = {"workload": "1D complex conv, A=2, B=1, L=1024, M=2048, complex128, unit disk",
                  "L": [1024], "M": [2048], "A": 2, "dtype": "c128", "config_id": 0}
            put("C1_single_hybrid_c128", lambda: leg(w1, "c128", "hybrid", sc, 5))
            put("C1_single_explicit_c128", lambda: leg(w1, "c128", "explicit", sc, 5))
            put("C1_plan_8192_copies_c128", lambda: leg(dict(w1, copies=8192), "c128", "hybrid", sb, 3))
            # the 2D and 3D workloads, on the same GPU
            w4, w5 = workload("c4"), workload("c5_3d")
            for dt in ("c64", "c128"):
                put("C4_2048x2048_hybrid_%s" % dt, lambda: leg(w4, dt, "hybrid", 20, 3))
            put("C4_2048x2048_explicit_c64", lambda: leg(w4, "c64", "explicit", 10, 2))
            if have_model:
                put("C4_2048x2048_hybrid_c64_model", lambda: leg(w4, "c64", "hybrid", 20, 3, tuner="model"))
            put("C5_256cube_hybrid_c64", lambda: leg(w5, "c64", "hybrid", 30, 5))
            if have_model:
                put("C5_256cube_hybrid_c64_model", lambda: leg(w5, "c64", "hybrid", 30, 5, tuner="model"))
            # centered convolutions (padding 3L/2 per dimension)
            wc, wc4 = workload("c2_centered"), workload("c4_centered")
            for dt in ("c64", "c128"):
                put("centered_1M_hybrid_%s" % dt, lambda: leg(wc, dt, "hybrid", sc, 5))
                put("centered_1M_hybrid_%s_folded" % dt,
                    lambda: leg(wc, dt, "hybrid", sc, 5, m=4096, p=128, variant="multipass"))
                put("centered_1M_hybrid_%s_tuned" % dt, lambda: leg(wc, dt, "hybrid", sc, 5, tuner="exhaustive"))
                put("centered_1M_explicit_%s" % dt, lambda: explicit_best(wc, dt, sc, 5))
            put("centered_2048x2048_hybrid_c64", lambda: leg(wc4, "c64", "hybrid", 20, 3))
            put("centered_2048x2048_hybrid_c64_tuned", lambda: leg(wc4, "c64", "hybrid", 20, 3, tuner="exhaustive"))
            put("centered_2048x2048_explicit_c64", lambda: leg(wc4, "c64", "explicit", 10, 2))
            # Hermitian convolutions (half storage, M = 3L/2)
            wh = workload("c2_hermitian")
            for dt in ("c64", "c128"):
                put("hermitian_1M_hybrid_%s" % dt, lambda: leg(wh, dt, "hybrid", sc, 5))
                put("hermitian_1M_hybrid_%s_tuned" % dt, lambda: leg(wh, dt, "hybrid", sc, 5, tuner="exhaustive"))
                put("hermitian_1M_explicit_%s" % dt, lambda: explicit_best(wh, dt, sc, 5))
            # 3D cubes of incremental, mostly non-power-of-two extents (M = 2L):
            # hybrid against explicit padding to the next supported size
            sweep = {}
            for n in (96, 100, 127, 150, 181, 200, 229, 256):
                w3 = {"workload": "3D sweep", "L": [n] * 3, "M": [2 * n] * 3, "A": 2, "dtype": "c64",
                      "config_id": 4}
                h = run("sweep3d_%d" % n, lambda: leg(w3, "c64", "hybrid", 20, 5))
                x = run("sweep3d_%d_explicit" % n, lambda: leg(w3, "c64", "explicit", 3, 1))
                if h and x:
                    sweep[str(n)] = {"hybrid_ms": h[0]["ms"], "explicit_ms": x[0]["ms"],
                                     "speedup": x[0]["ms"] / h[0]["ms"],
                                     "ns_per_NlogN_hybrid": h[0]["ns_per_NlogN"]}
            compare["sweep3d_c64"] = sweep
            wh4 = workload("c4_hermitian")
            put("hermitian_2047x2048_hybrid_c64", lambda: leg(wh4, "c64", "hybrid", 20, 3))
            put("hermitian_2047x2048_hybrid_c64_tuned", lambda: leg(wh4, "c64", "hybrid", 20, 3, tuner="exhaustive"))
            put("hermitian_2047x2048_explicit_c64", lambda: leg(wh4, "c64", "explicit", 10, 2))
            # quadratic operators (Basdevant and MHD forms): one plan for all outputs against
            # the pairwise products it replaces (u^2, v^2, uv in 2D; six pairs in 3D; nine
            # pairs z+_i z-_j for MHD)
            for nm, wq, base, pairs in (("basdevant_2047x2048_hermitian_c64", workload("basdevant2d_hermitian"),
                                         "hermitian_2047x2048_hybrid_c64", 3),
                                        ("basdevant_256cube_c64", workload("basdevant3d"),
                                         "C5_256cube_hybrid_c64", 6),
                                        ("mhd_256cube_c64", workload("mhd3d"), "C5_256cube_hybrid_c64", 9)):
                r = put(nm, lambda: leg(wq, "c64", "hybrid", 10, 3))
                if r and "ms" in compare.get(base, {}):
                    compare[nm]["pairwise_products_ms"] = pairs * compare[base]["ms"]
                    compare[nm]["speedup_vs_pairwise"] = pairs * compare[base]["ms"] / compare[nm]["ms"]
        for v in compare.values():
            v.pop("stats", None)
            v.pop("info", None)
        for k, v in compare.items():
            if "error" in v or "ms" not in v:
                continue
            dom = v.get("dominant", {"kernel": "-", "frac": float("nan")})
            log("%-22s %.4f ms  %.3e outputs/s  dominant %s %.3f" % (k, v["ms"], v["outputs_per_s"],
                                                                     dom["kernel"], dom["frac"]))
    cpu = None
    errs = {}
    if not args.no_cpu:
        cpu, errs = cpu_baseline(wl, xs_by, outs, args.cpu_budget)
        log("cpu oracle:", cpu, "errors:", errs)

    dom = main_leg["dominant"]
    agg_bytes = None
    for k, v in main_leg["kernels"].items():
        if k == dom["kernel"]:
            agg_bytes = v["GBps"]
    achieved = agg_bytes
    traffic = read_traffic(dom["kernel"], args.workload, khash)
    dom_bytes = [v["bytes"] / v["launches"] for k, v in dominant(main_prof)[3].items() if k == dom["kernel"]][0]
    copy_gbps = copy_baseline(dom_bytes)
    flops = kernel_flops(dom["kernel"], main_info, wl["A"])
    alu = None
    if flops:
        tf = flops / (dom["avg_ms"] * 1e-3) / 1e12
        # FP32 vector peak 157.3 TFLOP/s counts packed FP32 instructions,
        # which the library's kernels are compiled without: 78.6 TFLOP/s without them
        pk = 157.3 if wl["dtype"] == "c64" else 78.6
        alu = {"achieved": tf, "peak": pk, "unit": "TFLOP/s", "frac": tf / pk,
               "peak_without_packed_fp32": 78.6, "flops_per_launch": flops}
    n_out = 1
    for l in wl["L"]:
        n_out *= l
    line = {
        "metric": METRIC,
        "value": main_leg["outputs_per_s"],
        "unit": "outputs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl["dtype"] == "c64" else "f64",
        "data": "synthetic (seeded, unit disk)",
        "config": {"workload": wl["workload"], "L": wl["L"], "M": wl["M"], "A": wl["A"], "B": 1,
                   "plan": main_leg["plan"], "kernel_src": khash},
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": traffic, "avg_ms": dom["avg_ms"], "bytes_per_launch": dom_bytes,
                     "copy_same_bytes_GBps": copy_gbps, "frac_of_copy": achieved / copy_gbps if achieved else None,
                     "alu": alu},
        "cpu_baseline": cpu,
        "err_rel_l2": errs,
        "compulsory_frac": main_leg["compulsory_frac"],
        "traffic_by_design_GBps": main_leg["traffic_by_design_GBps"],
        "kernels": main_leg["kernels"],
        "compare": compare,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
