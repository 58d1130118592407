#!/usr/bin/env python3
"""Throughput of hybrid-dealiased complex convolution on one MI355X.

Headline workload: the 3D complex convolution of two 256^3 complex64 arrays
padded to 512^3 (A = 2 inputs, B = 1 output, entries uniform in the unit
disk from a fixed seed), hybrid dealiasing as planned by libhdconv (Sec. 5
decomposition).  A step is one hdconv_execute over inputs resident in HBM.

The last stdout line is ONE compact JSON object: outputs/s (value), the
roofline of the step's dominant kernel (algorithmic bytes per launch / its
average HIP-event duration, against the 8 TB/s HBM peak), the FP64 CPU oracle
timed on the host cores (a baseline), the error against that oracle, and one
short entry per comparison leg on the same GPU (explicit padding, FP64, the
1D, batched, 2D and other workloads).  The full comparison record goes to
gpurun_out/bench_compare.json and one stderr line per leg.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "conv outputs/s + %HBM roofline: hybrid vs explicit pad, FP32 vs FP64 (err≤1e-5)"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed FP32 instructions (the build keeps them out):
# 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
ALU_PEAK_F32 = 78.6
ALU_PEAK_F64 = 78.6
# sources that decide the kernels a plan runs and their code (the counter
# summaries under profiles/ record the hash of these)
KERNEL_SOURCES = ["hd_k_fused.hip", "hd_k_lean.hip", "hd_k_multi.hip", "hd_k_outer.hip", "hd_k_batch.hip",
                  "hd_kcommon.hpp", "hd_lean.hpp", "hd_fft.hpp", "hd_common.hpp", "hd_engine.hpp", "hd_plan.cpp"]
COMPARE_OUT = os.path.join(ROOT, "gpurun_out", "bench_compare.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2303_17510_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Basdevant forms of the Navier-Stokes nonlinearity (coefficients c[b][i][j], i <= j)
BASDEVANT_2D = [[[1, 0], [0, -1]], [[0, 1], [0, 0]]]
BASDEVANT_3D = [[[1, 0, 0], [0, 0, 0], [0, 0, -1]], [[0, 0, 0], [0, 1, 0], [0, 0, -1]],
                [[0, 1, 0], [0, 0, 0], [0, 0, 0]], [[0, 0, 1], [0, 0, 0], [0, 0, 0]],
                [[0, 0, 0], [0, 0, 1], [0, 0, 0]]]


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


WORKLOADS = {
    "c5_3d": {"workload": "3D complex conv, A=2, B=1, 256^3, M=512^3, complex64, unit disk, hybrid",
              "L": [256] * 3, "M": [512] * 3, "A": 2, "dtype": "c64", "config_id": 4},
    "c2": {"workload": "1D complex conv, A=2, B=1, L=2^20, M=2^21, complex64, unit disk, hybrid",
           "L": [1 << 20], "M": [1 << 21], "A": 2, "dtype": "c64", "config_id": 1},
    "c2_1p5m": {"workload": "1D complex conv, A=2, B=1, L=1500000, M=2999999, complex64, unit disk, hybrid",
                "L": [1500000], "M": [2999999], "A": 2, "dtype": "c64", "config_id": 1},
    "c1": {"workload": "1D complex conv, A=2, B=1, L=1024, M=2048, complex128, unit disk",
           "L": [1024], "M": [2048], "A": 2, "dtype": "c128", "config_id": 0},
    "c4": {"workload": "2D complex conv, A=2, B=1, 2048x2048, M=4096x4096, complex64, Gaussian, hybrid",
           "L": [2048, 2048], "M": [4096, 4096], "A": 2, "dtype": "c64", "config_id": 3, "dist": "gauss"},
    "c2_centered": {"workload": "1D centered complex conv, A=2, B=1, L=2^20, M=3*2^19, complex64, unit disk",
                    "L": [1 << 20], "M": [3 << 19], "A": 2, "dtype": "c64", "config_id": 1, "centered": True},
    "c4_centered": {"workload": "2D centered complex conv, A=2, B=1, 2048x2048, M=3072x3072, complex64, Gaussian",
                    "L": [2048, 2048], "M": [3072, 3072], "A": 2, "dtype": "c64", "config_id": 3,
                    "dist": "gauss", "centered": True},
    "c2_hermitian": {"workload": "1D Hermitian complex conv, A=2, B=1, L=2^20 (2^19 stored), M=3*2^19, "
                                 "complex64, unit disk",
                     "L": [1 << 20], "M": [3 << 19], "A": 2, "dtype": "c64", "config_id": 1, "hermitian": True},
    "c4_hermitian": {"workload": "2D Hermitian complex conv, A=2, B=1, 2047x2048 (2047x1024 stored), "
                                 "M=3072x3072, complex64, Gaussian",
                     "L": [2047, 2048], "M": [3072, 3072], "A": 2, "dtype": "c64", "config_id": 3,
                     "dist": "gauss", "hermitian": True},
    "c5_hermitian": {"workload": "3D Hermitian complex conv, A=2, B=1, 255x255x256 (255x255x128 stored), "
                                 "M=384^3, complex64, unit disk",
                     "L": [255, 255, 256], "M": [384, 384, 384], "A": 2, "dtype": "c64", "config_id": 4,
                     "hermitian": True},
    "basdevant2d_hermitian": {"workload": "2D Hermitian quadratic conv (Basdevant: u^2-v^2, uv), A=2, B=2, "
                                          "2047x2048, M=3072^2, complex64, Gaussian",
                              "L": [2047, 2048], "M": [3072, 3072], "A": 2, "dtype": "c64", "config_id": 3,
                              "dist": "gauss", "hermitian": True, "B": 2, "coef": BASDEVANT_2D},
    "basdevant3d": {"workload": "3D quadratic conv (Basdevant, 5 outputs), A=3, B=5, 256^3, M=512^3, complex64",
                    "L": [256] * 3, "M": [512] * 3, "A": 3, "dtype": "c64", "config_id": 4, "B": 5,
                    "coef": BASDEVANT_3D},
    "mhd3d": {"workload": "3D quadratic conv (MHD, Elsasser form), A=6, B=8, 256^3, M=512^3, complex64",
              "L": [256] * 3, "M": [512] * 3, "A": 6, "dtype": "c64", "config_id": 4, "B": 8,
              "coef": mhd_coefficients()},
}


def n_outputs(wl) -> int:
    """Outputs of one step: prod(L) per output array (a Hermitian result of
    length L counts L outputs, half of them stored), all B arrays, all copies."""
    n = wl.get("B", 1) * wl.get("copies", 1)
    for v in wl["L"]:
        n *= v
    return n


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
    """ms per execute over `steps` back-to-back executes (events on the
    execute stream), then per-launch event statistics over `steps` more."""
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
    plan.profile_begin(steps)
    for _ in range(steps):
        plan.execute(dev, out)
    torch.cuda.synchronize()
    stats = plan.profile_end()
    return ms, stats, out


def aggregate(stats):
    """Per kernel name: summed time, launches and algorithmic bytes."""
    agg = {}
    for s in stats:
        a = agg.setdefault(s["name"], {"total_ms": 0.0, "launches": 0, "bytes": 0.0})
        a["total_ms"] += s["total_ms"]
        a["launches"] += s["launches"]
        a["bytes"] += s["bytes_per_launch"] * s["launches"]
    return agg


def dominant(agg):
    """The kernel with the largest total time per step."""
    name = max(agg, key=lambda k: agg[k]["total_ms"])
    a = agg[name]
    return name, a["total_ms"] / a["launches"], a["bytes"] / a["launches"]


def read_traffic(kernel: str, wlname: str, khash: str):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary of this workload, if it was taken on the current kernel sources."""
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


def plan_kwargs(wl, m=None, **extra):
    kw = dict(extra)
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
    return kw


def leg(wl, dtype, method, steps, warmup, tuner="heuristic", m=None, **plan_kw):
    """Time one plan of a workload; returns (record, host inputs, device output)."""
    from paper_2303_17510_amd import Plan
    xs, dev = make_inputs(wl, dtype)
    t0 = time.perf_counter()
    with Plan(tuple(wl["L"]), tuple(wl["M"]), A=wl["A"], dtype=dtype, method=method, tuner=tuner,
              **plan_kwargs(wl, m, **plan_kw)) as p:
        plan_s = time.perf_counter() - t0
        info = p.info()
        ms, stats, out = time_plan(p, dev, steps, warmup)
    agg = aggregate(stats)
    name, avg_ms, bpl = dominant(agg)
    n_out = n_outputs(wl)
    r = {"dtype": dtype, "method": method, "tuner": tuner, "plan_s": plan_s,
         "candidates": info.get("tuned_candidates"), "timed_candidates": info.get("timed_candidates"),
         "ms": ms, "outputs_per_s": n_out / (ms * 1e-3),
         "ns_per_NlogN": ms * 1e6 / (n_out * math.log2(max(2, n_out))),
         "plan": [(d["variant"], d["m"], d["p"], d["n"], d["q"], d["E_m"]) for d in info["dims"]],
         "launches": info["launches"],
         "design_bytes": info["traffic_bytes"], "compulsory_bytes": info["compulsory_bytes"],
         "design_frac": info["traffic_bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
         "compulsory_frac": info["compulsory_bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
         "dominant": {"kernel": name, "avg_ms": avg_ms, "bytes_per_launch": bpl,
                      "frac": bpl / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
         "kernels": {k: {"avg_ms": v["total_ms"] / v["launches"], "launches_per_step": v["launches"] / steps,
                         "GBps": (v["bytes"] / v["launches"]) / (v["total_ms"] / v["launches"] * 1e-3) / 1e9}
                     for k, v in agg.items()}}
    return r, xs, out, info


def explicit_best(wl, dtype, steps, warmup):
    """Explicit padding with the fastest split N' = p m among a few m (the
    baseline gets its own small search, as the hybrid plan gets the tuner)."""
    best = None
    cands = (None,) if len(wl["L"]) > 1 else (None, 2048, 4096, 8192)
    for m in cands:
        try:
            r = leg(wl, dtype, "explicit", steps, warmup, m=m)
        except Exception as e:  # noqa: BLE001  (a split the planner rejects)
            log("explicit split m=%s: %s" % (m, e))
            continue
        if best is None or r[0]["ms"] < best[0]["ms"]:
            best = r
    return best


def batched_leg(steps, warmup, dtype="c64", count=4096, tuner="heuristic", Ls=None, config_id=2, grouped=False):
    """Independent 1D convolutions in one graph launch: by default the 4096
    lengths L log-uniform in [64, 65536] (seeded), M = 2L.  The heuristic
    plan runs as one persistent kernel (``grouped``: per-group launches)."""
    import numpy as np
    import torch
    from paper_2303_17510_amd import BatchPlan, synth
    if Ls is None:
        Ls = [int(v) for v in synth.batched_lengths(count=count)]
    count = len(Ls)
    tot = sum(Ls)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = synth.batched_inputs(Ls, 2, config_id, dtype=npdt)
    big = [torch.from_numpy(x).cuda() for x in xs]
    out_big = torch.empty_like(big[0])
    offs = np.concatenate([[0], np.cumsum(Ls)])
    ins = [[big[a][offs[i]:offs[i + 1]] for a in range(2)] for i in range(count)]
    outs = [out_big[offs[i]:offs[i + 1]] for i in range(count)]
    t0 = time.perf_counter()
    with BatchPlan(Ls, dtype=dtype, tuner=tuner, grouped=grouped) as bp:
        plan_s = time.perf_counter() - t0
        groups = bp.groups()
        stats = bp.stats()
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
    form = "persistent kernel" if stats["persistent"] else "grouped launches"
    rec = {"dtype": dtype, "method": "hybrid, batched graph (%s)" % form, "tuner": tuner, "plan_s": plan_s,
           "persistent": stats["persistent"], "grid": stats["grid"], "tasks": stats["tasks"],
           "convolutions": count, "outputs": tot, "ms": ms, "outputs_per_s": tot / (ms * 1e-3),
           "compulsory_frac": 3 * w * tot / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "groups": [(g["variant"], g["m"], g["p"], g["q"], g["count"]) for g in groups]}
    return rec, xs, out_big, Ls


def oracle_ref(wl, xs):
    """FP64 oracle result of a workload (explicitly padded FFT convolution)."""
    import oracle
    from paper_2303_17510_amd import synth
    ins = [synth.as_oracle(x) for x in xs]
    if wl.get("hermitian"):
        return oracle.conv_hermitian_explicit(ins)
    if wl.get("centered"):
        return oracle.conv_centered_explicit(ins)
    return oracle.conv_explicit(ins)


def batched_error(xs, out, Ls):
    """Largest relative L2 error over the convolutions of a batched leg."""
    import numpy as np
    import oracle
    from paper_2303_17510_amd import synth
    o = out.cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(Ls)])
    worst = 0.0
    for i in range(len(Ls)):
        a, b = offs[i], offs[i + 1]
        ref = oracle.conv_explicit([synth.as_oracle(xs[0][a:b]), synth.as_oracle(xs[1][a:b])])
        worst = max(worst, oracle.rel_l2(o[a:b], ref))
    return worst


def copy_baseline(nbytes, reps=50):
    """GB/s of a plain device copy moving the same bytes (half read, half
    written) as one launch of the dominant kernel."""
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


def kernel_flops(name, info, A=2):
    """Algorithmic floating-point operations of one launch of a 1D plan's
    kernel: 5 N log2 N per N-point complex FFT, 6 per complex multiply."""
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
    return None


def row_flops(info, A=2):
    """Algorithmic flops of one launch of a 2D/3D plan's innermost whole-row
    pass: per row and residue, A forward and one inverse m-point FFT
    (5 m log2 m each), the residue twiddles (6 per point per input and on the
    output) and the product (6 per point per extra input)."""
    d = info["dims"][-1]
    if d["variant"] != "fused":
        return None
    m, q = d["m"], d["q"]
    rows = 1
    for e in info["dims"][:-1]:
        rows *= e["q"] * e["m"]
    per_res = (A + 1) * 5.0 * m * math.log2(m) + 6.0 * m * (A + 1) + 6.0 * m * (A - 1)
    return rows * q * per_res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c5_3d", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle (baseline and errors)")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison legs")
    ap.add_argument("--full", action="store_true", help="also the 3D size sweep and the quadratic operators")
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

    wl = WORKLOADS[args.workload]
    khash = kernel_hash()
    log("workload:", wl["workload"])
    main_rec, xs_main, out_main, main_info = leg(wl, wl["dtype"], "hybrid", args.steps, args.warmup)
    log("headline %s: %.4f ms, %.3e outputs/s, dominant %s" % (args.workload, main_rec["ms"],
                                                              main_rec["outputs_per_s"], main_rec["dominant"]))

    # comparison legs: (name, workload key or None, fn) -> (record, xs, out[, Ls])
    compare = {}
    refs = {}   # (workload, dtype) -> oracle result, computed once

    def ref_of(wkey, dtype, xs):
        if (wkey, dtype) not in refs:
            refs[(wkey, dtype)] = oracle_ref(WORKLOADS[wkey], xs)
        return refs[(wkey, dtype)]

    def put(name, wkey, fn):
        """Run one comparison leg; a failing leg is reported, not fatal."""
        try:
            r = fn()
        except Exception as e:  # noqa: BLE001
            log("leg %s failed: %s" % (name, e))
            compare[name] = {"error": str(e)}
            return None
        if r is None:
            return None
        rec = r[0]
        if not args.no_cpu and wkey is not None:
            try:
                if wkey == "batched":
                    rec["err_rel_l2_max"] = batched_error(r[1], r[2], r[3])
                else:
                    rec["err_rel_l2"] = oracle_ref_err(wkey, rec["dtype"], r[1], r[2])
            except Exception as e:  # noqa: BLE001
                rec["err_note"] = "oracle failed: %s" % e
        compare[name] = rec
        err = rec.get("err_rel_l2", rec.get("err_rel_l2_max", float("nan")))
        dom = rec.get("dominant", {})
        log("%-34s %9.4f ms  %.3e outputs/s  compulsory %.3f  dominant %s %.3f  err %.2e" % (
            name, rec["ms"], rec["outputs_per_s"], rec.get("compulsory_frac", float("nan")),
            dom.get("kernel", "-"), dom.get("frac", float("nan")), err))
        return r

    def oracle_ref_err(wkey, dtype, xs, out):
        import oracle
        o = out if isinstance(out, list) else [out]
        ref = ref_of(wkey, dtype, xs)
        return max(oracle.rel_l2(t.cpu().numpy(), ref) for t in o[:1])

    # the headline's own error and CPU baseline: one oracle run of the workload
    cpu = None
    err_main = None
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        ref = ref_of(args.workload, wl["dtype"], xs_main)
        cpu_s = time.perf_counter() - t0
        err_main = oracle.rel_l2(out_main.cpu().numpy(), ref)
        cpu = {"value": n_outputs(wl) / cpu_s, "unit": "outputs/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "one full run of the headline workload (%s) through the FP64 oracle's explicitly "
                         "zero-padded FFT convolution (own radix-2 FFT, OpenMP over transform lines), "
                         "%.1f s" % (wl["workload"].split(",")[0] + " " + "x".join(map(str, wl["L"])), cpu_s)}
        log("cpu oracle: %.3e outputs/s on %d threads (%.1f s); headline error %.3e" % (
            cpu["value"], cpu["cores"], cpu_s, err_main))

    if not args.no_compare:
        sc = 20
        put("explicit_c64", args.workload, lambda: explicit_best(wl, "c64", 10, 2))
        put("hybrid_c128", args.workload, lambda: leg(wl, "c128", "hybrid", sc, 3))
        put("explicit_c128", args.workload, lambda: explicit_best(wl, "c128", 5, 2))
        from paper_2303_17510_amd import tune as _tune
        have_model = os.path.exists(_tune.TRAINED_MODEL)
        if have_model:
            put("hybrid_c64_model", args.workload, lambda: leg(wl, "c64", "hybrid", sc, 3, tuner="model"))
        put("hybrid_c64_exhaustive", args.workload, lambda: leg(wl, "c64", "hybrid", sc, 3, tuner="exhaustive"))
        if args.workload == "c5_3d":
            put("herm3d_255x255x256_c64", "c5_hermitian", lambda: leg(WORKLOADS["c5_hermitian"], "c64", "hybrid",
                                                                      sc, 3))
            put("herm3d_255x255x256_explicit_c64", "c5_hermitian",
                lambda: leg(WORKLOADS["c5_hermitian"], "c64", "explicit", 5, 2))
            w2 = WORKLOADS["c2"]
            for dt in ("c64", "c128"):
                put("1d_2^20_hybrid_%s" % dt, "c2", lambda: leg(w2, dt, "hybrid", 100, 10))
                put("1d_2^20_explicit_%s" % dt, "c2", lambda: explicit_best(w2, dt, 50, 5))
            w15 = WORKLOADS["c2_1p5m"]
            for dt in ("c64", "c128"):
                put("1d_1.5M_hybrid_%s" % dt, "c2_1p5m", lambda: leg(w15, dt, "hybrid", 50, 5))
                put("1d_1.5M_explicit_%s" % dt, "c2_1p5m", lambda: explicit_best(w15, dt, 20, 5))
            put("batched_4096_c64", "batched", lambda: batched_leg(20, 3))
            put("batched_4096_c64_grouped", None, lambda: batched_leg(20, 3, grouped=True))
            put("batched_4096_c64_exhaustive", None, lambda: batched_leg(20, 3, tuner="exhaustive"))
            w1 = WORKLOADS["c1"]
            put("c1_single_hybrid_c128", "c1", lambda: leg(w1, "c128", "hybrid", 100, 10))
            put("c1_single_explicit_c128", "c1", lambda: leg(w1, "c128", "explicit", 100, 10))
            put("c1_8192_copies_c128", None, lambda: leg(dict(w1, copies=8192), "c128", "hybrid", 20, 3))
            w4 = WORKLOADS["c4"]
            for dt in ("c64", "c128"):
                put("2d_2048^2_hybrid_%s" % dt, "c4", lambda: leg(w4, dt, "hybrid", 20, 3))
            put("2d_2048^2_explicit_c64", "c4", lambda: leg(w4, "c64", "explicit", 10, 2))
            put("centered_1d_2^20_c64", "c2_centered", lambda: leg(WORKLOADS["c2_centered"], "c64", "hybrid",
                                                                   100, 10))
            put("centered_2d_2048^2_c64", "c4_centered", lambda: leg(WORKLOADS["c4_centered"], "c64", "hybrid",
                                                                     20, 3))
            put("hermitian_1d_2^20_c64", "c2_hermitian", lambda: leg(WORKLOADS["c2_hermitian"], "c64", "hybrid",
                                                                     100, 10))
            put("hermitian_2d_2047x2048_c64", "c4_hermitian",
                lambda: leg(WORKLOADS["c4_hermitian"], "c64", "hybrid", 20, 3))
        if args.full:
            sweep = {}
            for n in (96, 100, 127, 150, 181, 200, 229, 256):
                w3 = {"workload": "3D sweep", "L": [n] * 3, "M": [2 * n] * 3, "A": 2, "dtype": "c64",
                      "config_id": 4}
                try:
                    h = leg(w3, "c64", "hybrid", 20, 5)[0]
                    x = leg(w3, "c64", "explicit", 3, 1)[0]
                    sweep[str(n)] = {"hybrid_ms": h["ms"], "explicit_ms": x["ms"],
                                     "speedup": x["ms"] / h["ms"], "ns_per_NlogN_hybrid": h["ns_per_NlogN"]}
                    log("sweep %d: hybrid %.3f ms explicit %.3f ms" % (n, h["ms"], x["ms"]))
                except Exception as e:  # noqa: BLE001
                    sweep[str(n)] = {"error": str(e)}
            compare["sweep3d_c64"] = sweep
            for nm, wk in (("basdevant_2047x2048_hermitian_c64", "basdevant2d_hermitian"),
                           ("basdevant_256cube_c64", "basdevant3d"), ("mhd_256cube_c64", "mhd3d")):
                put(nm, None, lambda: leg(WORKLOADS[wk], "c64", "hybrid", 10, 3))

    # roofline of the headline step's dominant kernel
    dom = main_rec["dominant"]
    achieved = dom["bytes_per_launch"] / (dom["avg_ms"] * 1e-3) / 1e9
    traffic = read_traffic(dom["kernel"], args.workload, khash)
    copy_gbps = copy_baseline(dom["bytes_per_launch"])
    # vector-ALU rate of the whole-row pass (the step's arithmetic-bound kernel)
    alu = None
    row_k = next((k for k in ("rows_lean", "fused1d") if k in main_rec["kernels"]), None)
    flops = kernel_flops(dom["kernel"], main_info, wl["A"]) if len(wl["L"]) == 1 else (
        row_flops(main_info, wl["A"]) if row_k else None)
    if flops:
        k_ms = dom["avg_ms"] if len(wl["L"]) == 1 else main_rec["kernels"][row_k]["avg_ms"]
        tf = flops / (k_ms * 1e-3) / 1e12
        pk = ALU_PEAK_F32 if wl["dtype"] == "c64" else ALU_PEAK_F64
        alu = {"kernel": dom["kernel"] if len(wl["L"]) == 1 else row_k, "achieved": round(tf, 2), "peak": pk,
               "unit": "TFLOP/s", "frac": round(tf / pk, 3)}

    def short(rec):
        if "ms" not in rec:
            return {"error": rec.get("error", "?")[:80]}
        s = {"ms": round(rec["ms"], 4), "ops": float("%.4g" % rec["outputs_per_s"])}
        if "dominant" in rec:
            s["dom_frac"] = round(rec["dominant"]["frac"], 3)
        if "compulsory_frac" in rec:
            s["comp_frac"] = round(rec["compulsory_frac"], 3)
        for k in ("err_rel_l2", "err_rel_l2_max"):
            if k in rec:
                s["err"] = float("%.2e" % rec[k])
        return s

    line = {
        "metric": METRIC,
        "value": main_rec["outputs_per_s"],
        "unit": "outputs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_rec["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl["dtype"] == "c64" else "f64",
        "data": "synthetic (seeded, %s)" % ("Gaussian" if wl.get("dist") == "gauss" else "unit disk"),
        "config": {"workload": wl["workload"], "L": wl["L"], "M": wl["M"], "A": wl["A"], "B": wl.get("B", 1),
                   "plan": main_rec["plan"], "kernel_src": khash},
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "avg_ms": round(dom["avg_ms"], 5),
                     "bytes_per_launch": dom["bytes_per_launch"],
                     "copy_same_bytes_GBps": round(copy_gbps, 1), "alu_tflops": alu,
                     "step_design_frac": round(main_rec["design_frac"], 4),
                     "step_compulsory_frac": round(main_rec["compulsory_frac"], 4)},
        "kernels_ms": {k: round(v["avg_ms"], 4) for k, v in main_rec["kernels"].items()},
        "cpu_baseline": cpu,
        "err_rel_l2": err_main,
        "legs": {k: short(v) for k, v in compare.items() if isinstance(v, dict) and ("ms" in v or "error" in v)},
    }
    try:
        os.makedirs(os.path.dirname(COMPARE_OUT), exist_ok=True)
        with open(COMPARE_OUT, "w") as fh:
            json.dump({"headline": main_rec, "compare": compare, "line": line}, fh, indent=1, default=str)
    except OSError as e:
        log("could not write %s: %s" % (COMPARE_OUT, e))
    print(json.dumps(line, separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
