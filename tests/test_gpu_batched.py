"""Batched plans: many independent convolutions of uneven length in one launch.

Every convolution of the batch is compared with the FP64 oracle; the graph
path (captured on the second execute) is replayed several times with eager
work in between and each replay is checked against the eager result.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_17510_amd import BatchPlan, Plan, synth

pytestmark = pytest.mark.gpu
TOL = {"c64": 1e-5, "c128": 1e-12}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def batch_case(Ls, dtype, seed, A=2, Ms=None):
    import torch
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = [[synth.unit_disk((L,), seed + 10 * i + a).astype(npdt) for a in range(A)] for i, L in enumerate(Ls)]
    ins = [[torch.from_numpy(x).cuda() for x in row] for row in xs]
    outs = [torch.full((L,), float("nan"), dtype=ins[0][0].dtype, device="cuda") for L in Ls]
    return xs, ins, outs


def check_all(xs, outs, dtype):
    worst = 0.0
    for row, o in zip(xs, outs):
        ins = [synth.as_oracle(x) for x in row]
        ref = oracle.conv_direct(ins) if ins[0].size <= 4096 else oracle.conv_explicit(ins)
        err = oracle.rel_l2(o.cpu().numpy(), ref)
        worst = max(worst, err)
    return worst


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_batched_mixed_lengths(gpu, dtype):
    import torch
    Ls = [int(v) for v in synth.batched_lengths(count=160, lo_log2=0.0, span_log2=15.0, seed=4242)]
    Ls += [1, 2, 3, 64, 8191, 8192, 8193, 65536]
    say("batch of", len(Ls), "lengths", min(Ls), "..", max(Ls))
    xs, ins, outs = batch_case(Ls, dtype, 500)
    with BatchPlan(Ls, dtype=dtype) as bp:
        say("groups", [(g["variant"], g["m"], g["p"], g["q"], g["count"]) for g in bp.groups()])
        bp.execute(ins, outs)
        torch.cuda.synchronize()
    worst = check_all(xs, outs, dtype)
    say("worst rel L2 %.3e" % worst)
    assert worst <= TOL[dtype]


def test_batched_graph_replays_match_eager(gpu):
    import torch
    Ls = [int(v) for v in synth.batched_lengths(count=64, lo_log2=4.0, span_log2=12.0, seed=77)]
    xs, ins, outs = batch_case(Ls, "c64", 900)
    eager = [torch.empty_like(o) for o in outs]
    with BatchPlan(Ls, dtype="c64", graph=False) as bp:
        bp.execute(ins, eager)
    torch.cuda.synchronize()
    with BatchPlan(Ls, dtype="c64", graph=True) as bp:
        for rep in range(4):   # first eager, second captures, then replays
            for o in outs:
                o.fill_(float("nan"))
            bp.execute(ins, outs)
            junk = torch.randn(1 << 16, device="cuda").sum()   # unrelated eager work
            torch.cuda.synchronize()
            assert float(junk) == float(junk)
            for a, b in zip(outs, eager):
                assert torch.equal(a, b), "replay %d differs from eager" % rep


def test_batched_same_as_single_plans(gpu):
    import torch
    Ls = [100, 1000, 5000, 20000, 70000]
    xs, ins, outs = batch_case(Ls, "c128", 1300)
    with BatchPlan(Ls, dtype="c128") as bp:
        bp.execute(ins, outs)
    torch.cuda.synchronize()
    for i, L in enumerate(Ls):
        with Plan((L,), (2 * L,), dtype="c128") as p:
            single = p(*ins[i])
            torch.cuda.synchronize()
        assert oracle.rel_l2(outs[i].cpu().numpy(), single.cpu().numpy()) <= 1e-13


def test_batched_pointer_change_between_executes(gpu):
    import torch
    Ls = [50, 700, 9000]
    xs1, ins1, outs1 = batch_case(Ls, "c64", 1)
    xs2, ins2, outs2 = batch_case(Ls, "c64", 2)
    with BatchPlan(Ls, dtype="c64") as bp:
        for _ in range(3):
            bp.execute(ins1, outs1)
            bp.execute(ins2, outs2)
        torch.cuda.synchronize()
    assert check_all(xs1, outs1, "c64") <= 1e-5
    assert check_all(xs2, outs2, "c64") <= 1e-5


def _batch_ms(bp, ins, outs, reps=10):
    import torch
    bp.execute(ins, outs)
    bp.execute(ins, outs)   # captured
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        bp.execute(ins, outs)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return sorted(ts)[len(ts) // 2]


def test_batched_tuned_per_bucket(gpu):
    """Exhaustive per-group tuning: results stay exact, and the tuned batch is
    not slower than the heuristic grouped one (each group's default is a
    candidate; tuning applies to the grouped form)."""
    import torch
    Ls = [int(v) for v in synth.batched_lengths(count=96, lo_log2=6.0, span_log2=10.0, seed=31337)]
    xs, ins, outs = batch_case(Ls, "c64", 2100)
    with BatchPlan(Ls, dtype="c64", grouped=True) as bp:
        t_heur = _batch_ms(bp, ins, outs)
        ng_heur = len(bp.groups())
    with BatchPlan(Ls, dtype="c64") as bp:
        t_persist = _batch_ms(bp, ins, outs)
    for o in outs:
        o.fill_(float("nan"))
    with BatchPlan(Ls, dtype="c64", tuner="exhaustive", tune_reps=3) as bp:
        groups = bp.groups()
        say("tuned groups", [(g["variant"], g["m"], g["p"], g["rows_per_block"], g["count"]) for g in groups])
        assert sum(g["count"] for g in groups) == len(Ls)
        t_tuned = _batch_ms(bp, ins, outs)
        torch.cuda.synchronize()
    worst = check_all(xs, outs, "c64")
    say("groups %d -> %d, heuristic %.3f ms, tuned %.3f ms (persistent %.3f ms), worst rel L2 %.3e" % (
        ng_heur, len(groups), t_heur, t_tuned, t_persist, worst))
    assert worst <= TOL["c64"]
    assert t_tuned <= 1.15 * t_heur


@pytest.mark.parametrize("tuner", ["heuristic", "exhaustive"])
def test_batched_benchmark_workload(gpu, tuner):
    # the benchmark's batch itself: 4096 complex64 convolutions, L
    # log-uniform in [64, 65536] from its seed, M = 2L, inputs from the
    # benchmark's generator; every convolution against the oracle
    import torch
    Ls = [int(v) for v in synth.batched_lengths()]
    assert len(Ls) == 4096
    xs = synth.batched_inputs(Ls, 2, 2, dtype=np.complex64)
    big = [torch.from_numpy(x).cuda() for x in xs]
    out_big = torch.full_like(big[0], float("nan"))
    offs = np.concatenate([[0], np.cumsum(Ls)])
    ins = [[big[a][offs[i]:offs[i + 1]] for a in range(2)] for i in range(len(Ls))]
    outs = [out_big[offs[i]:offs[i + 1]] for i in range(len(Ls))]
    with BatchPlan(Ls, dtype="c64", tuner=tuner) as bp:
        say("groups", [(g["variant"], g["m"], g["p"], g["q"], g["count"]) for g in bp.groups()])
        bound = bp.bind(ins, outs)
        for _ in range(3):   # eager, capture, replay: the bench times replays
            bound.execute()
        torch.cuda.synchronize()
    o = out_big.cpu().numpy()
    worst = 0.0
    for i in range(len(Ls)):
        a, b = offs[i], offs[i + 1]
        ref = oracle.conv_explicit([synth.as_oracle(xs[0][a:b]), synth.as_oracle(xs[1][a:b])])
        worst = max(worst, oracle.rel_l2(o[a:b], ref))
    say("4096-convolution batch (%s): worst rel L2 %.3e" % (tuner, worst))
    assert worst <= TOL["c64"]
