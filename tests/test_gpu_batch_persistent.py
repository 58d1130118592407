"""The persistent form of batched plans: one launch over a device task queue.

Every convolution is compared with the FP64 oracle.  The launch clears its
own queue head and dependency counters, so replays (eager and captured) are
run back to back, with eager work in between, and each is checked against the
first result bit for bit (every output is computed by one workgroup in a
fixed order, whatever the schedule).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_17510_amd import BatchPlan, synth

pytestmark = pytest.mark.gpu
TOL = {"c64": 1e-5, "c128": 1e-12}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def batch_case(Ls, dtype, seed, A=2):
    import torch
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = [[synth.unit_disk((L,), seed + 10 * i + a).astype(npdt) for a in range(A)] for i, L in enumerate(Ls)]
    ins = [[torch.from_numpy(x).cuda() for x in row] for row in xs]
    outs = [torch.full((L,), float("nan"), dtype=ins[0][0].dtype, device="cuda") for L in Ls]
    return xs, ins, outs


def worst_error(xs, outs, Ms=None):
    worst = 0.0
    for i, (row, o) in enumerate(zip(xs, outs)):
        ins = [synth.as_oracle(x) for x in row]
        ref = oracle.conv_direct(ins) if ins[0].size <= 4096 else oracle.conv_explicit(ins)
        worst = max(worst, oracle.rel_l2(o.cpu().numpy(), ref))
    return worst


def describe(bp):
    st = bp.stats()
    say("   stats", st, "groups", [(g["variant"], g["m"], g["p"], g["q"], g["count"]) for g in bp.groups()])
    return st


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_persistent_matches_oracle_and_grouped(gpu, dtype):
    # lengths across every compiled body: whole rows of 64 .. 2048 points
    # (1024 in complex128) and the inner form with p = 2 .. 64 (and 12 .. 96)
    import torch
    top = 17.0 if dtype == "c64" else 16.0  # longest compiled lengths: 2^17 (complex64), 2^16 (complex128)
    Ls = [int(v) for v in synth.batched_lengths(count=120, lo_log2=0.0, span_log2=top, seed=2303)]
    Ls += [1, 2, 63, 64, 65, 1024, 1025, 2048, 2049, 4096, 4097, 65536, 65537 if dtype == "c64" else 65536]
    if dtype == "c64":  # columns of p = 12, 24, 48, 96 points (3 * 2^k), up to the longest, 96 * 2048
        Ls += [20000, 40000, 90000, 150000, 96 * 2048]
    say("case persistent", dtype, len(Ls), "lengths", min(Ls), "..", max(Ls))
    xs, ins, outs = batch_case(Ls, dtype, 900)
    with BatchPlan(Ls, dtype=dtype) as bp:
        assert describe(bp)["persistent"]
        bp.execute(ins, outs)
        torch.cuda.synchronize()
    e = worst_error(xs, outs)
    say("   persistent worst rel L2 %.3e" % e)
    assert e <= TOL[dtype]
    outs2 = [torch.full_like(o, float("nan")) for o in outs]
    with BatchPlan(Ls, dtype=dtype, grouped=True) as bp:
        assert not describe(bp)["persistent"]
        bp.execute(ins, outs2)
        torch.cuda.synchronize()
    worst = max(oracle.rel_l2(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(outs, outs2))
    say("   persistent vs grouped worst %.3e" % worst)
    assert worst <= 2 * TOL[dtype]


def test_persistent_replays_are_identical(gpu):
    # eager executes and graph replays, with eager work between them
    import torch
    Ls = [int(v) for v in synth.batched_lengths(count=300, lo_log2=6.0, span_log2=11.0, seed=99)]
    say("case replays", len(Ls))
    xs, ins, outs = batch_case(Ls, "c64", 1200)
    with BatchPlan(Ls, dtype="c64") as bp:
        describe(bp)
        bound = bp.bind(ins, outs)
        bound.execute()  # eager
        torch.cuda.synchronize()
        first = [o.clone() for o in outs]
        for r in range(5):  # the second execute captures, the rest replay
            for o in outs:
                o.fill_(float("nan"))
            junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
            bound.execute()
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            for a, b in zip(first, outs):
                assert torch.equal(a, b), "replay %d differs" % r
    e = worst_error(xs, first)
    say("   worst rel L2 %.3e" % e)
    assert e <= TOL["c64"]


def test_persistent_three_inputs_and_wide_padding(gpu):
    # A = 3 with M = 3L - 2, and A = 2 with M = 5L (more residues per row)
    import torch
    Ls = [int(v) for v in synth.batched_lengths(count=60, lo_log2=2.0, span_log2=14.0, seed=5)]
    say("case A=3", len(Ls))
    xs, ins, outs = batch_case(Ls, "c64", 40, A=3)
    with BatchPlan(Ls, A=3, dtype="c64") as bp:
        assert describe(bp)["persistent"]
        bp.execute(ins, outs)
        torch.cuda.synchronize()
    e = worst_error(xs, outs)
    say("   A=3 worst rel L2 %.3e" % e)
    assert e <= TOL["c64"]
    say("case M=5L")
    xs, ins, outs = batch_case(Ls, "c64", 41)
    Ms = [5 * L for L in Ls]
    with BatchPlan(Ls, Ms, dtype="c64") as bp:
        describe(bp)
        bp.execute(ins, outs)
        torch.cuda.synchronize()
    e = worst_error(xs, outs)
    say("   M=5L worst rel L2 %.3e" % e)
    assert e <= TOL["c64"]


def test_persistent_pointer_change_and_single(gpu):
    # new output tensors between executes (the task table is uploaded again),
    # then the same pointers (no upload); and a batch of one convolution
    import torch
    Ls = [3000, 70000, 129, 20000]
    xs, ins, outs = batch_case(Ls, "c64", 77)
    with BatchPlan(Ls, dtype="c64") as bp:
        describe(bp)
        bp.execute(ins, outs)
        outs_b = [torch.full_like(o, float("nan")) for o in outs]
        bp.execute(ins, outs_b)
        bp.execute(ins, outs_b)
    for a, b in zip(outs, outs_b):
        assert torch.equal(a, b)
    assert worst_error(xs, outs) <= TOL["c64"]
    for L in (1, 5000):
        xs, ins, outs = batch_case([L], "c128", 3)
        with BatchPlan([L], dtype="c128") as bp:
            assert describe(bp)["persistent"]
            bp.execute(ins, outs)
        assert worst_error(xs, outs) <= TOL["c128"]
