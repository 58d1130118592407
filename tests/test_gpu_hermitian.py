"""GPU parity of Hermitian convolutions against the FP64 CPU oracle.

Hermitian plans (the paper's Hermitian symmetric case, one dimension) take
the ceil(L/2) stored non-negative indices of each input and return those of
the output.  The cases run through the C ABI and are compared element by
element with the oracle's Hermitian convolution (conjugate-mirror expansion,
then the centered direct sums, or its explicit FFT form for large sizes):
relative L2 <= 1e-12 for complex128 and <= 1e-5 for complex64.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_17510_amd import BatchPlan, Plan, synth
from paper_2303_17510_amd.hdconv import hermitian_min_padding

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(Lh, A, dtype, seed):
    import torch
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = [synth.unit_disk((Lh,), 7300 + seed + a).astype(npdt) for a in range(A)]
    return xs, [torch.from_numpy(x).cuda() for x in xs]


def reference(xs, direct_max=20000):
    ins = [synth.as_oracle(x) for x in xs]
    if ins[0].size <= direct_max:
        return oracle.conv_hermitian_direct(ins)
    return oracle.conv_hermitian_explicit(ins)


def run(plan, dev):
    import torch
    out = torch.empty_like(dev[0])
    plan.execute(dev, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(L, dtype, A=2, M=None, seed=0, **kw):
    M = hermitian_min_padding(L, A) if M is None else M
    Lh = (L + 1) // 2
    say("hermitian case", L, M, dtype, "A=%d" % A, kw)
    xs, dev = make_inputs(Lh, A, dtype, seed)
    with Plan((L,), (M,), A=A, dtype=dtype, hermitian=True, **kw) as p:
        info = p.info()
        got = run(p, dev)
    want = reference(xs)
    err = oracle.rel_l2(got, want)
    d = info["dims"][0]
    say("   ->", (d["variant"], d["m"], d["p"], d["q"], d["D"]), "err=%.3e" % err)
    assert got.shape == (Lh,) and np.all(np.isfinite(got))
    assert err <= TOL[dtype], "rel L2 %.3e" % err
    return got, info


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L", [1, 2, 3, 8, 101, 1024, 4096, 8193, 65536])
def test_hermitian_default(gpu, dtype, L):
    _, info = check(L, dtype)
    assert info["dims"][0]["hermitian"]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("m", [1024, 1536, 2048, 3072, 4096])
def test_hermitian_direct_form_every_m(gpu, dtype, m):
    # L = 2048: 1024 stored entries, full centered length 2047, M = 3070
    _, info = check(2048, dtype, m=m, variant="fused")
    d = info["dims"][0]
    assert (d["m"], d["p"]) == (m, 2)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,m,p,D", [
    (2000, 32, 32, 0),   # folded: the 64-block span on 32 column positions
    (2000, 32, 64, 0),   # unfolded
    (2000, 16, 96, 0),   # folded, p = 3 * 32 (span 126)
    (2001, 32, 32, 1),   # folded, one residue per block: FP64 accumulator
])
def test_hermitian_inner_form(gpu, dtype, L, m, p, D):
    _, info = check(L, dtype, m=m, p=p, D=D or None, variant="multipass")
    assert info["dims"][0]["p"] == p


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L", [9, 600, 3001])
def test_hermitian_three_inputs(gpu, dtype, L):
    check(L, dtype, A=3)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("kw", [{}, {"m": 4096, "p": 384, "variant": "multipass"}])
def test_hermitian_1m(gpu, dtype, kw):
    # L = 2^20 with the paper's Hermitian benchmark padding M = 3L/2
    L = 1 << 20
    Lh = L // 2
    xs, dev = make_inputs(Lh, 2, dtype, 3)
    with Plan((L,), (3 << 19,), dtype=dtype, hermitian=True, **kw) as p:
        d = p.info()["dims"][0]
        got = run(p, dev)
    ins = [synth.as_oracle(x) for x in xs]
    rng = np.random.default_rng(13)
    idx = np.unique(np.concatenate([[0, 1, Lh - 2, Lh - 1], rng.integers(0, Lh, 60)]))
    err = oracle.rel_l2(got[idx], oracle.conv_hermitian_direct(ins, idx=idx))
    say("   1M hermitian", kw, (d["m"], d["p"], d["n"], d["q"]), "sampled err=%.3e" % err)
    assert err <= TOL[dtype]
    assert oracle.rel_l2(got, oracle.conv_hermitian_explicit(ins)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L", [1, 100, 1024, 5001])
def test_hermitian_explicit_method(gpu, dtype, L):
    _, info = check(L, dtype, method="explicit")
    assert info["method"] == "explicit"


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_hermitian_centre_and_real_output_centre(gpu, dtype):
    import torch
    L = 3000
    Lh = (L + 1) // 2
    xs, dev = make_inputs(Lh, 2, dtype, 7)
    with Plan((L,), dtype=dtype, hermitian=True) as p:
        a = run(p, dev)
        # the imaginary part of a stored centre is ignored
        dev2 = [t.clone() for t in dev]
        dev2[0][0] = dev2[0][0] + 3j
        b = run(p, dev2)
    tol = TOL[dtype]
    assert oracle.rel_l2(b, a) <= tol
    assert abs(a[0].imag) <= 10 * tol * np.linalg.norm(a) / np.sqrt(Lh)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_hermitian_batched(gpu, dtype):
    import torch
    rng = np.random.default_rng(23)
    Ls = [int(v) for v in np.concatenate([[1, 2, 3, 2048, 3000], rng.integers(1, 12000, 30), [40000, 140000]])]
    say("hermitian batched", dtype, len(Ls), "convolutions")
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = [[synth.unit_disk(((L + 1) // 2,), 8500 + 2 * i + a).astype(npdt) for a in range(2)]
          for i, L in enumerate(Ls)]
    ins = [[torch.from_numpy(x).cuda() for x in pair] for pair in xs]
    outs = [torch.empty_like(pair[0]) for pair in ins]
    wants = [reference(pair) for pair in xs]
    with BatchPlan(Ls, dtype=dtype, hermitian=True) as bp:
        assert all(g["hermitian"] for g in bp.groups())
        for _ in range(3):  # eager, captured, replayed
            for o in outs:
                o.zero_()
            bp.execute(ins, outs)
            torch.cuda.synchronize()
            for i, L in enumerate(Ls):
                err = oracle.rel_l2(outs[i].cpu().numpy(), wants[i])
                assert err <= TOL[dtype], (i, L, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape,kw", [
    ((1, 5), {}), ((33, 64), {}), ((33, 63), {}), ((255, 512), {}), ((7, 3000), {"m": (0, 64), "variant": ("outer", "multipass")}),
    ((9, 11, 20), {}), ((31, 31, 31), {}),
    # 128 outer lines x 96 rows per line: the FP32 row pass pairs its rows too
    ((65, 4000), {"m": (0, 64), "variant": ("outer", "multipass")}),
    ((33, 64), {"method": "explicit"}), ((9, 11, 20), {"method": "explicit"}),
])
def test_hermitian_multidim(gpu, dtype, shape, kw):
    # outer dimensions centered (odd extents), the last one Hermitian
    import torch
    say("hermitian nd case", shape, dtype, kw)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    with Plan(shape, dtype=dtype, hermitian=True, **kw) as p:
        io = p.io_shape
        xs = [synth.unit_disk(io, 7400 + a).astype(npdt) for a in range(2)]
        dev = [torch.from_numpy(x).cuda() for x in xs]
        info = p.info()
        got = run(p, dev)
    ins = [synth.as_oracle(x) for x in xs]
    want = oracle.conv_hermitian_direct(ins) if np.prod(io) <= 6000 else oracle.conv_hermitian_explicit(ins)
    err = oracle.rel_l2(got, want)
    say("   ->", [(d["variant"], d["m"], d["p"], d["q"]) for d in info["dims"]], "err=%.3e" % err)
    assert got.shape == io and err <= TOL[dtype]


def test_hermitian_2d_tuned(gpu):
    import torch
    shape = (65, 128)
    with Plan(shape, dtype="c64", hermitian=True, tuner="exhaustive", tune_reps=2) as p:
        xs = [synth.unit_disk(p.io_shape, 7500 + a).astype(np.complex64) for a in range(2)]
        got = run(p, [torch.from_numpy(x).cuda() for x in xs])
        assert p.info()["timed_candidates"] > 1
    want = oracle.conv_hermitian_explicit([synth.as_oracle(x) for x in xs])
    assert oracle.rel_l2(got, want) <= TOL["c64"]


@pytest.mark.parametrize("tuner", ["exhaustive", "model"])
def test_hermitian_and_centered_tuned_batches(gpu, tuner):
    # batched plans tune per size bucket with the centered / Hermitian flag
    import torch
    rng = np.random.default_rng(29)
    Ls = [int(v) for v in rng.integers(50, 5000, 24)]
    for flag in ("centered", "hermitian"):
        io = [((L + 1) // 2 if flag == "hermitian" else L) for L in Ls]
        xs = [[synth.unit_disk((n,), 8700 + 2 * i + a).astype(np.complex64) for a in range(2)]
              for i, n in enumerate(io)]
        ins = [[torch.from_numpy(x).cuda() for x in pair] for pair in xs]
        outs = [torch.empty_like(pair[0]) for pair in ins]
        with BatchPlan(Ls, dtype="c64", tuner=tuner, tune_reps=2, **{flag: True}) as bp:
            bp.execute(ins, outs)
            torch.cuda.synchronize()
        for i in range(len(Ls)):
            o = [synth.as_oracle(x) for x in xs[i]]
            want = oracle.conv_hermitian_direct(o) if flag == "hermitian" else oracle.conv_centered_direct(o)
            assert oracle.rel_l2(outs[i].cpu().numpy(), want) <= TOL["c64"], (flag, i)


def test_hermitian_model_tuned_plan(gpu):
    _, info = check(1 << 16, "c64", tuner="model")
    assert info["tuner"] == "model"
