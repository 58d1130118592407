"""GPU parity of centered convolutions against the FP64 CPU oracle.

Centered plans (the paper's centered case: indices -H .. L-1-H with
H = floor(L/2) stored at positions c + H, padding down to 3L/2 for A = 2)
run through the C ABI on seeded inputs and are compared element by element
with the oracle's centered direct sums (or its windowed explicit FFT
convolution for large sizes, and sampled direct sums at the largest):
relative L2 <= 1e-12 for complex128 and <= 1e-5 for complex64.  The cases
cover the direct form (p = 2, residue counts 1 to 3), the inner form with
and without folding of the negative blocks onto the positive ones, residue
blocks with the FP64 accumulator, three inputs, 2D/3D, the explicit method,
batched plans of uneven lengths and a tuned plan.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_17510_amd import BatchPlan, Plan, synth
from paper_2303_17510_amd.hdconv import centered_min_padding

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(shape, A, dtype, seed):
    import torch
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = [synth.unit_disk(shape, 7100 + seed + a).astype(npdt) for a in range(A)]
    return xs, [torch.from_numpy(x).cuda() for x in xs]


def reference(xs, direct_max=20000):
    ins = [synth.as_oracle(x) for x in xs]
    if ins[0].size <= direct_max:
        return oracle.conv_centered_direct(ins)
    return oracle.conv_centered_explicit(ins)


def run(plan, dev):
    import torch
    out = torch.empty_like(dev[0])
    plan.execute(dev, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(shape, dtype, A=2, M=None, seed=0, ref=None, **kw):
    shape = tuple(shape)
    if M is None:
        M = tuple(centered_min_padding(n, A) for n in shape)
    say("centered case", shape, M, dtype, "A=%d" % A, kw)
    xs, dev = make_inputs(shape, A, dtype, seed)
    with Plan(shape, M, A=A, dtype=dtype, centered=True, **kw) as p:
        info = p.info()
        got = run(p, dev)
    want = reference(xs) if ref is None else ref(xs)
    err = oracle.rel_l2(got, want)
    say("   ->", [(d["variant"], d["m"], d["p"], d["q"], d["D"]) for d in info["dims"]], "err=%.3e" % err)
    assert np.all(np.isfinite(got))
    assert err <= TOL[dtype], "rel L2 %.3e" % err
    return got, info


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L", [1, 2, 3, 7, 100, 1000, 1023, 1024, 4096, 8192])
def test_centered_1d_default(gpu, dtype, L):
    _, info = check((L,), dtype)
    d = info["dims"][0]
    assert d["centered"]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("m", [512, 768, 1024, 1536, 2048])
def test_centered_direct_form_every_m(gpu, dtype, m):
    # L = 1024, M = 3L/2: p = 2 throughout, q = ceil(1536/m) = 3, 2, 2, 1, 1
    _, info = check((1024,), dtype, m=m, variant="fused")
    d = info["dims"][0]
    assert (d["m"], d["p"], d["q"]) == (m, 2, -(-1536 // m))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L", [10, 301, 2000])
def test_centered_three_inputs(gpu, dtype, L):
    check((L,), dtype, A=3)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,m,p,D", [
    (1000, 32, 16, 0),    # folded: 16 blocks of the 32-block span share positions
    (1000, 32, 32, 0),    # unfolded, p = span
    (1024, 64, 24, 0),    # unfolded, p = 3 * 8 above the span
    (1001, 16, 48, 0),    # odd L, folded (span 64)
    (1000, 16, 32, 1),    # folded, one residue per block: FP64 accumulator
    (777, 16, 32, 2),
])
def test_centered_inner_form(gpu, dtype, L, m, p, D):
    _, info = check((L,), dtype, m=m, p=p, D=D or None, variant="multipass")
    d = info["dims"][0]
    assert d["variant"] == "multipass" and d["m"] == m and d["p"] == p


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L", [16384, 65536, 100000])
def test_centered_inner_form_default(gpu, dtype, L):
    _, info = check((L,), dtype)
    assert info["dims"][0]["variant"] == "multipass"


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("kw", [{}, {"m": 4096, "p": 128, "variant": "multipass"}])
def test_centered_1m_sampled(gpu, dtype, kw):
    # L = 2^20, M = 3 * 2^19: the default plan (p = 384, one residue block)
    # and the folded plan of the paper's centered inner form (p = 128, n = 3)
    L = 1 << 20
    xs, dev = make_inputs((L,), 2, dtype, 5)
    with Plan((L,), (3 << 19,), dtype=dtype, centered=True, **kw) as p:
        info = p.info()
        got = run(p, dev)
    d = info["dims"][0]
    assert d["q"] * d["m"] == 3 << 19
    rng = np.random.default_rng(11)
    idx = np.unique(np.concatenate([[0, 1, L // 2 - 1, L // 2, L // 2 + 1, L - 2, L - 1],
                                    rng.integers(0, L, 57)]))
    ins = [synth.as_oracle(x) for x in xs]
    want = oracle.conv_centered_direct(ins, idx=idx)
    err = oracle.rel_l2(got[idx], want)
    say("   1M centered", kw, (d["m"], d["p"], d["n"], d["q"]), "sampled err=%.3e" % err)
    assert err <= TOL[dtype]
    full = oracle.conv_centered_explicit(ins)
    assert oracle.rel_l2(got, full) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(1, 1), (4, 4), (16, 16), (33, 47), (100, 7), (256, 256)])
def test_centered_2d(gpu, dtype, shape):
    check(shape, dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(2, 3, 4), (8, 12, 10), (16, 16, 16), (32, 32, 32)])
def test_centered_3d(gpu, dtype, shape):
    check(shape, dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_centered_2d_inner_rows(gpu, dtype):
    check((6, 3000), dtype, m=(0, 64), variant=("outer", "multipass"))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(1000,), (1024,), (33, 47), (9, 10, 11)])
def test_centered_explicit_method(gpu, dtype, shape):
    check(shape, dtype, method="explicit")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_centered_batched(gpu, dtype):
    import torch
    rng = np.random.default_rng(21)
    Ls = [int(v) for v in np.concatenate([[1, 2, 3, 1024, 1536], rng.integers(1, 6000, 40), [20000, 70000]])]
    say("centered batched", dtype, len(Ls), "convolutions")
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = [[synth.unit_disk((L,), 8300 + 2 * i + a).astype(npdt) for a in range(2)] for i, L in enumerate(Ls)]
    ins = [[torch.from_numpy(x).cuda() for x in pair] for pair in xs]
    outs = [torch.empty_like(pair[0]) for pair in ins]
    wants = [reference(pair) for pair in xs]
    with BatchPlan(Ls, dtype=dtype, centered=True) as bp:
        assert all(g["centered"] for g in bp.groups())
        for _ in range(3):  # eager, captured, replayed
            for o in outs:
                o.zero_()
            bp.execute(ins, outs)
            torch.cuda.synchronize()
            for i, L in enumerate(Ls):
                err = oracle.rel_l2(outs[i].cpu().numpy(), wants[i])
                assert err <= TOL[dtype], (i, L, err)


def test_centered_tuned_plan(gpu):
    _, info = check((3000,), "c64", tuner="exhaustive", tune_reps=2)
    assert info["tuner"] == "exhaustive" and info["timed_candidates"] > 1
