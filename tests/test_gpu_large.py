"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

The oracle evaluates sampled outputs one by one by direct sums (the first and
last outputs plus seeded random ones), and, where it is affordable on the
host, every output through its explicitly padded FFT convolution.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_17510_amd import Plan, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def sample_idx(shape, n, seed):
    total = int(np.prod(shape))
    rng = np.random.Generator(np.random.PCG64(seed))
    head = np.arange(min(32, total))
    tail = np.arange(max(0, total - 32), total)
    mid = rng.integers(0, total, size=n)
    return np.unique(np.concatenate([head, tail, mid]))


def run_case(shape, M, dtype, config_id, dist="disk", method="hybrid", **kw):
    import torch
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = synth.inputs(config_id, 2, shape, dist, dtype=npdt)
    dev = [torch.from_numpy(x).cuda() for x in xs]
    say("case", shape, M, dtype, method, kw)
    with Plan(shape, M, A=2, dtype=dtype, method=method, **kw) as p:
        info = p.info()
        out = torch.empty_like(dev[0])
        p.execute(dev, out)
        torch.cuda.synchronize()
    say("   plan", [(d["variant"], d["m"], d["p"], d["n"], d["q"]) for d in info["dims"]])
    return [synth.as_oracle(x) for x in xs], out.cpu().numpy()


def sampled_err(ins, got, nsamp, seed):
    idx = sample_idx(ins[0].shape, nsamp, seed)
    want = oracle.conv_direct(ins, idx=idx)
    return oracle.rel_l2(got.ravel()[idx], want)


TOL = {"c64": 1e-5, "c128": 1e-12}


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("method", ["hybrid", "explicit"])
def test_c2_pow2(gpu, dtype, method):
    L = 1 << 20
    ins, got = run_case((L,), (2 * L,), dtype, 1, method=method)
    e_s = sampled_err(ins, got, 512, 1)
    e_f = oracle.rel_l2(got, oracle.conv_explicit(ins))
    say("   sampled err %.3e  full err %.3e" % (e_s, e_f))
    assert e_s <= TOL[dtype] and e_f <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("method", ["hybrid", "explicit"])
def test_c2_1p5m(gpu, dtype, method):
    L = 1500000
    ins, got = run_case((L,), (2 * L - 1,), dtype, 1, method=method)
    e_s = sampled_err(ins, got, 512, 2)
    e_f = oracle.rel_l2(got, oracle.conv_explicit(ins))
    say("   sampled err %.3e  full err %.3e" % (e_s, e_f))
    assert e_s <= TOL[dtype] and e_f <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_c4_2d_2048(gpu, dtype):
    # every output against the explicitly padded oracle, plus direct sums
    ins, got = run_case((2048, 2048), (4096, 4096), dtype, 3, dist="gauss")
    e_s = sampled_err(ins, got, 96, 3)
    e_f = oracle.rel_l2(got, oracle.conv_explicit(ins))
    say("   sampled err %.3e  full err %.3e" % (e_s, e_f))
    assert e_s <= TOL[dtype] and e_f <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_c5_3d_256(gpu, dtype):
    # the headline workload: all 256^3 outputs against the oracle
    ins, got = run_case((256, 256, 256), (512, 512, 512), dtype, 4)
    e_s = sampled_err(ins, got, 24, 4)
    e_f = oracle.rel_l2(got, oracle.conv_explicit(ins))
    say("   sampled err %.3e  full err %.3e" % (e_s, e_f))
    assert e_s <= TOL[dtype] and e_f <= TOL[dtype]


def test_c4_centered_2048(gpu):
    # centered 2048^2 at the paper's centered padding M = 3L/2 per dimension
    import torch
    xs = synth.inputs(3, 2, (2048, 2048), "gauss", dtype=np.complex64)
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan((2048, 2048), (3072, 3072), A=2, dtype="c64", centered=True) as p:
        out = torch.empty_like(dev[0])
        p.execute(dev, out)
        torch.cuda.synchronize()
    ins = [synth.as_oracle(x) for x in xs]
    e = oracle.rel_l2(out.cpu().numpy(), oracle.conv_centered_explicit(ins))
    say("   centered 2048^2 full err %.3e" % e)
    assert e <= TOL["c64"]


def test_c4_hermitian_2047x2048(gpu):
    # Hermitian 2047 x 2048 (2047 x 1024 stored), M = 3072^2
    import torch
    xs = synth.inputs(3, 2, (2047, 1024), "gauss", dtype=np.complex64)
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan((2047, 2048), (3072, 3072), A=2, dtype="c64", hermitian=True) as p:
        out = torch.empty_like(dev[0])
        p.execute(dev, out)
        torch.cuda.synchronize()
    ins = [synth.as_oracle(x) for x in xs]
    e = oracle.rel_l2(out.cpu().numpy(), oracle.conv_hermitian_explicit(ins))
    say("   Hermitian 2047x2048 full err %.3e" % e)
    assert e <= TOL["c64"]


def test_c5_hermitian_3d(gpu):
    # 3D Hermitian 255 x 255 x 256 (255 x 255 x 128 stored), M = 384^3
    import torch
    xs = synth.inputs(4, 2, (255, 255, 128), "disk", dtype=np.complex64)
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan((255, 255, 256), (384, 384, 384), A=2, dtype="c64", hermitian=True) as p:
        out = torch.empty_like(dev[0])
        p.execute(dev, out)
        torch.cuda.synchronize()
    ins = [synth.as_oracle(x) for x in xs]
    e = oracle.rel_l2(out.cpu().numpy(), oracle.conv_hermitian_explicit(ins))
    say("   Hermitian 255x255x256 full err %.3e" % e)
    assert e <= TOL["c64"]


# default-plan rules that only particular shapes select: the shape is
# asserted, then every output compared with the oracle
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_2d_three_inputs_whole_outer(gpu, dtype):
    # 2D with A = 3 around L = 350: one whole outer transform (m >= M)
    import torch
    shape, M = (350, 40), (3 * 350 - 2, 3 * 40 - 2)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = synth.inputs(3, 3, shape, "gauss", dtype=npdt)
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan(shape, M, A=3, dtype=dtype) as p:
        dims = p.info()["dims"]
        # whole 512-point outer transforms, three residues (not halves of 256)
        assert (dims[0]["variant"], dims[0]["m"], dims[0]["p"], dims[0]["q"]) == ("outer", 512, 1, 3)
        out = torch.empty_like(dev[0])
        p.execute(dev, out)
        torch.cuda.synchronize()
    ins = [synth.as_oracle(x) for x in xs]
    e = oracle.rel_l2(out.cpu().numpy(), oracle.conv_direct(ins))
    say("   A=3 350x40 %s plan %s err %.3e" % (dtype, [(d["m"], d["p"], d["q"]) for d in dims], e))
    assert e <= TOL[dtype]


def test_2d_rows_just_above_power_of_two(gpu):
    # rows of 2200 points take two 2048-point blocks (p = 2)
    ins, got = run_case((2200, 2200), (4400, 4400), "c64", 3, dist="gauss")
    with Plan((2200, 2200), (4400, 4400), A=2, dtype="c64", host_only=True) as p:
        d = p.info()["dims"]
    assert (d[1]["variant"], d[1]["m"], d[1]["p"]) == ("fused", 2048, 2)
    assert (d[0]["variant"], d[0]["p"]) == ("outer", 2)
    e = oracle.rel_l2(got, oracle.conv_explicit(ins))
    say("   2200^2 full err %.3e" % e)
    assert e <= TOL["c64"]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_3d_inner_form_more_than_65535_rows(gpu, dtype):
    # outer transforms of 256 points (q = 1) leave 256 * 256 = 65536 rows for
    # the inner-form column passes of the last dimension
    shape, M = (74, 74, 74), (148, 148, 148)
    ins, got = run_case(shape, M, dtype, 4, m=(256, 256, 32), variant=("outer", "outer", "multipass"))
    e = sampled_err(ins, got, 64, 5)
    say("   sampled err %.3e" % e)
    assert e <= TOL[dtype]


def test_1d_maximum_length(gpu):
    # the largest 1D length the planner supports: 8192-point rows times
    # 4096-point columns, L = 2^25 (complex64), checked on sampled outputs
    L = 1 << 25
    ins, got = run_case((L,), (2 * L,), "c64", 1)
    e = sampled_err(ins, got, 24, 6)
    say("   sampled err %.3e" % e)
    assert e <= TOL["c64"]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n", [150, 229])
def test_3d_non_power_of_two(gpu, dtype, n):
    # default 3D plans for lengths well below a power of two: two blocks of
    # half the power of two in every dimension (150: 128-point blocks, q = 3),
    # else one block of the power of two (229: 256 points, q = 2)
    ins, got = run_case((n,) * 3, (2 * n,) * 3, dtype, 4)
    e = sampled_err(ins, got, 48, 7)
    say("   sampled err %.3e" % e)
    assert e <= TOL[dtype]
