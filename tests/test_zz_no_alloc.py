"""hdconv_execute_noalloc: the same launches as hdconv_execute, with the
library's static device scratch as the workspace (nothing allocated).

Each case runs a plan created without a workspace through the no-alloc entry
point and the same plan with its own workspace through hdconv_execute, on the
same seeded inputs, and compares both with each other and with the FP64
oracle.  Two calls follow each other, the second on a smaller problem, so the
second runs over what the first left in the scratch.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_17510_amd import Plan, _lib, synth

pytestmark = pytest.mark.gpu
TOL = {"c64": 1e-5, "c128": 1e-12}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_pair(shape, M, dtype, seed, **kw):
    """Output of the no-alloc entry point and of hdconv_execute, and the oracle's."""
    import torch
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = [synth.unit_disk(shape, seed + a).astype(npdt) for a in range(2)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    say("case", shape, M, dtype, kw)
    with Plan(shape, M, A=2, dtype=dtype, no_workspace=True, **kw) as pn, \
            Plan(shape, M, A=2, dtype=dtype, **kw) as po:
        info = pn.info()
        assert 0 < info["workspace_bytes"] <= _lib.SCRATCH_BYTES
        assert [(d["variant"], d["m"], d["q"], d["D"]) for d in info["dims"]] == \
            [(d["variant"], d["m"], d["q"], d["D"]) for d in po.info()["dims"]]
        out_n = torch.full_like(dev[0], float("nan"))
        out_o = torch.full_like(dev[0], float("nan"))
        pn.execute_noalloc(dev, out_n)
        po.execute(dev, out_o)
        torch.cuda.synchronize()
    got_n, got_o = out_n.cpu().numpy(), out_o.cpu().numpy()
    ins = [synth.as_oracle(x) for x in xs]
    want = oracle.conv_explicit(ins)
    return got_n, got_o, want, info


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_1d_accumulating_blocks(gpu, dtype):
    # inner form with one residue per block: the FP64 accumulator and the
    # work rows live in the scratch; the second, smaller call reuses them
    for L, m, seed in ((300000, 4096, 910), (70001, 2048, 920)):
        got_n, got_o, want, info = run_pair((L,), (2 * L,), dtype, seed, variant="multipass", D=1, m=m)
        assert info["dims"][0]["D"] == 1 and info["dims"][0]["n"] > 1
        e_no = oracle.rel_l2(got_n, got_o)
        e_n, e_o = oracle.rel_l2(got_n, want), oracle.rel_l2(got_o, want)
        say("   L=%d ws=%d  noalloc vs execute %.2e  vs oracle %.2e / %.2e" % (
            L, info["workspace_bytes"], e_no, e_n, e_o))
        assert e_no <= TOL[dtype] and e_n <= TOL[dtype] and e_o <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_2d_levels(gpu, dtype):
    # 2D: the outer level buffers live in the scratch
    for shape, seed in (((300, 200), 930), ((97, 50), 940)):
        M = tuple(2 * v for v in shape)
        got_n, got_o, want, info = run_pair(shape, M, dtype, seed)
        e_no = oracle.rel_l2(got_n, got_o)
        e_n = oracle.rel_l2(got_n, want)
        say("   %s ws=%d  noalloc vs execute %.2e  vs oracle %.2e" % (shape, info["workspace_bytes"], e_no, e_n))
        assert e_no <= TOL[dtype] and e_n <= TOL[dtype]


def test_noalloc_rules(gpu):
    import torch
    # a plan without a workspace does not run through hdconv_execute
    x = [torch.zeros(5000, dtype=torch.complex64, device="cuda") for _ in range(2)]
    with Plan((5000,), (10000,), A=2, dtype="c64", variant="multipass", no_workspace=True) as p:
        assert p.info()["workspace_bytes"] > 0
        with pytest.raises(_lib.HdconvError) as ei:
            p.execute(x, torch.empty_like(x[0]))
        assert ei.value.code == _lib.EINVAL
    # a workspace beyond the scratch is rejected before anything runs
    big = (160, 160, 160)
    y = [torch.zeros(big, dtype=torch.complex64, device="cuda") for _ in range(2)]
    with Plan(big, tuple(2 * v for v in big), A=2, dtype="c64", no_workspace=True) as p:
        assert p.info()["workspace_bytes"] > _lib.SCRATCH_BYTES
        out = torch.full_like(y[0], 7.0)
        with pytest.raises(_lib.HdconvError) as ei:
            p.execute_noalloc(y, out)
        assert ei.value.code == _lib.EUNSUPPORTED
        torch.cuda.synchronize()
        assert bool((out == 7.0).all())
