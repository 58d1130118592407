"""Residue blocks on the first outer dimension (Sec. 5: the outer residues
are taken D at a time through the inner dimensions, the level buffers reused,
each block's inverse added to the output): every output against the FP64
oracle for 2D and 3D plans, lean and general outer kernels (centered and
Hermitian outer dimensions), quadratic operators and copies; the workspace
shrinks to one block's worth, A D m (inner extent) words at the first level,
and a workspace cap picks the block size by itself.  In-place execution is
refused for blocked plans (later blocks read the inputs again).
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


def run(shape, M, dtype, D0, A=2, seed=8500, kind="plain", **kw):
    import torch
    npdt = np.complex64 if dtype == "c64" else np.complex128
    io = shape[:-1] + ((shape[-1] + 1) // 2,) if kind == "hermitian" else shape
    xs = [synth.unit_disk(io, seed + a).astype(npdt) for a in range(A)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    D = tuple([D0] + [0] * (len(shape) - 1))
    with Plan(shape, M, A=A, dtype=dtype, D=D, centered=kind == "centered", hermitian=kind == "hermitian",
              **kw) as p:
        info = p.info()
        out = torch.full_like(dev[0], float("nan"))
        p.execute(dev, out)
        torch.cuda.synchronize()
    d0 = info["dims"][0]
    say("   %s %s %s D=%d: dim0 m=%d p=%d q=%d D=%d ws=%d" % (shape, dtype, kind, D0, d0["m"], d0["p"], d0["q"],
                                                            d0["D"], info["workspace_bytes"]))
    ins = [synth.as_oracle(x) for x in xs]
    if kind == "hermitian":
        want = oracle.conv_hermitian_explicit(ins)
    elif kind == "centered":
        want = oracle.conv_centered_explicit(ins)
    elif A == 3:
        want = oracle.conv_direct(ins)
    else:
        want = oracle.conv_explicit(ins)
    return oracle.rel_l2(out.cpu().numpy(), want), info


CASES = [
    ((1024, 100), (2048, 200), 1),       # 2D, q = 2, one residue a block (lean outer)
    ((700, 90), (1400, 180), 1),         # 2D outer two blocks of 512, q = 3
    ((700, 90), (1400, 180), 2),         # blocks of 2 and 1 residues
    ((96, 40, 50), (192, 80, 100), 1),   # 3D: the first dimension blocked, the second whole
    ((150, 30, 40), (300, 60, 80), 2),
]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("shape,M,D0", CASES, ids=["1024x100_D1", "700x90_D1", "700x90_D2", "96_D1", "150_D2"])
def test_blocks_plain(gpu, shape, M, D0, dtype):
    e, info = run(shape, M, dtype, D0)
    d0 = info["dims"][0]
    assert d0["D"] == D0 < d0["q"]
    say("   err %.2e" % e)
    assert e <= TOL[dtype]


def test_blocks_three_inputs(gpu):
    e, _ = run((200, 60), (598, 178), "c64", 1, A=3)
    say("   err %.2e" % e)
    assert e <= TOL["c64"]


@pytest.mark.parametrize("kind", ["centered", "hermitian"])
def test_blocks_centered_outer(gpu, kind):
    # centered outer dimensions run the general outer kernels with blocks
    shape = (255, 300) if kind == "hermitian" else (256, 300)
    M = (384, 450)
    e, info = run(shape, M, "c64", 1, kind=kind)
    assert info["dims"][0]["D"] == 1 < info["dims"][0]["q"]
    say("   err %.2e" % e)
    assert e <= TOL["c64"]


def test_blocks_quadratic_and_copies(gpu):
    import torch
    # Basdevant 2D (two outputs, each accumulated over the blocks)
    coef = [[[1, 0], [0, -1]], [[0, 1], [0, 0]]]
    shape, M = (300, 64), (600, 128)
    xs = [synth.unit_disk(shape, 8600 + a).astype(np.complex64) for a in range(2)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan(shape, M, A=2, B=2, dtype="c64", mult="quadratic", coef=coef, D=(1, 0)) as p:
        assert p.info()["dims"][0]["D"] == 1
        outs = [torch.full_like(dev[0], float("nan")) for _ in range(2)]
        p.execute(dev, outs)
        torch.cuda.synchronize()
    want = oracle.conv_quadratic([synth.as_oracle(x) for x in xs], coef)
    for b in range(2):
        e = oracle.rel_l2(outs[b].cpu().numpy(), want[b])
        say("   quadratic output %d err %.2e" % (b, e))
        assert e <= 1e-5
    # three copies, blocked
    xs = [synth.unit_disk((3, 100, 70), 8700 + a).astype(np.complex64) for a in range(2)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan((100, 70), (200, 140), A=2, dtype="c64", copies=3, D=(1, 0)) as p:
        out = torch.full_like(dev[0], float("nan"))
        p.execute(dev, out)
        torch.cuda.synchronize()
    got = out.cpu().numpy()
    for c in range(3):
        e = oracle.rel_l2(got[c], oracle.conv_explicit([synth.as_oracle(x[c]) for x in xs]))
        assert e <= 1e-5


def test_blocks_workspace_and_rules(gpu, monkeypatch):
    import torch
    shape, M = (1024, 100), (2048, 200)
    with Plan(shape, M, A=2, dtype="c64", host_only=True) as p:
        full = p.info()
    with Plan(shape, M, A=2, dtype="c64", D=(1, 0), host_only=True) as p:
        one = p.info()
    d0 = full["dims"][0]
    # one residue block: A D m (inner extent) complex words at the first level
    assert d0["q"] == 2
    assert one["workspace_bytes"] == 2 * 1 * d0["m"] * 100 * 8
    assert full["workspace_bytes"] == 2 * d0["q"] * d0["m"] * 100 * 8
    # in place is refused for a blocked plan
    x = [torch.zeros(shape, dtype=torch.complex64, device="cuda") for _ in range(2)]
    with Plan(shape, M, A=2, dtype="c64", D=(1, 0)) as p:
        with pytest.raises(_lib.HdconvError) as ei:
            p.execute(x, x[0])
        assert ei.value.code == _lib.EINVAL
    # residue blocks on a later outer dimension are refused
    with pytest.raises(_lib.HdconvError):
        Plan((64, 300, 20), (128, 600, 40), A=2, dtype="c64", D=(0, 1, 0), host_only=True)
    # a workspace cap between one block's and all blocks' size picks D by itself
    monkeypatch.setenv("HDCONV_WORKSPACE_CAP", str(one["workspace_bytes"]))
    e, info = run(shape, M, "c64", 0)
    assert info["dims"][0]["D"] == 1 and info["workspace_bytes"] <= one["workspace_bytes"]
    assert e <= 1e-5


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_inner_form_blocks_accumulate_in_output(gpu, dtype):
    # inner form with blocks of one residue: the contributions add into the
    # output array (no FP64 accumulation buffer: 16 L bytes less workspace)
    import torch
    L, M = 50000, 100000
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = [synth.unit_disk((L,), 8800 + a).astype(npdt) for a in range(2)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    kw = dict(A=2, dtype=dtype, m=2048, variant="multipass", D=1)
    with Plan((L,), (M,), host_only=True, **kw) as p:
        ws_acc = p.info()["workspace_bytes"]
    with Plan((L,), (M,), accumulate_output=True, **kw) as p:
        info = p.info()
        assert info["dims"][0]["n"] == 2 and info["dims"][0]["D"] == 1
        assert ws_acc - info["workspace_bytes"] >= 16 * L
        out = torch.full_like(dev[0], float("nan"))
        p.execute(dev, out)
        torch.cuda.synchronize()
        with pytest.raises(_lib.HdconvError) as ei:
            p.execute(dev, dev[0])
        assert ei.value.code == _lib.EINVAL
    e = oracle.rel_l2(out.cpu().numpy(), oracle.conv_explicit([synth.as_oracle(x) for x in xs]))
    say("   workspace %d -> %d bytes, err %.2e" % (ws_acc, info["workspace_bytes"], e))
    assert e <= TOL[dtype]
