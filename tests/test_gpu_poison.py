"""Workspace never read before it is written.

With HDCONV_POISON_WORKSPACE set, a plan's new workspace is filled with NaN
bytes before the first execute, so any kernel reading a workspace word that
no earlier kernel of the execute wrote would turn outputs into NaN.  One plan
of each workspace layout (inner-form work rows and the FP64 accumulator,
outer level buffers in 2D and 3D, the explicit method's padded arrays,
quadratic operators' result buffers) is run this way and compared with the
FP64 oracle.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2303_17510_amd import Plan, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = [
    ("1d inner form, accumulating blocks", (40000,), (80000,), {"variant": "multipass", "D": 1}),
    ("1d inner form, one block", (40000,), (80000,), {"variant": "multipass"}),
    ("2d", (130, 96), (260, 192), {}),
    ("3d", (24, 20, 33), (48, 40, 66), {}),
    ("3d inner-form rows", (12, 10, 300), (24, 20, 600), {"variant": ("outer", "outer", "multipass")}),
    ("2d centered", (64, 80), (96, 120), {"centered": True}),
    ("1d Hermitian inner form", (8191,), None, {"hermitian": True, "variant": "multipass"}),
    ("2d explicit", (100, 60), (200, 120), {"method": "explicit"}),
    ("1d explicit", (3000,), (6000,), {"method": "explicit"}),
]


@pytest.fixture
def poisoned(monkeypatch):
    monkeypatch.setenv("HDCONV_POISON_WORKSPACE", "1")
    yield


@pytest.mark.parametrize("name,shape,M,kw", CASES, ids=[c[0] for c in CASES])
def test_poisoned_workspace(gpu, poisoned, name, shape, M, kw):
    import torch
    assert os.environ.get("HDCONV_POISON_WORKSPACE") == "1"
    herm = kw.get("hermitian", False)
    io = shape[:-1] + ((shape[-1] + 1) // 2,) if herm else shape
    xs = [synth.unit_disk(io, 950 + a).astype(np.complex64) for a in range(2)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan(shape, M, A=2, dtype="c64", **kw) as p:
        assert p.info()["workspace_bytes"] > 0, "case has no workspace"
        out = torch.empty_like(dev[0])
        p.execute(dev, out)
        torch.cuda.synchronize()
    got = out.cpu().numpy()
    ins = [synth.as_oracle(x) for x in xs]
    if herm:
        want = oracle.conv_hermitian_explicit(ins)
    elif kw.get("centered"):
        want = oracle.conv_centered_explicit(ins)
    else:
        want = oracle.conv_explicit(ins)
    assert np.isfinite(got).all(), "NaN from the poisoned workspace"
    e = oracle.rel_l2(got, want)
    say("   %s err %.2e" % (name, e))
    assert e <= 1e-5


def test_poisoned_workspace_quadratic(gpu, poisoned):
    # Basdevant 2D (A = B = 2): the result rows and the innermost level's
    # result of one output live in the workspace
    import torch
    coef = [[[1, 0], [0, -1]], [[0, 1], [0, 0]]]
    shape, M = (64, 48), (128, 96)
    xs = [synth.unit_disk(shape, 960 + a).astype(np.complex64) for a in range(2)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan(shape, M, A=2, B=2, dtype="c64", mult="quadratic", coef=coef) as p:
        assert p.info()["workspace_bytes"] > 0
        outs = [torch.empty_like(dev[0]) for _ in range(2)]
        p.execute(dev, outs)
        torch.cuda.synchronize()
    ins = [synth.as_oracle(x) for x in xs]
    want = oracle.conv_quadratic(ins, coef)
    for b in range(2):
        got = outs[b].cpu().numpy()
        assert np.isfinite(got).all(), "NaN from the poisoned workspace"
        e = oracle.rel_l2(got, want[b])
        say("   quadratic output %d err %.2e" % (b, e))
        assert e <= 1e-5
