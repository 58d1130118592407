"""GPU parity of plans with several copies (the problem descriptor's C
copies at a distance): every copy is compared with the FP64 oracle on its
own inputs, and the words between copies must be left as they were."""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_17510_amd import Plan, synth

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}
SENTINEL = 12345.0 - 678.0j


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def reference(kind, ins):
    n = ins[0].size
    if kind == "centered":
        return oracle.conv_centered_direct(ins) if n <= 8000 else oracle.conv_centered_explicit(ins)
    if kind == "hermitian":
        return oracle.conv_hermitian_direct(ins) if n <= 8000 else oracle.conv_hermitian_explicit(ins)
    return oracle.conv_direct(ins) if n <= 8000 else oracle.conv_explicit(ins)


def check(shape, dtype, copies, dist=0, kind="plain", A=2, in_place=False, **kw):
    import torch
    say("copies case", shape, dtype, copies, dist, kind, kw)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    flags = {"centered": kind == "centered", "hermitian": kind == "hermitian"}
    with Plan(shape, A=A, dtype=dtype, copies=copies, dist=dist, **flags, **kw) as p:
        io = p.io_shape
        n = int(np.prod(io))
        step = dist or n
        span = (copies - 1) * step + n
        xs = [[synth.unit_disk(io, 7600 + 10 * c + a).astype(npdt) for a in range(A)] for c in range(copies)]
        flat = []
        for a in range(A):
            buf = np.full(span, SENTINEL, dtype=npdt)
            for c in range(copies):
                buf[c * step: c * step + n] = xs[c][a].ravel()
            flat.append(buf)
        dev = [torch.from_numpy(b).cuda() for b in flat]
        if not dist:
            dev = [t.reshape((copies,) + io) for t in dev]
        out = dev[0] if in_place else torch.full_like(dev[0], SENTINEL)
        p.execute(dev, out)
        torch.cuda.synchronize()
        info = p.info()
    got = out.cpu().numpy().ravel()
    for c in range(copies):
        want = reference(kind, [synth.as_oracle(x) for x in xs[c]])
        err = oracle.rel_l2(got[c * step: c * step + n], want.ravel())
        assert err <= TOL[dtype], (c, err)
        if c + 1 < copies and step > n:  # the gap after copy c is untouched
            gap = got[c * step + n: (c + 1) * step]
            assert np.all(gap == npdt(SENTINEL)), c
    say("   ->", [(d["variant"], d["m"], d["p"], d["q"]) for d in info["dims"]], "ok")
    return info


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_copies_1d_fused(gpu, dtype):
    info = check((1000,), dtype, 8)
    assert info["dims"][0]["variant"] == "fused"


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_copies_1d_multipass_gaps_and_accumulator(gpu, dtype):
    check((3000,), dtype, 3, dist=3300, m=64, variant="multipass", D=1)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(33, 47), (8, 12, 10)])
def test_copies_multidim(gpu, dtype, shape):
    check(shape, dtype, 3)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_copies_2d_gap(gpu, dtype):
    check((20, 30), dtype, 2, dist=700)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("kind,shape", [("centered", (1000,)), ("centered", (33, 40)), ("hermitian", (3001,)),
                                        ("hermitian", (21, 64))])
def test_copies_centered_hermitian(gpu, dtype, kind, shape):
    check(shape, dtype, 3, kind=kind)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape,dist", [((1000,), 1100), ((20, 30), 0)])
def test_copies_explicit(gpu, dtype, shape, dist):
    check(shape, dtype, 3, dist=dist, method="explicit")


def test_copies_three_inputs_and_in_place(gpu):
    check((500,), "c128", 4, A=3)
    check((2000,), "c128", 3, dist=2100, in_place=True, m=32, variant="multipass")


def test_convolve_helper_flags(gpu):
    import torch
    from paper_2303_17510_amd import convolve
    f, g = (synth.unit_disk((3, 40), 7700 + a) for a in range(2))
    out = convolve(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), copies=3, centered=True)
    for c in range(3):
        assert oracle.rel_l2(out[c].cpu().numpy(), oracle.conv_centered_direct([f[c], g[c]])) <= 1e-12
    h = convolve(torch.from_numpy(f[0]).cuda(), torch.from_numpy(g[0]).cuda(), hermitian=True)
    assert oracle.rel_l2(h.cpu().numpy(), oracle.conv_hermitian_direct([f[0], g[0]])) <= 1e-12


def _positions(io, strides):
    """Flat positions of a strided copy's elements (row-major over io)."""
    st = list(strides) + [1]
    if len(io) == 3 and len(strides) == 1:
        st = [strides[0], io[2], 1]
    grids = np.meshgrid(*[np.arange(n) * s for n, s in zip(io, st)], indexing="ij")
    return sum(grids).ravel()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape,strides,copies,dist,kind,kw", [
    ((20, 30), (40,), 1, 0, "plain", {}),
    ((20, 30), (33,), 3, 700, "plain", {}),
    ((6, 7, 9), (120, 12), 2, 0, "plain", {}),
    ((6, 7, 9), (80,), 1, 0, "plain", {}),
    ((33, 40), (48,), 2, 0, "centered", {}),
    ((21, 64), (40,), 2, 0, "hermitian", {}),
    ((20, 30), (40,), 2, 0, "plain", {"method": "explicit"}),
    ((6, 7, 9), (120, 12), 1, 0, "plain", {"method": "explicit"}),
    ((21, 64), (40,), 1, 0, "hermitian", {"method": "explicit"}),
])
def test_strided_layouts(gpu, dtype, shape, strides, copies, dist, kind, kw):
    import torch
    say("strided case", shape, strides, copies, dist, kind, dtype, kw)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    flags = {"centered": kind == "centered", "hermitian": kind == "hermitian"}
    with Plan(shape, dtype=dtype, copies=copies, dist=dist, strides=strides, **flags, **kw) as p:
        io, span = p.io_shape, p.span
        step = dist or span
        pos = _positions(io, strides)
        total = (copies - 1) * step + span
        xs = [[synth.unit_disk(io, 7800 + 10 * c + a).astype(npdt) for a in range(2)] for c in range(copies)]
        bufs = []
        for a in range(2):
            b = np.full(total, SENTINEL, dtype=npdt)
            for c in range(copies):
                b[c * step + pos] = xs[c][a].ravel()
            bufs.append(torch.from_numpy(b).cuda())
        out = torch.full_like(bufs[0], SENTINEL)
        p.execute(bufs, out)
        torch.cuda.synchronize()
    got = out.cpu().numpy()
    touched = np.zeros(total, bool)
    for c in range(copies):
        want = reference(kind, [synth.as_oracle(x) for x in xs[c]])
        assert oracle.rel_l2(got[c * step + pos], want.ravel()) <= TOL[dtype], c
        touched[c * step + pos] = True
    assert np.all(got[~touched] == npdt(SENTINEL))  # padding and gaps untouched
