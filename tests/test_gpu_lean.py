"""The lean whole-row kernel (rows of one block, p = 1, product operator, many
rows): every output against the FP64 oracle, for each supported transform
size, both points-per-lane widths, two and three inputs, full and partial
rows (L < m), one and several residues, and both precisions.  Each case also
checks, from the library's per-launch record, that the lean kernel is the
one that ran.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2303_17510_amd import Plan, synth

pytestmark = pytest.mark.gpu
TOL = {"c64": 1e-5, "c128": 1e-12}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run(shape, M, A, dtype, E, seed, copies=1, **kw):
    import torch
    npdt = np.complex64 if dtype == "c64" else np.complex128
    full = ((copies,) + tuple(shape)) if copies > 1 else tuple(shape)
    xs = [synth.unit_disk(full, seed + a).astype(npdt) for a in range(A)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    dims = len(shape)
    Em = tuple([0] * (dims - 1) + [E])
    with Plan(shape, M, A=A, dtype=dtype, E_m=Em, copies=copies, **kw) as p:
        d = p.info()["dims"][-1]
        out = torch.full_like(dev[0], float("nan"))
        p.profile_begin(1)
        p.execute(dev, out)
        torch.cuda.synchronize()
        names = [s["name"] for s in p.profile_end()]
    say("   %s M=%s A=%d %s E=%d copies=%d: rows m=%d q=%d kernels %s" % (
        shape, M, A, dtype, E, copies, d["m"], d["q"], names))
    assert d["variant"] == "fused" and d["p"] == 1 and d["E_m"] == E
    assert "rows_lean" in names
    got = out.cpu().numpy()
    ins = [synth.as_oracle(x) for x in xs]
    if copies > 1:
        want = np.stack([oracle.conv_direct([x[c] for x in ins]) for c in range(copies)])
    elif A == 3 or np.prod(shape) <= 4096:
        want = oracle.conv_direct(ins)
    else:
        want = oracle.conv_explicit(ins)
    return oracle.rel_l2(got, want)


CASES = [
    # (shape, M, A): rows of 64 .. 2048 points, full and partial, q = 1, 2, 3
    ((40, 36, 256), (80, 72, 512), 2),     # full rows, q = 2
    ((20, 24, 200), (40, 48, 400), 2),     # partial rows (L = 200 < m = 256)
    ((33, 20, 64), (66, 40, 128), 2),      # m = 64
    ((17, 130, 100), (34, 260, 200), 2),   # m = 128, partial
    ((300, 512), (600, 1024), 2),          # 2D rows of 1024 points, q = 1
    ((64, 2048), (128, 4096), 2),          # 2D rows of 2048 points, q = 2
    ((30, 20, 100), (88, 58, 298), 3),     # three inputs, q = 3
    ((9, 11, 512), (18, 22, 1024), 2),     # m = 512
]


@pytest.mark.parametrize("E", [8, 16])
@pytest.mark.parametrize("shape,M,A", CASES, ids=["x".join(map(str, c[0])) + "_A%d" % c[2] for c in CASES])
def test_lean_rows_c64(gpu, shape, M, A, E):
    e = run(shape, M, A, "c64", E, 7100)
    say("   err %.2e" % e)
    assert e <= TOL["c64"]


@pytest.mark.parametrize("E", [4, 8])
@pytest.mark.parametrize("shape,M,A", CASES[:3] + CASES[6:7], ids=["256", "200", "64", "A3"])
def test_lean_rows_c128(gpu, shape, M, A, E):
    e = run(shape, M, A, "c128", E, 7200)
    say("   err %.2e" % e)
    assert e <= TOL["c128"]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_lean_rows_1d_copies(gpu, dtype):
    # 1D copies: the rows of a 1D plan; 777 rows is not a multiple of the
    # rows per workgroup
    e = run((1000,), (2000,), 2, dtype, 8 if dtype == "c64" else 4, 7300, copies=777)
    say("   err %.2e" % e)
    assert e <= TOL[dtype]


def test_lean_rows_persistent_loop(gpu):
    # more rows than resident workgroups: every workgroup loops
    e = run((96, 96, 128), (192, 192, 256), 2, "c64", 8, 7400)
    say("   err %.2e" % e)
    assert e <= TOL["c64"]


def test_lean_rows_in_place(gpu):
    # output over the first input (the paper's in-place convention)
    import torch
    shape, M = (24, 20, 256), (48, 40, 512)
    xs = [synth.unit_disk(shape, 7500 + a).astype(np.complex64) for a in range(2)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan(shape, M, A=2, dtype="c64", E_m=(0, 0, 16)) as p:
        p.execute(dev, dev[0])
        torch.cuda.synchronize()
    want = oracle.conv_explicit([synth.as_oracle(x) for x in xs])
    e = oracle.rel_l2(dev[0].cpu().numpy(), want)
    say("   in place err %.2e" % e)
    assert e <= TOL["c64"]


def run_outer(shape, M, A, dtype, E, S, seed, copies=1, method="hybrid"):
    import torch
    npdt = np.complex64 if dtype == "c64" else np.complex128
    full = ((copies,) + tuple(shape)) if copies > 1 else tuple(shape)
    xs = [synth.unit_disk(full, seed + a).astype(npdt) for a in range(A)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    dims = len(shape)
    Em = tuple([E] * (dims - 1) + [0])
    Ss = tuple([S] * (dims - 1) + [0])
    with Plan(shape, M, A=A, dtype=dtype, E_m=Em, S=Ss, copies=copies, method=method) as p:
        ds = p.info()["dims"]
        out = torch.full_like(dev[0], float("nan"))
        p.profile_begin(1)
        p.execute(dev, out)
        torch.cuda.synchronize()
        names = [s["name"] for s in p.profile_end()]
    say("   %s M=%s A=%d %s E=%d S=%d copies=%d %s: outer %s kernels %s" % (
        shape, M, A, dtype, E, S, copies, method, [(d["m"], d["q"]) for d in ds[:-1]], names))
    assert all(d["p"] == 1 and d["E_m"] == E and d["S"] == S for d in ds[:-1])
    assert names.count("outer_lean_fwd") >= dims - 1 and names.count("outer_lean_bwd") == dims - 1
    got = out.cpu().numpy()
    ins = [synth.as_oracle(x) for x in xs]
    if copies > 1:
        want = np.stack([oracle.conv_explicit([x[c] for x in ins]) for c in range(copies)])
    elif A == 3:
        want = oracle.conv_direct(ins)
    else:
        want = oracle.conv_explicit(ins)
    return oracle.rel_l2(got, want)


OUTER = [
    ((256, 24, 20), (512, 48, 40), 2),     # 3D outer 256-point halves, q = 2 (3D rule)
    ((200, 30), (400, 60), 2),             # 2D, partial columns (L = 200 < m)
    ((64, 40, 36), (128, 80, 72), 2),      # m = 128 one transform
    ((30, 500), (60, 1000), 2),            # m = 64
    ((500, 16), (1000, 32), 2),            # m = 1024
    ((80, 40, 30), (238, 118, 88), 3),     # three inputs
    ((33, 17, 257), (66, 34, 514), 2),     # R not a multiple of S
]


def outer_fits(shape, M, A, E, S):
    # the planner allows at most 1024 lanes per lean outer workgroup (and
    # 32 columns only up to 256 points)
    dims = len(shape)
    try:
        with Plan(shape, M, A=A, dtype="c64", E_m=tuple([E] * (dims - 1) + [0]),
                  S=tuple([S] * (dims - 1) + [0]), host_only=True):
            return True
    except Exception:
        return False


@pytest.mark.parametrize("E,S", [(8, 16), (16, 16), (8, 8), (16, 8), (8, 32), (16, 32)])
@pytest.mark.parametrize("shape,M,A", OUTER, ids=["x".join(map(str, c[0])) + "_A%d" % c[2] for c in OUTER])
def test_lean_outer_c64(gpu, shape, M, A, E, S):
    if not outer_fits(shape, M, A, E, S):
        pytest.skip("outer tile of %d columns x %d lanes exceeds the workgroup limit" % (S, max(M) // E))
    e = run_outer(shape, M, A, "c64", E, S, 7600)
    say("   err %.2e" % e)
    assert e <= TOL["c64"]


@pytest.mark.parametrize("shape,M,A", OUTER[:2] + OUTER[5:6], ids=["256", "200", "A3"])
def test_lean_outer_c128(gpu, shape, M, A):
    e = run_outer(shape, M, A, "c128", 8, 8, 7700)
    say("   err %.2e" % e)
    assert e <= TOL["c128"]


def test_lean_outer_c128_wide_tiles(gpu):
    # 32 columns of 256-point FP64 transforms: 1024 lanes, 128 KB of exchange
    e = run_outer(OUTER[0][0], OUTER[0][1], 2, "c128", 8, 32, 7750)
    say("   err %.2e" % e)
    assert e <= TOL["c128"]


def test_lean_outer_copies_and_explicit(gpu):
    # copies: the first outer pass reads planes dist apart; explicit padding:
    # one whole transform of the padded extent per outer dimension
    e = run_outer((64, 48), (128, 96), 2, "c64", 16, 16, 7800, copies=5)
    say("   copies err %.2e" % e)
    assert e <= TOL["c64"]
    e = run_outer((100, 60), (200, 120), 2, "c64", 16, 16, 7900, method="explicit")
    say("   explicit err %.2e" % e)
    assert e <= TOL["c64"]


# two blocks (p = 2, m < L <= 2m): rows and outer dimensions
P2_ROWS = [
    ((20, 24, 150), (40, 48, 300), 2, (0, 0, 128)),    # 3D rows of two 128-point blocks, q = 3
    ((6, 2200), (12, 4400), 2, (0, 2048)),             # 2D rows of two 2048-point blocks
    ((10, 12, 100), (28, 34, 298), 3, (0, 0, 64)),     # three inputs, q = 5
]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("shape,M,A,m", P2_ROWS, ids=["150", "2200", "A3"])
def test_lean_rows_two_blocks(gpu, shape, M, A, m, dtype):
    import torch
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = [synth.unit_disk(shape, 8100 + a).astype(npdt) for a in range(A)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan(shape, M, A=A, dtype=dtype, m=m) as p:
        d = p.info()["dims"][-1]
        out = torch.full_like(dev[0], float("nan"))
        p.profile_begin(1)
        p.execute(dev, out)
        torch.cuda.synchronize()
        names = [s["name"] for s in p.profile_end()]
    say("   %s rows m=%d p=%d q=%d E=%d kernels %s" % (shape, d["m"], d["p"], d["q"], d["E_m"], names))
    assert d["variant"] == "fused" and d["p"] == 2 and "rows_lean" in names
    ins = [synth.as_oracle(x) for x in xs]
    want = oracle.conv_direct(ins) if A == 3 else oracle.conv_explicit(ins)
    e = oracle.rel_l2(out.cpu().numpy(), want)
    say("   err %.2e" % e)
    assert e <= TOL[dtype]


P2_OUTER = [
    ((300, 40), (600, 80), 2, (256, 0)),               # 2D outer two 256-point blocks, q = 3
    ((2048, 64), (4096, 128), 2, (1024, 0)),           # the 2D 2048 outer shape: two 1024-point blocks, q = 4
    ((150, 20, 30), (300, 40, 60), 2, (128, 0, 0)),    # 3D outer two 128-point blocks
    ((100, 30, 20), (298, 88, 58), 3, (64, 0, 0)),     # three inputs
]


@pytest.mark.parametrize("shape,M,A", [((150, 40, 64), (300, 80, 128), 2), ((150, 20, 24), (448, 58, 70), 3)],
                         ids=["A2", "A3"])
def test_lean_outer_two_blocks_wide_tiles(gpu, shape, M, A):
    # two 128-point blocks with 32 columns per workgroup (the 3D default
    # from 256^3 on)
    import torch
    xs = [synth.unit_disk(shape, 8150 + a).astype(np.complex64) for a in range(A)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan(shape, M, A=A, dtype="c64", m=(128, 0, 0), E_m=(8, 0, 0), S=(32, 0, 0)) as p:
        d = p.info()["dims"][0]
        out = torch.full_like(dev[0], float("nan"))
        p.profile_begin(1)
        p.execute(dev, out)
        torch.cuda.synchronize()
        names = [s["name"] for s in p.profile_end()]
    say("   %s outer m=%d p=%d q=%d E=%d S=%d kernels %s" % (shape, d["m"], d["p"], d["q"], d["E_m"], d["S"], names))
    assert d["p"] == 2 and d["S"] == 32 and "outer_lean_fwd" in names
    ins = [synth.as_oracle(x) for x in xs]
    want = oracle.conv_direct(ins) if A == 3 else oracle.conv_explicit(ins)
    e = oracle.rel_l2(out.cpu().numpy(), want)
    say("   err %.2e" % e)
    assert e <= TOL["c64"]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("shape,M,A,m", P2_OUTER, ids=["300", "2048", "150", "A3"])
def test_lean_outer_two_blocks(gpu, shape, M, A, m, dtype):
    import torch
    if dtype == "c128" and m[0] == 1024:
        pytest.skip("FP64 1024-point outer transforms take 4 columns per workgroup (the general outer kernel)")
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = [synth.unit_disk(shape, 8200 + a).astype(npdt) for a in range(A)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan(shape, M, A=A, dtype=dtype, m=m) as p:
        d = p.info()["dims"][0]
        out = torch.full_like(dev[0], float("nan"))
        p.profile_begin(1)
        p.execute(dev, out)
        torch.cuda.synchronize()
        names = [s["name"] for s in p.profile_end()]
    say("   %s outer m=%d p=%d q=%d E=%d S=%d kernels %s" % (shape, d["m"], d["p"], d["q"], d["E_m"], d["S"], names))
    assert d["variant"] == "outer" and d["p"] == 2 and "outer_lean_fwd" in names and "outer_lean_bwd" in names
    ins = [synth.as_oracle(x) for x in xs]
    want = oracle.conv_direct(ins) if A == 3 else oracle.conv_explicit(ins)
    e = oracle.rel_l2(out.cpu().numpy(), want)
    say("   err %.2e" % e)
    assert e <= TOL[dtype]
