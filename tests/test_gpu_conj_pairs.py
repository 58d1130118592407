"""Conjugate-symmetry pairing in the inner form's forward column pass (the
paper's conjugate symmetry optimization, complex case): residues v and n - v
share their twiddles, the second transformed from conj(zeta_q^{vt}) f_t and
stored one frequency down.  Every output against the FP64 oracle, with the
pairing on and off, for odd and even n (n/2 is its own pair) and both
precisions; a block of fewer than all residues runs unpaired.
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


CASES = [
    # (shape, M, A, m): n residue blocks of size p m
    ((30000,), (3 * 30000 - 2,), 3, 2048),   # three inputs: n = 3
    ((20000,), (4 * 20000,), 2, 2048),       # n = 4 (v = 2 alone)
    ((12000,), (5 * 12000,), 2, 1024),       # n = 5
    ((6, 9000), (12, 4 * 9000), 2, 1024),    # 2D rows in the inner form, n = 3
]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("shape,M,A,m", CASES, ids=["n3_A3", "n4", "n5", "2d_n3"])
def test_conj_pairs(gpu, shape, M, A, m, dtype):
    import torch
    npdt = np.complex64 if dtype == "c64" else np.complex128
    xs = [synth.unit_disk(shape, 8300 + a).astype(npdt) for a in range(A)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    mm = tuple([0] * (len(shape) - 1) + [m])
    var = tuple(["outer"] * (len(shape) - 1) + ["multipass"])
    outs = {}
    for pairs in (True, False):
        with Plan(shape, M, A=A, dtype=dtype, m=mm, variant=var, conj_pairs=pairs) as p:
            d = p.info()["dims"][-1]
            out = torch.full_like(dev[0], float("nan"))
            p.execute(dev, out)
            torch.cuda.synchronize()
        outs[pairs] = out.cpu().numpy()
        say("   %s %s pairs=%s: m=%d p=%d n=%d D=%d" % (shape, dtype, pairs, d["m"], d["p"], d["n"], d["D"]))
        assert d["n"] >= 3 and d["D"] == d["n"]
    ins = [synth.as_oracle(x) for x in xs]
    want = oracle.conv_explicit(ins) if A == 2 else oracle.conv_direct(ins)
    e_on, e_off = oracle.rel_l2(outs[True], want), oracle.rel_l2(outs[False], want)
    say("   err paired %.2e unpaired %.2e" % (e_on, e_off))
    assert e_on <= TOL[dtype] and e_off <= TOL[dtype]


def test_conj_pairs_partial_blocks(gpu):
    # blocks of one residue: the pairing does not apply, the result is the same
    import torch
    L, M = 20000, 80000
    xs = [synth.unit_disk((L,), 8400 + a).astype(np.complex64) for a in range(2)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan((L,), (M,), A=2, dtype="c64", m=2048, variant="multipass", D=1) as p:
        out = torch.empty_like(dev[0])
        p.execute(dev, out)
        torch.cuda.synchronize()
    e = oracle.rel_l2(out.cpu().numpy(), oracle.conv_explicit([synth.as_oracle(x) for x in xs]))
    say("   D=1 err %.2e" % e)
    assert e <= 1e-5
