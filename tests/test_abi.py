"""Host-side checks of libhdconv: exports, planner rules, validation, errors.

No GPU is needed: plans are made with HDCONV_PLAN_HOST_ONLY, which computes
the geometry and sizes without device memory.
"""
import ctypes
import json
import math
import os
import re

import pytest

from paper_2303_17510_amd import Plan, geometry
from paper_2303_17510_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def declared_symbols():
    with open(os.path.join(ROOT, "include", "hdconv.h")) as fh:
        src = fh.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(hdconv_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    names = declared_symbols()
    assert names, "no declarations found"
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_version():
    assert b"hdconv" in _lib.lib().hdconv_version()


def test_fig1_geometry():
    g = json.load(open(os.path.join(GOLDEN, "fig1_hybrid_padding.json")))
    r = geometry(g["L"], g["M"], g["m"])
    assert (r["p"], r["q"]) == (g["p"], g["q"])
    assert r["p"] * r["m"] == g["pm"] and r["q"] * r["m"] == g["qm"]


def test_inner_loop_rules():
    g = json.load(open(os.path.join(GOLDEN, "inner_loop_rules.json")))
    for c in g["cases"]:
        r = geometry(c["L"], c["M"], c["m"])
        assert (r["p"], r["n"], r["q"]) == (c["p"], c["n"], c["q"]), c
        assert r["variant"] == "multipass"
    ce = g["centered_example"]
    # the library's centered geometry (hdconv_geometry_ex): the paper's p
    # counts the m-point blocks the signed indices span; the column DFT folds
    # the negative blocks onto the non-negative ones, so it has p/2 points,
    # and n = ceil(M/((p/2) m)) = ceil(2M/(p m)), q = n p/2 (Sec. 6.2, 7.2)
    from paper_2303_17510_amd.hdconv import geometry_centered
    r = geometry_centered(ce["L"], ce["M"], ce["m"])
    assert r["span"] == ce["p"]
    assert (2 * r["p"], r["n"], r["q"]) == (ce["p"], ce["n"], ce["q"])
    assert r["variant"] == "multipass" and r["centered"] == 1


def _brute_min_padding(L, A, centered):
    # least M such that no A-fold index sum other than an output index c is
    # congruent to c modulo M (plain indices 0 .. L-1, outputs 0 .. L-1;
    # centered -H .. L-1-H for both)
    H = L // 2 if centered else 0
    lo, hi = -A * H, A * (L - 1 - H)
    outs = range(-H, L - H)
    M = 1
    while True:
        if all(s == c or (s - c) % M != 0 for c in outs for s in range(lo, hi + 1)):
            return M
        M += 1


@pytest.mark.parametrize("L", [1, 2, 3, 4, 7, 8, 16, 31])
@pytest.mark.parametrize("A", [2, 3])
def test_min_padding_matches_brute_force(L, A):
    from paper_2303_17510_amd.hdconv import min_padding
    assert min_padding(L, A) == _brute_min_padding(L, A, False) == A * (L - 1) + 1
    assert min_padding(L, A, centered=True) == _brute_min_padding(L, A, True)
    # a Hermitian half of nominal length L stands for the centered length 2 ceil(L/2) - 1
    Lc = 2 * ((L + 1) // 2) - 1
    assert min_padding(L, A, hermitian=True) == _brute_min_padding(Lc, A, True)


def test_min_padding_paper_values():
    from paper_2303_17510_amd.hdconv import min_padding
    # centered and Hermitian benchmarks use M = 3L/2 (Sec. 7): the centered
    # minimum for even L and two factors
    for L in (2, 64, 2048, 1 << 20):
        assert min_padding(L, 2, centered=True) == 3 * L // 2
        assert min_padding(L, 2, hermitian=True) <= 3 * L // 2
    with pytest.raises(_lib.HdconvError):
        min_padding(0, 2)
    with pytest.raises(_lib.HdconvError):
        min_padding(10, 4)


def test_workspace_cap(monkeypatch):
    # the cap is checked on the host before any device call: an inner-form
    # plan needs work rows, a whole-row plan none
    with Plan((1 << 20,), (1 << 21,), host_only=True) as p:
        need = p.info()["workspace_bytes"]
    assert need > 0
    monkeypatch.setenv("HDCONV_WORKSPACE_CAP", str(need - 1))
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((1 << 20,), (1 << 21,))
    assert ei.value.code == _lib.ENOMEM and "HDCONV_WORKSPACE_CAP" in str(ei.value)
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((1 << 20,), (1 << 21,), host_only=True)
    assert ei.value.code == _lib.ENOMEM
    monkeypatch.setenv("HDCONV_WORKSPACE_CAP", str(need))
    Plan((1 << 20,), (1 << 21,), host_only=True).close()


@pytest.mark.parametrize("L", [1, 2, 3, 7, 100, 1023, 1024, 1025, 4096, 100000])
@pytest.mark.parametrize("ratio", [1, 2, 3])
def test_geometry_invariants(L, ratio):
    M = max(1, ratio * L - (1 if ratio > 1 else 0))
    for m in (1, 2, 3, 4, 8, 16, 100, 1024, 4096):
        r = geometry(L, M, m)
        assert r["p"] == math.ceil(L / m) or r["p"] == max(math.ceil(L / m), 0)
        assert r["p"] * m >= L and r["q"] * m >= M and r["q"] >= r["p"]
        if r["p"] <= 2:
            assert r["q"] == math.ceil(M / m) and r["variant"] == "fused"
        else:
            assert r["q"] == r["n"] * r["p"] and r["n"] == math.ceil(M / (r["p"] * m))
        # m >= M is explicit padding: p = q = 1
        if m >= M:
            assert r["p"] == r["q"] == 1


def test_p_min_allows_more_explicit_padding():
    r = geometry(1500000, 2999999, 8192, p_min=192)
    assert r["p"] == 192 and r["n"] == 2 and r["q"] == 384 and r["q"] * r["m"] >= 2999999


def test_plan_info_host_only():
    p = Plan((1 << 20,), (1 << 21,), dtype="c64", host_only=True)
    i = p.info()
    d = i["dims"][0]
    assert d["variant"] == "multipass" and d["p"] * d["m"] >= 1 << 20 and d["q"] * d["m"] >= 1 << 21
    assert i["compulsory_bytes"] == 3 * (1 << 20) * 8
    # 3 passes: read inputs, 2 (A+B) q m round trips, write output
    assert i["traffic_bytes"] == pytest.approx(8 * (3 * (1 << 20) + 6 * d["q"] * d["m"]))
    assert i["launches"] == 3
    p.close()


@pytest.mark.parametrize("L,A,dtype,E", [
    ((256, 256, 256), 2, "c64", 16),   # 256-point rows, two residues: 16 points per lane
    ((128, 128, 128), 2, "c64", 16),
    ((64, 64, 64), 2, "c64", 8),
    ((256, 256, 256), 3, "c64", 8),    # three inputs keep 8
    ((256, 256, 256), 2, "c128", 8),
    ((64, 64, 64), 2, "c128", 8),
])
def test_default_row_points_per_lane(L, A, dtype, E):
    # the planner's measured rule for the whole-row pass of 2D/3D plans
    with Plan(L, tuple(A * v for v in L), A=A, dtype=dtype, host_only=True) as p:
        d = p.info()["dims"][-1]
    assert d["variant"] == "fused" and d["E_m"] == E


@pytest.mark.parametrize("L,dtype,outer", [
    ((256, 256, 256), "c64", (128, 2, 32)),   # 2^16+ columns: 32-column tiles, two half blocks on the tie
    ((128, 128, 128), "c64", (128, 1, 16)),   # fewer columns: 16-column tiles, one block
    ((256, 256, 256), "c128", (256, 1, 8)),   # FP64 keeps its tiles
])
def test_default_3d_outer_tiles(L, dtype, outer):
    with Plan(L, tuple(2 * v for v in L), dtype=dtype, host_only=True) as p:
        ds = p.info()["dims"]
    assert all((d["variant"], d["m"], d["p"], d["S"]) == ("outer",) + outer for d in ds[:-1])


def test_workspace_accounting_2d():
    # Sec. 5: the decomposition keeps q_x m_x rows of L_y per input
    p = Plan((2048, 2048), (4096, 4096), dtype="c64", host_only=True)
    i = p.info()
    dx = i["dims"][0]
    assert i["workspace_bytes"] >= 2 * dx["q"] * dx["m"] * 2048 * 8


def test_explicit_plan_pads_to_smooth_size():
    p = Plan((1500000,), (2999999,), dtype="c64", method="explicit", host_only=True)
    assert p.info()["npad"] == [3 * (1 << 20)]


def test_explicit_plan_takes_a_forced_split():
    for m in (2048, 4096, 8192):
        with Plan((1 << 20,), (1 << 21,), dtype="c64", method="explicit", m=m, host_only=True) as p:
            d = p.info()["dims"][0]
            assert (d["m"], d["p"], d["n"], d["q"]) == (m, (1 << 21) // m, 1, (1 << 21) // m)
    with pytest.raises(_lib.HdconvError):
        Plan((1 << 20,), (1 << 21,), dtype="c64", method="explicit", m=3072, host_only=True)


@pytest.mark.parametrize("bad", [
    dict(L=(10,), M=(18,)),            # M < 2L - 1
    dict(L=(10,), M=(27,), A=3),       # M < 3L - 2
    dict(L=(0,), M=(4,)),
    dict(L=(10, 10, 10, 10), M=(20,) * 4),
])
def test_invalid_arguments(bad):
    with pytest.raises((_lib.HdconvError, ValueError)) as ei:
        Plan(host_only=True, **bad)
    if isinstance(ei.value, _lib.HdconvError):
        assert ei.value.code == _lib.EINVAL


def test_unsupported_arguments():
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((10,), (20,), A=2, B=2, host_only=True)
    assert ei.value.code == _lib.EUNSUPPORTED
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((10,), (40,), A=4, host_only=True)
    assert ei.value.code == _lib.EUNSUPPORTED
    # beyond the longest supported 1D length (8192-point rows x 4096-point columns)
    with pytest.raises(_lib.HdconvError) as ei:
        Plan(((1 << 25) + 1,), ((1 << 26) + 2,), host_only=True)
    assert ei.value.code == _lib.EUNSUPPORTED
    with Plan((1 << 25,), (1 << 26,), host_only=True) as p:
        d = p.info()["dims"][0]
        assert d["p"] * d["m"] >= 1 << 25 and d["q"] * d["m"] >= 1 << 26
    # q m would not fit the 32-bit residue twiddle exponents
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((1000,), (1 << 32,), host_only=True)
    assert ei.value.code == _lib.EUNSUPPORTED


def test_forced_p_gt_2_needs_multipass():
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((1024,), (2048,), m=16, variant="fused", host_only=True)
    assert ei.value.code == _lib.EINVAL


def test_execute_rejects_host_only_and_null():
    lib = _lib.lib()
    p = Plan((16,), (32,), host_only=True)
    ins = (ctypes.c_void_p * 2)(1, 2)
    outs = (ctypes.c_void_p * 1)(3)
    assert lib.hdconv_execute(p._h, ins, outs, None) == _lib.EINVAL
    assert lib.hdconv_execute(None, ins, outs, None) == _lib.EINVAL
    code, msg = _lib.last_error()
    assert code == _lib.EINVAL and msg


def test_device_plan_without_gpu_reports_enodev():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((16,), (32,))
    assert ei.value.code == _lib.ENODEV


def test_every_config_plans():
    cases = [((1024,), (2048,), "c128"), ((1 << 20,), (1 << 21,), "c64"), ((1 << 20,), (1 << 21,), "c128"),
             ((1500000,), (2999999,), "c64"), ((2048, 2048), (4096, 4096), "c64"),
             ((256, 256, 256), (512, 512, 512), "c64")]
    for L, M, dt in cases:
        for method in ("hybrid", "explicit"):
            Plan(L, M, dtype=dt, method=method, host_only=True).close()


# ------------------------------------------------------ centered plans ----
def _centered_min(L, A):
    # -H .. L-1-H per input; A-fold sums must not alias an output index
    H = L // 2
    P = L - 1 - H
    return max(A * P + H, P + A * H) + 1


@pytest.mark.parametrize("L,A", [(1, 2), (2, 2), (7, 2), (8, 2), (1024, 2), (1023, 2), (100, 3), (101, 3)])
def test_centered_padding_rule(L, A):
    Mc = _centered_min(L, A)
    if L % 2 == 0 and A == 2:
        assert Mc == 3 * L // 2  # the padding the paper quotes for the centered case
    with Plan((L,), (Mc,), A=A, centered=True, host_only=True) as p:
        d = p.info()["dims"][0]
        assert d["centered"] and d["q"] * d["m"] >= Mc
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((L,), (Mc - 1,), A=A, centered=True, host_only=True)
    assert ei.value.code == _lib.EINVAL
    if Mc < A * (L - 1) + 1:  # below the uncentered minimum: only centered plans take it
        with pytest.raises(_lib.HdconvError):
            Plan((L,), (Mc,), A=A, host_only=True)


def test_centered_shapes():
    from paper_2303_17510_amd.hdconv import centered_min_padding
    for L in (10, 1000, 1024, 4096, 8192, 16384, 1 << 16, 1 << 20):
        for dt in ("c64", "c128"):
            with Plan((L,), A=2, dtype=dt, centered=True, host_only=True) as p:
                d = p.info()["dims"][0]
                assert p.M == (centered_min_padding(L, 2),)
                H = L // 2
                tneg, tpos = -(-H // d["m"]), -(-(L - H) // d["m"])
                if d["variant"] == "fused":
                    assert d["p"] == tneg + tpos <= 2
                else:
                    assert tpos <= d["p"] and d["q"] == d["n"] * d["p"]
                assert d["q"] * d["m"] >= p.M[0]
                if L in (1 << 16, 1 << 20):
                    assert d["q"] * d["m"] == 3 * L // 2  # the centered padding is reached
                if L == 1024:  # a lone row: one power-of-two transform (3 * 2^k rows run slower)
                    assert d["variant"] == "fused" and d["q"] == 1 and d["m"] == 2048
    # forced shapes: direct form p = 2 with m = L/2, and the folded inner form
    with Plan((1024,), (1536,), centered=True, m=512, host_only=True) as p:
        d = p.info()["dims"][0]
        assert (d["variant"], d["p"], d["q"]) == ("fused", 2, 3)
    with Plan((1 << 20,), (3 << 19,), centered=True, m=4096, p=128, variant="multipass", host_only=True) as p:
        d = p.info()["dims"][0]
        assert (d["p"], d["n"], d["q"]) == (128, 3, 384)
    # a smaller p is a minimum only: the positive half needs 128 blocks
    with Plan((1 << 20,), (3 << 19,), centered=True, m=4096, p=64, variant="multipass", host_only=True) as p:
        assert p.info()["dims"][0]["p"] == 128


def test_centered_multidim_and_explicit_plans():
    with Plan((256, 256), centered=True, host_only=True) as p:
        for d in p.info()["dims"]:
            assert d["centered"] and d["q"] * d["m"] == 384
    with Plan((1024,), centered=True, method="explicit", host_only=True) as p:
        assert p.info()["npad"] == [1536]


# ----------------------------------------------------- Hermitian plans ----
@pytest.mark.parametrize("L,A", [(1, 2), (2, 2), (7, 2), (8, 2), (1024, 2), (1023, 3)])
def test_hermitian_padding_rule(L, A):
    Lh = (L + 1) // 2
    Mh = (A + 1) * (Lh - 1) + 1  # the centered minimum of the full length 2 Lh - 1
    with Plan((L,), (Mh,), A=A, hermitian=True, host_only=True) as p:
        d = p.info()["dims"][0]
        assert d["hermitian"] and d["L"] == 2 * Lh - 1 and d["q"] * d["m"] >= Mh
        assert p.io_shape == (Lh,)
        # the stored halves are what the kernels read and write
        assert p.info()["compulsory_bytes"] == (A + 1) * Lh * 8
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((L,), (Mh - 1,), A=A, hermitian=True, host_only=True)
    assert ei.value.code == _lib.EINVAL


def test_hermitian_multidim_shapes():
    # outer dimensions are centered with a symmetric (odd) range
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((16, 16), hermitian=True, host_only=True)
    assert ei.value.code == _lib.EINVAL
    with Plan((33, 64), hermitian=True, host_only=True) as p:
        assert p.io_shape == (33, 32)
        dims = p.info()["dims"]
        assert [d["hermitian"] for d in dims] == [False, True] and all(d["centered"] for d in dims)
        assert dims[0]["q"] * dims[0]["m"] >= 49 and dims[1]["L"] == 63
    with Plan((9, 11, 20), hermitian=True, method="explicit", host_only=True) as p:
        assert p.io_shape == (9, 11, 10) and p.info()["npad"] == [16, 16, 32]
    # the paper's Hermitian benchmark padding M = 3L/2 is accepted
    with Plan((1 << 20,), (3 << 19,), hermitian=True, host_only=True) as p:
        d = p.info()["dims"][0]
        assert d["q"] * d["m"] >= 3 << 19


def test_explicit_c128_long_rows_split():
    # one 8192-point complex128 row of A = 2 inputs does not fit LDS: the
    # explicit method splits N' = p m instead of failing
    for L, M in (((4097,), (8193,)), ((5000,), (9999,))):
        with Plan(L, M, dtype="c128", method="explicit", host_only=True) as p:
            d = p.info()["dims"][0]
            assert d["variant"] == "multipass" and d["p"] * d["m"] == p.info()["npad"][0]


def test_copies_validation_and_accounting():
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((100,), copies=2, dist=50, host_only=True)
    assert ei.value.code == _lib.EINVAL
    with Plan((1024,), copies=1, host_only=True) as p1, Plan((1024,), copies=8, host_only=True) as p8:
        # copies share the launches and multiply the designed traffic
        assert p8.info()["launches"] == p1.info()["launches"]
        assert p8.info()["traffic_bytes"] == pytest.approx(8 * p1.info()["traffic_bytes"])
    with Plan((1000,), copies=5, method="explicit", host_only=True) as p:
        assert p.info()["launches"] == 5 * 4  # pads, transform, truncation per copy


def test_strides_validation():
    with Plan((20, 30), strides=(40,), host_only=True) as p:
        assert p.span == 800
    for L, st in (((20, 30), (29,)), ((5, 6, 7), (50, 10)), ((100,), (200,))):
        with pytest.raises(_lib.HdconvError) as ei:
            Plan(L, strides=st, host_only=True)
        assert ei.value.code == _lib.EINVAL


def test_quadratic_operator_validation_and_accounting():
    basdevant = [[[1, 0], [0, -1]], [[0, 1], [0, 0]]]  # B = 2 outputs of A = 2 inputs
    # two factors per term: A = 3 inputs pad like A = 2
    coef3 = [[[1 if (i, j) == (0, 1) else 0 for j in range(3)] for i in range(3)]]
    with Plan((100,), (199,), A=3, B=1, mult="quadratic", coef=coef3, host_only=True) as p:
        assert p.info()["B"] == 1
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((100,), (198,), A=3, B=1, mult="quadratic", coef=coef3, host_only=True)
    assert ei.value.code == _lib.EINVAL
    # default M follows the two-factor rule too
    with Plan((100,), A=3, B=1, mult="quadratic", coef=coef3, host_only=True) as p:
        assert p.M == (200,)
    with pytest.raises(ValueError):
        Plan((100,), B=2, mult="quadratic", host_only=True)  # no coefficients
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((100,), B=9, mult="quadratic", coef=[basdevant[0]] * 9, host_only=True)
    assert ei.value.code == _lib.EINVAL
    # more than three inputs only with a quadratic operator, at most six
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((100,), A=4, host_only=True)
    assert ei.value.code == _lib.EUNSUPPORTED
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((100,), A=7, B=1, mult="quadratic", coef=[[[0] * 7] * 7], host_only=True)
    assert ei.value.code == _lib.EUNSUPPORTED
    with pytest.raises(_lib.HdconvError) as ei:
        Plan((100,), B=2, mult="quadratic", coef=basdevant, tuner="exhaustive")
    assert ei.value.code == _lib.EUNSUPPORTED
    # launches: the forward passes once, the row pass and inverse passes per output
    with Plan((4096,), B=2, mult="quadratic", coef=basdevant, variant="fused", host_only=True) as p:
        assert p.info()["launches"] == 2
    with Plan((256, 256), B=2, mult="quadratic", coef=basdevant, host_only=True) as p, \
            Plan((256, 256), host_only=True) as p1:
        assert p1.info()["launches"] == 3 and p.info()["launches"] == 5
        assert p.info()["traffic_bytes"] > p1.info()["traffic_bytes"]
    with Plan((1 << 20,), B=2, mult="quadratic", coef=basdevant, host_only=True) as p:
        d = p.info()["dims"][0]
        assert d["variant"] == "multipass" and d["D"] >= d["n"]
        assert p.info()["launches"] == 1 + 2 * 2
    with Plan((1 << 20,), B=2, mult="quadratic", coef=basdevant, m=d["m"], D=1,
              variant="multipass", host_only=True) as p:
        assert p.info()["dims"][0]["D"] == 1 and p.info()["dims"][0]["n"] == 2
        assert p.info()["launches"] == 2 * 3 * 2


def mhd_coefficients():
    """Elsasser form of the 3D MHD nonlinearity: inputs z+ (0, 1, 2) and z-
    (3, 4, 5); outputs z+_0 z-_0 - z+_2 z-_2, z+_1 z-_1 - z+_2 z-_2 and the
    six products z+_i z-_j, i != j (A = 6, B = 8)."""
    def out(terms):
        c = [[0.0] * 6 for _ in range(6)]
        for (i, j), w in terms.items():
            c[min(i, j)][max(i, j)] += w
        return c
    coef = [out({(0, 3): 1, (2, 5): -1}), out({(1, 4): 1, (2, 5): -1})]
    coef += [out({(i, 3 + j): 1}) for i in range(3) for j in range(3) if i != j]
    return coef


def test_six_input_quadratic_operator_shares():
    coef = mhd_coefficients()
    # outputs with four inputs run as two launches of two, the rest as one:
    # 2 + 2 + 6 row launches in 1D
    with Plan((1000,), A=6, B=8, mult="quadratic", coef=coef, variant="fused", host_only=True) as p:
        assert p.M == (2000,) and p.info()["launches"] == 10
    # 2D: the outer forward pass in two launches of three inputs, per output
    # its row launches and one outer inverse pass
    with Plan((33, 47), A=6, B=8, mult="quadratic", coef=coef, host_only=True) as p:
        assert p.info()["launches"] == 2 + 10 + 8
    # inner-form rows with two residue blocks: per block two column launches,
    # then per share a row and a column launch
    with Plan((3000,), A=6, B=8, mult="quadratic", coef=coef, m=64, variant="multipass", D=1,
              host_only=True) as p:
        d = p.info()["dims"][0]
        assert d["n"] == 2 and p.info()["launches"] == 8 * 2 * 2 + 2 * 2 * 10


def test_batched_plans_reject_quadratic_operators():
    lib = _lib.lib()
    opt = _lib.Options()
    lib.hdconv_options_init(ctypes.byref(opt))
    opt.mult = _lib.MULT_QUADRATIC
    coef = (ctypes.c_double * 4)(1, 0, 0, 1)
    opt.mult_coef = ctypes.cast(coef, ctypes.POINTER(ctypes.c_double))
    Ls = (ctypes.c_int64 * 2)(100, 200)
    Ms = (ctypes.c_int64 * 2)(200, 400)
    h = lib.hdconv_plan_batched(Ls, Ms, 2, 2, 1, 1, _lib.C64, ctypes.byref(opt))
    assert not h
    assert _lib.last_error()[0] == _lib.EUNSUPPORTED
