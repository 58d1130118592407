"""Host-side checks of the tuner interface (no GPU needed)."""
import numpy as np

from paper_2303_17510_amd import tune


def test_candidates_follow_decoupled_search():
    c = tune.candidates((2048, 2048), (4096, 4096))
    assert c[0][0] == -1                        # the default plan first
    base = c[0][1]
    for v, shape in c[1:]:
        assert v in (0, 1)
        # exactly one dimension differs from the default plan
        other = 1 - v
        assert shape[other] == base[other]
        assert shape[v] != base[v]


def test_candidates_respect_geometry_rules():
    for L, M in [((1000,), (1999,)), ((1 << 20,), (1 << 21,)), ((300, 300), (600, 600))]:
        for v, shape in tune.candidates(L, M):
            for d, s in enumerate(shape):
                assert s["p"] * s["m"] >= L[d] and s["q"] * s["m"] >= M[d] and s["q"] >= s["p"]


def test_features_are_deterministic_and_finite():
    c = tune.candidates((12345,), (24690,))
    f1 = np.stack([tune.features((12345,), (24690,), s) for _, s in c])
    f2 = np.stack([tune.features((12345,), (24690,), s) for _, s in c])
    assert np.array_equal(f1, f2) and np.all(np.isfinite(f1))
    assert f1.shape == (len(c), tune.NF)
    assert len({tuple(r) for r in f1}) == len(c)   # candidates are distinguishable


def test_geometry_generator_is_seeded():
    a = tune.geometries(50, 7)
    b = tune.geometries(50, 7)
    assert a == b
    for g in a:
        assert all(M == g["A"] * L for L, M in zip(g["L"], g["M"]))
