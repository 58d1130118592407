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


def test_candidates_include_inner_form_on_outer_dimensions():
    # an outer dimension spanning more than two blocks of m = 64 .. 1024 also
    # lists the inner form (p > 2, q = n p); centered problems do not
    c = tune.candidates((3000, 64), (6000, 128))
    inner = [s[0] for v, s in c if v == 0 and s[0]["variant"] == "outer" and s[0]["p"] > 2]
    assert inner, "no inner-form candidate on dimension 0"
    for s in inner:
        assert 64 <= s["m"] <= 1024 and s["q"] % s["p"] == 0 and s["p"] * s["m"] >= 3000
    ctr = tune.candidates((3001, 64), (4502, 96), flags=4)
    assert not [s for v, s in ctr if s[0]["p"] > 2]


def test_candidates_of_centered_and_hermitian_problems():
    # the tuner lists shapes for centered and Hermitian problems too; they
    # carry the flag the time and feature functions read
    for flags, L, M in ((4, (2048,), (3072,)), (8, (2047, 2048), (3072, 3072))):
        c = tune.candidates(L, M, flags=flags)
        assert c[0][0] == -1 and len(c) > 3
        for v, shape in c:
            assert shape[-1]["centered"] == (2 if flags == 8 else 1)
            f = tune.features(L, M, shape)
            assert f[44] == 1.0 and f[45] == (1.0 if flags == 8 else 0.0)


def _rows(gids, ys, varied, dims):
    n = len(gids)
    return {"X": np.zeros((n, tune.NF), dtype=np.float32), "y": np.log(np.array(ys, dtype=np.float32)),
            "gid": np.array(gids, dtype=np.int64), "varied": np.array(varied, dtype=np.int64),
            "dims": np.array(dims, dtype=np.int64), "L": np.ones((n, 3), dtype=np.int64),
            "M": np.ones((n, 3), dtype=np.int64), "A": np.full(n, 2, dtype=np.int64),
            "shape": np.zeros((n, 3, 9), dtype=np.int64)}


def test_costmodel_load_later_files_replace_geometries(tmp_path):
    from paper_2303_17510_amd import costmodel
    a = _rows([0, 0, 1, 1], [1.0, 2.0, 3.0, 4.0], [-1, 0, -1, 0], [1, 1, 1, 1])
    b = _rows([1, 1, 1], [5.0, 6.0, 7.0], [-1, 0, 0], [1, 1, 1])
    costmodel.save(a, str(tmp_path / "a.npz"))
    costmodel.save(b, str(tmp_path / "b.npz"))
    d = costmodel.load([str(tmp_path / "a.npz"), str(tmp_path / "b.npz")])
    # geometry 0 keeps its two rows from a; geometry 1 has only b's three rows
    assert sorted(d["gid"].tolist()) == [0, 0, 1, 1, 1]
    assert np.allclose(np.sort(np.exp(d["y"][d["gid"] == 1])), [5.0, 6.0, 7.0], rtol=1e-5)


class _FixedModel:
    def __init__(self, pred):
        self.pred = np.asarray(pred, dtype=np.float64)

    def predict(self, X):
        return self.pred


def test_costmodel_evaluate_decision_regret():
    from paper_2303_17510_amd import costmodel
    # one 2D geometry: default (2 ms), two variations of dim 0 (1 ms, 3 ms), one of dim 1 (4 ms)
    d = _rows([7, 7, 7, 7], [2.0, 1.0, 3.0, 4.0], [-1, 0, 0, 1], [2, 2, 2, 2])
    # the model ranks the 3 ms variation first for dim 0 and the default first for dim 1
    r = costmodel.evaluate(_FixedModel([np.log(2.0), np.log(1.5), np.log(0.5), np.log(5.0)]), d)
    assert r["geometries"] == 1 and r["decisions"] == 2
    assert abs(r["regret_max"] - 2.0) < 1e-6                 # picked 3 ms, best 1 ms
    assert abs(r["decision_regret_max"] - 2.0) < 1e-6        # dim 0: 3 ms against 1 ms; dim 1: 2 against 2
    assert abs(r["decision_regret_geomean"] - (np.sqrt(3.0) - 1.0)) < 1e-6
    assert abs(r["gain_over_default_geomean"] - 2.0 / 3.0) < 1e-6
