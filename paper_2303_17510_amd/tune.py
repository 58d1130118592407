"""Autotuning and the learned cost model, from Python.

Thin wrappers over the C ABI (include/hdconv.h): candidate enumeration
(``candidates``), device timing of one candidate (``time_shape``), the
cost-model feature vector (``features``), and ``CostModel`` around the
library's MLP (trained and evaluated by its HIP kernels).  Also the seeded
geometry generator of the cost-model workload and the regret measure.

The paper's optimizer (Sec. 7) picks the subtransform size and the residue
block count empirically, tuning each dimension independently; the
candidates here follow that decoupling: the default plan and the plan with
one dimension's shape replaced.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np

from . import _lib as _L
from .hdconv import dtype_code

NF = _L.NFEATURES
SHAPE_KEYS = ("variant", "m", "p", "q", "E_m", "E_p", "S", "rows_per_block")


def _arrs(L, M):
    L = [int(v) for v in L]
    M = [int(v) for v in M]
    return (ctypes.c_int64 * 3)(*(L + [1] * (3 - len(L)))), (ctypes.c_int64 * 3)(*(M + [1] * (3 - len(M)))), len(L)


def _shape_to_struct(shape):
    arr = (_L.DimInfo * len(shape))()
    for d, s in enumerate(shape):
        for k, v in s.items():
            if k == "variant":
                v = {"fused": 1, "multipass": 2, "outer": 3}.get(v, v)
            if hasattr(arr[d], k):
                setattr(arr[d], k, int(v))
    return arr


def _struct_to_shape(di):
    return {"L": di.L, "M": di.M, "m": di.m, "p": di.p, "n": di.n, "q": di.q, "D": di.D,
            "variant": _L.VARIANT_NAMES[di.variant], "E_m": di.E_m, "E_p": di.E_p, "S": di.S,
            "rows_per_block": di.rows_per_block, "tw_m": di.tw_m, "tw_p": di.tw_p, "centered": di.centered}


def candidates(L, M, A=2, dtype="c64", flags=0):
    """[(varied_dim, [per-dimension shape dicts])]; varied_dim -1 is the default plan.
    ``flags``: 0, PLAN_CENTERED or PLAN_HERMITIAN (the shapes then carry it)."""
    Ls, Ms, dims = _arrs(L, M)
    cnt = ctypes.c_int(0)
    _L.check(_L.lib().hdconv_candidates(Ls, Ms, A, 1, dims, dtype_code(dtype), int(flags), None, None, 0,
                                        ctypes.byref(cnt)))
    n = cnt.value
    out = (_L.DimInfo * (n * dims))()
    var = (ctypes.c_int * n)()
    _L.check(_L.lib().hdconv_candidates(Ls, Ms, A, 1, dims, dtype_code(dtype), int(flags), out, var, n,
                                        ctypes.byref(cnt)))
    return [(var[k], [_struct_to_shape(out[k * dims + d]) for d in range(dims)]) for k in range(n)]


def time_shape(L, M, shape, A=2, dtype="c64", reps=5) -> float:
    """Steady-state ms per execute of the plan with these per-dimension shapes
    (median over three blocks of `reps` back-to-back executes)."""
    Ls, Ms, dims = _arrs(L, M)
    ms = ctypes.c_double(0)
    _L.check(_L.lib().hdconv_time_shape(Ls, Ms, A, 1, dims, dtype_code(dtype), _shape_to_struct(shape), reps,
                                        ctypes.byref(ms)))
    return ms.value


def features(L, M, shape, A=2, dtype="c64") -> np.ndarray:
    Ls, Ms, dims = _arrs(L, M)
    out = (ctypes.c_float * NF)()
    _L.check(_L.lib().hdconv_features(Ls, Ms, A, 1, dims, dtype_code(dtype), _shape_to_struct(shape), out))
    return np.frombuffer(out, dtype=np.float32).copy()


def _fp(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class CostModel:
    """The library's MLP cost model (features -> predicted log ms)."""

    def __init__(self, hidden: int = 64, seed: int = 0):
        self.hidden = hidden
        self.handle = _L.lib().hdconv_model_create(hidden, seed)
        if not self.handle:
            raise _L.HdconvError(_L.EDEVICE, "hdconv_model_create failed")

    def params(self) -> np.ndarray:
        n = ctypes.c_int(0)
        _L.check(_L.lib().hdconv_model_params(self.handle, None, 0, ctypes.byref(n)))
        buf, ptr = _fp(np.zeros(n.value))
        _L.check(_L.lib().hdconv_model_params(self.handle, ptr, n.value, ctypes.byref(n)))
        return buf

    def load(self, params):
        buf, ptr = _fp(params)
        _L.check(_L.lib().hdconv_model_load(self.handle, ptr, buf.size))

    def train(self, X, y, epochs=200, batch=512, lr=1e-3, seed=0) -> float:
        X, xp = _fp(X)
        y, yp = _fp(y)
        loss = ctypes.c_float(0)
        _L.check(_L.lib().hdconv_model_train(self.handle, xp, yp, len(y), int(epochs), int(batch), float(lr),
                                             int(seed), ctypes.byref(loss)))
        return float(loss.value)

    def predict(self, X) -> np.ndarray:
        X, xp = _fp(X)
        n = X.shape[0]
        out, op = _fp(np.zeros(n))
        _L.check(_L.lib().hdconv_model_predict(self.handle, xp, n, op))
        return out

    def grad(self, X, y):
        X, xp = _fp(X)
        y, yp = _fp(y)
        n_net = self.params().size - (2 * NF + 2)
        g, gp = _fp(np.zeros(n_net))
        loss = ctypes.c_float(0)
        _L.check(_L.lib().hdconv_model_grad(self.handle, xp, yp, len(y), gp, ctypes.byref(loss)))
        return g, float(loss.value)

    def save(self, path: str, meta=None):
        """Parameters as little-endian float32 (path) plus a JSON header (path + '.json')."""
        p = self.params()
        p.astype("<f4").tofile(path)
        hdr = {"hidden": self.hidden, "nfeatures": NF, "nparams": int(p.size),
               "layout": "W1,b1,W2,b2,W3,b3,W4,b4,xmean,xstd,ymean,ystd"}
        hdr.update(meta or {})
        with open(path + ".json", "w") as fh:
            json.dump(hdr, fh, indent=1)

    @classmethod
    def load_file(cls, path: str) -> "CostModel":
        with open(path + ".json") as fh:
            hdr = json.load(fh)
        if int(hdr.get("nfeatures", -1)) != NF:
            raise ValueError("%s was trained on %s features; this library computes %d" % (path, hdr.get("nfeatures"), NF))
        m = cls(hidden=int(hdr["hidden"]))
        m.load(np.fromfile(path, dtype="<f4"))
        return m

    def close(self):
        h, self.handle = getattr(self, "handle", None), None
        if h:
            _L.lib().hdconv_model_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


TRAINED_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "trained", "picker_mlp.f32")


def load_default_model() -> "CostModel":
    """The picker trained on this library's own autotuner timings (shipped
    with the package as trained/picker_mlp.f32)."""
    if not os.path.exists(TRAINED_MODEL):
        raise FileNotFoundError("no trained cost model at " + TRAINED_MODEL)
    return CostModel.load_file(TRAINED_MODEL)


def geometries(count: int, seed: int, A_choices=(2, 3), mix=(0.60, 0.25, 0.15), l1=(256, 1 << 22),
               l2=(16, 4096), l3=(8, 384), flag_mix=(0.0, 0.0)):
    """Seeded geometries of the cost-model workload: 1D L log-uniform in l1,
    2D square L x L with L log-uniform in l2, 3D cubes with L log-uniform in
    l3 (fractions `mix`); A drawn from A_choices; M = A L per dimension.
    With ``flag_mix`` = (c, h), a fraction c are centered and h Hermitian
    (odd outer extents; M the least padding of each, as the library
    defines it); (0, 0) draws exactly the unflagged sequence."""
    from .hdconv import centered_min_padding, hermitian_min_padding
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        u = rng.random()
        dims = 1 if u < mix[0] else (2 if u < mix[0] + mix[1] else 3)
        lo, hi = {1: l1, 2: l2, 3: l3}[dims]
        L = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        A = int(A_choices[rng.integers(len(A_choices))])
        g = {"L": [L] * dims, "M": [A * L] * dims, "A": A, "flags": 0}
        if flag_mix[0] > 0 or flag_mix[1] > 0:
            f = rng.random()
            if f < flag_mix[0]:
                g["flags"] = _L.PLAN_CENTERED
                g["M"] = [centered_min_padding(L, A)] * dims
            elif f < flag_mix[0] + flag_mix[1]:
                Lo = L | 1  # outer extents of a Hermitian problem are odd
                g["flags"] = _L.PLAN_HERMITIAN
                g["L"] = [Lo] * (dims - 1) + [L]
                g["M"] = [centered_min_padding(Lo, A)] * (dims - 1) + [hermitian_min_padding(L, A)]
        out.append(g)
    return out


def regret(t_pick: float, t_best: float) -> float:
    return t_pick / t_best - 1.0
