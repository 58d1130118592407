"""FP64 CPU oracle for hybrid-dealiased complex convolutions.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_2303_17510_amd``) never imports it, and it imports nothing from the
product: the two share no code, kernels, headers, tables or helpers.  Inputs
reach both sides from the seeded generators, which hold none of the method's
arithmetic.

Functions (Murasko & Bowman, arXiv 2303.17510):

* :func:`conv_direct` -- O1, the definition of Sec. 2 (and its d-dimensional
  form, Sec. 5) evaluated as a compensated direct sum: the first ``L`` outputs
  per dimension of the linear convolution of the ``A`` inputs (``mult`` is the
  pointwise product of the ``A`` transforms, ``B = 1``).  Optional ``idx``
  evaluates only selected flat output indices (for large sizes).
* :func:`conv_explicit` -- O2, explicit zero padding to a power of two
  ``N' >= A(L-1)+1`` (the minimal padding of Sec. 2), this package's own FFT,
  pointwise product, inverse, truncation to the first ``L`` per dimension.
* :func:`conv_centered_direct` -- OC, centered convolution (the paper's
  centered case in one dimension, Sec. 5 per dimension): an extent-``L`` array
  holds centered indices ``-H .. L-1-H`` (``H = floor(L/2)``) at positions
  ``c + H``, and ``h_c = sum f_{c1} g_{c-c1}`` over the in-range ``c1``
  (``A = 3``: the triple sum), evaluated as compensated direct sums.
* :func:`conv_centered_explicit` -- OC by O2: entries ``(A-1)H ..
  (A-1)H+L-1`` per dimension of the explicitly padded linear convolution.
* :func:`conv_hermitian_direct` / :func:`conv_hermitian_explicit` -- OH,
  Hermitian convolutions (1D): arrays of ``Lh`` entries hold ``f_0 ..
  f_{Lh-1}`` of the centered Hermitian array ``f_{-j} = conj(f_j)`` (``f_0``
  taken real); the result is the centered convolution of the expanded arrays
  at ``c = 0 .. Lh-1`` (:func:`hermitian_expand` does the expansion).
* :func:`conv_quadratic` -- general convolutions whose multiplication
  operator is a quadratic form per output (``B`` outputs), through the
  pairwise convolutions above (linearity of the DFT).
* :func:`padded_dft` -- the padded DFT of Sec. 2,
  ``F_k = sum_{j<L} zeta_N^{kj} f_j`` with ``zeta_N = exp(+2 pi i/N)``.
* :func:`fft` / :func:`fft_nd` -- the unnormalised transform
  ``X_k = sum_j x_j exp(sign 2 pi i jk/N)`` (power-of-two sizes).

Parity status: every function here is pinned by ``tests/test_oracle.py``
against closed forms, library routines and invariants.  None is "parity
unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "conv.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_dblp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False, out: str | None = None, defines=()) -> str:
    """Compile ``conv.c`` into ``liboracle.so`` with gcc (FP64, OpenMP)."""
    target = out or _LIB
    if force or out or not os.path.exists(target) or os.path.getmtime(target) < os.path.getmtime(_SRC):
        tmp = target + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
               "-fno-fast-math", "-ffp-contract=off"] + ["-D" + d for d in defines] + \
              [_SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, target)
    return target


def _bind(path: str):
    lib = ctypes.CDLL(path)
    lib.oracle_direct2.argtypes = [_dblp, _dblp, ctypes.c_int, _i64p, _i64p, ctypes.c_int64, _dblp]
    lib.oracle_fft.argtypes = [_dblp, ctypes.c_int64, ctypes.c_int]
    lib.oracle_fft_nd.argtypes = [_dblp, ctypes.c_int, _i64p, ctypes.c_int]
    lib.oracle_explicit.argtypes = [ctypes.POINTER(_dblp), ctypes.c_int, ctypes.c_int, _i64p, _dblp]
    lib.oracle_explicit_centered.argtypes = [ctypes.POINTER(_dblp), ctypes.c_int, ctypes.c_int, _i64p, _dblp]
    lib.oracle_direct_centered.argtypes = [_dblp, _i64p, _i64p, _dblp, _i64p, _i64p, ctypes.c_int, _i64p, _i64p,
                                           _i64p, ctypes.c_int64, _dblp]
    lib.oracle_hermitian_expand.argtypes = [_dblp, ctypes.c_int64, _dblp]
    lib.oracle_hermitian_expand_nd.argtypes = [_dblp, _i64p, ctypes.c_int64, _dblp]
    lib.oracle_padded_dft.argtypes = [_dblp, ctypes.c_int64, ctypes.c_int64, _i64p, ctypes.c_int64, _dblp]
    lib.oracle_num_threads.argtypes = []
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    for fn in ("oracle_direct2", "oracle_fft", "oracle_fft_nd", "oracle_explicit", "oracle_explicit_centered",
               "oracle_direct_centered", "oracle_hermitian_expand", "oracle_hermitian_expand_nd",
               "oracle_padded_dft", "oracle_num_threads",
               "oracle_set_num_threads"):
        getattr(lib, fn).restype = ctypes.c_int
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = _bind(_LIB)
    return _lib


def use_library(path: str | None) -> None:
    """Bind the functions to another build of ``conv.c`` (``None``: the default).

    Only the pin-strength test uses this, to load builds with planted
    mistakes."""
    global _lib
    with _lock:
        _lib = None
    if path is not None:
        global _LIB
        saved = _LIB
        try:
            _LIB = path
            with _lock:
                _lib = _bind(path)
        finally:
            _LIB = saved


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_dblp)


def _ip(a: np.ndarray):
    return a.ctypes.data_as(_i64p)


def num_threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> int:
    """Set the OpenMP threads of the following oracle calls; returns the count."""
    return int(_load().oracle_set_num_threads(int(n)))


def _direct2(f: np.ndarray, g: np.ndarray, idx: np.ndarray | None) -> np.ndarray:
    shape = f.shape
    L = np.array(shape, dtype=np.int64)
    if idx is None:
        idx = np.arange(f.size, dtype=np.int64)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).ravel())
    out = np.empty(idx.size, dtype=np.complex128)
    rc = _load().oracle_direct2(_dp(f), _dp(g), len(shape), _ip(L), _ip(idx), idx.size, _dp(out))
    if rc != 0:
        raise ValueError("oracle_direct2 failed (%d)" % rc)
    return out


def conv_direct(inputs, idx=None) -> np.ndarray:
    """O1: first ``L`` outputs (per dimension) of the linear convolution.

    ``inputs`` is a list of ``A`` (2 or 3) complex arrays of one shape
    (1, 2 or 3 dimensions, row-major).  With ``idx`` (flat indices) only those
    outputs are returned (A = 2 only); otherwise the full array.
    """
    ins = [_c128(x) for x in inputs]
    if len(ins) not in (2, 3) or any(x.shape != ins[0].shape for x in ins):
        raise ValueError("need 2 or 3 inputs of one shape")
    if ins[0].ndim not in (1, 2, 3):
        raise ValueError("1 to 3 dimensions")
    if len(ins) == 2:
        out = _direct2(ins[0], ins[1], idx)
        return out if idx is not None else out.reshape(ins[0].shape)
    if idx is not None:
        raise ValueError("sampled outputs are for A = 2")
    # A = 3: indices are non-negative, so truncating the first product to the
    # output box loses nothing the second product needs.
    t = _direct2(ins[0], ins[1], None).reshape(ins[0].shape)
    return _direct2(t, ins[2], None).reshape(ins[0].shape)


def conv_explicit(inputs) -> np.ndarray:
    """O2: explicitly zero-padded FFT convolution, first ``L`` per dimension."""
    ins = [_c128(x) for x in inputs]
    if len(ins) not in (2, 3) or any(x.shape != ins[0].shape for x in ins):
        raise ValueError("need 2 or 3 inputs of one shape")
    shape = ins[0].shape
    L = np.array(shape, dtype=np.int64)
    ptrs = (_dblp * len(ins))(*[_dp(x) for x in ins])
    out = np.empty(shape, dtype=np.complex128)
    rc = _load().oracle_explicit(ptrs, len(ins), len(shape), _ip(L), _dp(out))
    if rc != 0:
        raise ValueError("oracle_explicit failed (%d)" % rc)
    return out


def _direct_centered(a: np.ndarray, ha, b: np.ndarray, hb, lo, ho, idx) -> np.ndarray:
    dims = a.ndim
    La = np.array(a.shape, dtype=np.int64)
    Lb = np.array(b.shape, dtype=np.int64)
    Lo = np.array(lo, dtype=np.int64)
    Ha = np.array(ha, dtype=np.int64)
    Hb = np.array(hb, dtype=np.int64)
    Ho = np.array(ho, dtype=np.int64)
    if idx is None:
        idx = np.arange(int(np.prod(Lo)), dtype=np.int64)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).ravel())
    out = np.empty(idx.size, dtype=np.complex128)
    rc = _load().oracle_direct_centered(_dp(a), _ip(La), _ip(Ha), _dp(b), _ip(Lb), _ip(Hb), dims, _ip(Lo), _ip(Ho),
                                        _ip(idx), idx.size, _dp(out))
    if rc != 0:
        raise ValueError("oracle_direct_centered failed (%d)" % rc)
    return out


def conv_centered_direct(inputs, idx=None) -> np.ndarray:
    """OC: centered convolution of ``A`` (2 or 3) arrays of one shape.

    Position ``i`` of a dimension of extent ``L`` holds centered index
    ``i - floor(L/2)``, for the inputs and the output alike; the output is
    ``h_c = sum_{c1 + ... + cA = c} f_{c1} ... `` over in-range indices.  With
    ``idx`` (flat output positions) only those outputs are returned.
    """
    ins = [_c128(x) for x in inputs]
    if len(ins) not in (2, 3) or any(x.shape != ins[0].shape for x in ins):
        raise ValueError("need 2 or 3 inputs of one shape")
    if ins[0].ndim not in (1, 2, 3):
        raise ValueError("1 to 3 dimensions")
    shape = ins[0].shape
    H = [n // 2 for n in shape]
    if len(ins) == 2:
        out = _direct_centered(ins[0], H, ins[1], H, shape, H, idx)
    else:
        # the full centered product of the first two factors: extent 2L-1,
        # centered indices -2H .. 2(L-1-H) at positions c + 2H
        full = [2 * n - 1 for n in shape]
        H2 = [2 * h for h in H]
        t = _direct_centered(ins[0], H, ins[1], H, full, H2, None).reshape(full)
        out = _direct_centered(t, H2, ins[2], H, shape, H, idx)
    return out if idx is not None else out.reshape(shape)


def conv_centered_explicit(inputs) -> np.ndarray:
    """OC by explicit zero padding: the centered window of the linear convolution."""
    ins = [_c128(x) for x in inputs]
    if len(ins) not in (2, 3) or any(x.shape != ins[0].shape for x in ins):
        raise ValueError("need 2 or 3 inputs of one shape")
    shape = ins[0].shape
    L = np.array(shape, dtype=np.int64)
    ptrs = (_dblp * len(ins))(*[_dp(x) for x in ins])
    out = np.empty(shape, dtype=np.complex128)
    rc = _load().oracle_explicit_centered(ptrs, len(ins), len(shape), _ip(L), _dp(out))
    if rc != 0:
        raise ValueError("oracle_explicit_centered failed (%d)" % rc)
    return out


def hermitian_expand(f) -> np.ndarray:
    """The centered array that a stored Hermitian half stands for.

    1D: ``Lh`` entries ``f_0 .. f_{Lh-1}`` give ``f_{-(Lh-1)} .. f_{Lh-1}``
    with ``f_{-j} = conj(f_j)`` and ``f_0`` real.  2D/3D: a box whose last
    axis holds ``c = 0 .. Lh-1`` and whose outer axes (odd extents) hold
    centered signed indices gives the box with ``c = -(Lh-1) .. Lh-1``,
    ``F(k, -c) = conj F(-k, c)`` and the ``c = 0`` plane replaced by its
    Hermitian part."""
    f = _c128(f)
    if f.ndim <= 1:
        f = f.ravel()
        out = np.empty(2 * f.size - 1, dtype=np.complex128)
        rc = _load().oracle_hermitian_expand(_dp(f), f.size, _dp(out))
        if rc != 0:
            raise ValueError("oracle_hermitian_expand failed (%d)" % rc)
        return out
    if f.ndim > 3:
        raise ValueError("1 to 3 dimensions")
    outer = list(f.shape[:-1])
    n = np.array(([1] * (2 - len(outer))) + outer, dtype=np.int64)
    Lh = f.shape[-1]
    out = np.empty(tuple(outer) + (2 * Lh - 1,), dtype=np.complex128)
    rc = _load().oracle_hermitian_expand_nd(_dp(f), _ip(n), Lh, _dp(out))
    if rc != 0:
        raise ValueError("oracle_hermitian_expand_nd failed (%d): outer extents must be odd" % rc)
    return out


def _herm_inputs(inputs):
    ins = [_c128(x) for x in inputs]
    if len(ins) not in (2, 3) or any(x.shape != ins[0].shape for x in ins):
        raise ValueError("need 2 or 3 inputs of one shape")
    return ins


def conv_hermitian_direct(inputs, idx=None) -> np.ndarray:
    """OH: Hermitian convolution of ``A`` (2 or 3) stored halves of one shape
    (1D, or 2D/3D with the Hermitian last axis); returns the stored half of
    the result (or the flat entries ``idx`` of it)."""
    ins = _herm_inputs(inputs)
    shape = ins[0].shape if ins[0].ndim > 1 else (ins[0].size,)
    Lh = shape[-1]
    full = [hermitian_expand(x) for x in ins]
    fshape = full[0].shape
    n = int(np.prod(shape))
    pos = np.arange(n, dtype=np.int64) if idx is None else np.asarray(idx, dtype=np.int64).ravel()
    if np.any(pos < 0) or np.any(pos >= n):
        raise ValueError("idx out of range")
    # stored entry (outer..., c) is entry (outer..., c + Lh - 1) of the expanded box
    outer, c = np.divmod(pos, Lh)
    fpos = outer * fshape[-1] + c + (Lh - 1)
    out = conv_centered_direct(full, idx=fpos)
    return out if idx is not None else out.reshape(shape)


def conv_hermitian_explicit(inputs) -> np.ndarray:
    """OH by explicit zero padding of the expanded arrays."""
    ins = _herm_inputs(inputs)
    Lh = ins[0].shape[-1] if ins[0].ndim > 1 else ins[0].size
    full = conv_centered_explicit([hermitian_expand(x) for x in ins])
    return full[..., Lh - 1:]


def conv_quadratic(inputs, coef, kind="plain") -> list:
    """General convolution with a quadratic multiplication operator (Sec. 2:
    ``mult`` maps the ``A`` transforms to ``B`` outputs pointwise): output b
    has transform ``sum_{i <= j} coef[b][i][j] F_i F_j``, so by linearity of
    the DFT it is ``sum_{i <= j} coef[b][i][j] (f_i * f_j)`` with ``*`` the
    convolution of ``kind`` ("plain": first L outputs, "centered",
    "hermitian").  ``coef`` is B x A x A (entries below the diagonal unused)."""
    ins = [_c128(x) for x in inputs]
    A = len(ins)
    c = np.asarray(coef, dtype=np.float64)
    if c.ndim != 3 or c.shape[1:] != (A, A):
        raise ValueError("coef must be B x A x A")
    pair = {"plain": conv_direct, "centered": conv_centered_direct, "hermitian": conv_hermitian_direct}[kind]
    cache = {}
    outs = []
    for b in range(c.shape[0]):
        acc = np.zeros(pair([ins[0], ins[0]]).shape, dtype=np.complex128)
        for i in range(A):
            for j in range(i, A):
                if c[b, i, j] != 0:
                    if (i, j) not in cache:
                        cache[(i, j)] = pair([ins[i], ins[j]])
                    acc += c[b, i, j] * cache[(i, j)]
        outs.append(acc)
    return outs


def padded_dft(f, N: int, ks) -> np.ndarray:
    """Padded DFT ``F_k = sum_{j<L} exp(2 pi i k j / N) f_j`` at the given ``ks``."""
    f = _c128(f).ravel()
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64).ravel())
    out = np.empty(ks.size, dtype=np.complex128)
    rc = _load().oracle_padded_dft(_dp(f), f.size, int(N), _ip(ks), ks.size, _dp(out))
    if rc != 0:
        raise ValueError("oracle_padded_dft failed (%d)" % rc)
    return out


def fft(x, sign: int = +1) -> np.ndarray:
    """Unnormalised 1D transform with kernel ``exp(sign 2 pi i jk/N)``."""
    y = _c128(x).copy()
    rc = _load().oracle_fft(_dp(y), y.size, int(sign))
    if rc != 0:
        raise ValueError("oracle_fft failed (%d)" % rc)
    return y


def fft_nd(x, sign: int = +1) -> np.ndarray:
    """Unnormalised n-D transform (row-column), power-of-two extents."""
    y = _c128(x).copy()
    N = np.array(y.shape, dtype=np.int64)
    rc = _load().oracle_fft_nd(_dp(y), y.ndim, _ip(N), int(sign))
    if rc != 0:
        raise ValueError("oracle_fft_nd failed (%d)" % rc)
    return y


def rel_l2(y, ref) -> float:
    """Relative L2 error ``||y - ref|| / ||ref||`` computed in FP64."""
    y = np.asarray(y, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(y - ref) / (den if den > 0 else 1.0))
