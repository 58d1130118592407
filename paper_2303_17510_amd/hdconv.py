"""Python front end of libhdconv: plans and execution on torch tensors.

Only marshalling lives here.  Tensors supply device pointers, the current
torch stream supplies the hipStream_t, and the library's kernels do all the
arithmetic.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

from . import _lib as _L

_METHODS = {"auto": _L.METHOD_AUTO, "hybrid": _L.METHOD_HYBRID, "explicit": _L.METHOD_EXPLICIT}
_VARIANTS = {None: 0, "auto": 0, "fused": 1, "multipass": 2, "outer": 3}


def _torch():
    import torch
    return torch


def dtype_code(dtype) -> int:
    torch = _torch()
    if dtype in (torch.complex64, "c64", "complex64"):
        return _L.C64
    if dtype in (torch.complex128, "c128", "complex128"):
        return _L.C128
    raise ValueError("dtype must be complex64 or complex128")


def _tup(x, dims, default=0):
    if x is None:
        return (default,) * dims
    if isinstance(x, int):
        return (x,) * dims
    x = tuple(int(v) for v in x)
    if len(x) != dims:
        raise ValueError("expected %d values" % dims)
    return x


def geometry(L: int, M: int, m: int, p_min: int = 0, force_inner: bool = False) -> dict:
    """The paper's (p, n, q) for one dimension and a given m (host only)."""
    out = _L.DimInfo()
    _L.check(_L.lib().hdconv_geometry(int(L), int(M), int(m), int(p_min), int(bool(force_inner)),
                                       ctypes.byref(out)))
    return {"L": out.L, "M": out.M, "m": out.m, "p": out.p, "n": out.n, "q": out.q,
            "variant": _L.VARIANT_NAMES[out.variant]}


def min_padding(L: int, A: int = 2, centered: bool = False, hermitian: bool = False) -> int:
    """Least M the library accepts for one dimension of extent L with A
    factors per product: A(L-1)+1, or the centered / Hermitian minimum."""
    flags = _L.PLAN_HERMITIAN if hermitian else (_L.PLAN_CENTERED if centered else 0)
    out = ctypes.c_int64()
    _L.check(_L.lib().hdconv_min_padding(int(L), int(A), flags, ctypes.byref(out)))
    return int(out.value)


def centered_min_padding(L: int, A: int = 2) -> int:
    """Least M of a centered dimension (indices -H .. L-1-H, H = L // 2)."""
    return min_padding(L, A, centered=True)


def hermitian_min_padding(L: int, A: int = 2) -> int:
    """Least M of a Hermitian dimension of nominal length L."""
    return min_padding(L, A, hermitian=True)


def geometry_centered(L: int, M: int, m: int, p_min: int = 0, force_inner: bool = False,
                      hermitian: bool = False) -> dict:
    """The library's centered (or Hermitian) geometry for one dimension and m."""
    out = _L.DimInfo()
    flags = _L.PLAN_HERMITIAN if hermitian else _L.PLAN_CENTERED
    _L.check(_L.lib().hdconv_geometry_ex(int(L), int(M), int(m), int(p_min), int(bool(force_inner)), flags,
                                          ctypes.byref(out)))
    return {"L": out.L, "M": out.M, "m": out.m, "p": out.p, "n": out.n, "q": out.q,
            "variant": _L.VARIANT_NAMES[out.variant], "centered": out.centered,
            "span": int(_L.lib().hdconv_centered_span(int(out.L), int(m)))}


class Plan:
    """A planned convolution of ``A`` inputs of shape ``L`` padded to ``M``.

    ``method``: "hybrid" (default) or "explicit" (materialised zero padding).
    ``m``, ``p``, ``D``, ``variant`` force per-dimension choices (None: the
    planner decides).  ``host_only`` plans geometry without device memory.
    ``centered``: arrays hold the indices -L//2 .. L-1-L//2 (index 0 at
    position L//2) and the result is the centered convolution; ``M`` then
    defaults to the centered minimum (3L/2 for A = 2, even L).
    ``copies`` (C) and ``dist``: each array holds C copies of the problem,
    ``dist`` words apart (default: dense, tensors of shape ``(C, *shape)``;
    with ``dist`` a flat tensor of at least ``(C-1) dist + n`` words).
    ``strides`` (2D/3D): element strides of the outer dimensions (padded
    rows); the tensors are then flat, of at least ``(C-1) dist + L[0]
    strides[0]`` words.
    ``hermitian``: the last dimension holds the ``ceil(L/2)`` non-negative
    indices of a Hermitian centered array (``f_{-c} = conj f_c``; 2D/3D:
    ``F(k, -c) = conj F(-k, c)`` with centered outer dimensions of odd
    extent), and so does the output; ``M`` defaults to the minimum padding.
    ``no_workspace``: the plan allocates no workspace and runs only through
    :meth:`execute_noalloc` (the library's static device scratch).
    ``conj_pairs``: the inner form's forward column pass computes residues v
    and n - v together (conjugate symmetry) where a block holds all residues.
    ``accumulate_output``: residue blocks add into the output array instead
    of an FP64 accumulation buffer (out of place only).
    ``mult="quadratic"`` with real coefficients ``coef`` of shape
    ``(B, A, A)``: B outputs, output b = sum_{i <= j} coef[b][i][j] F_i F_j
    pointwise in transform space (entries below the diagonal unused); the
    padding rule is that of two factors.
    """

    def __init__(self, L: Sequence[int], M: Sequence[int] | None = None, A: int = 2, B: int = 1,
                 dtype="c64", method: str = "hybrid", m=None, p=None, D=None, variant=None,
                 host_only: bool = False, E_m=None, E_p=None, S=None, rows_per_block=None,
                 twiddles=None, tuner: str = "heuristic", model=None, tune_reps: int = 0, margin: float = 0.0,
                 db_path: str | None = None, centered: bool = False, hermitian: bool = False,
                 copies: int = 1, dist: int = 0, strides=None, mult: str = "product", coef=None,
                 no_workspace: bool = False, conj_pairs: bool = True, accumulate_output: bool = False):
        L = (int(L),) if isinstance(L, int) else tuple(int(v) for v in L)
        dims = len(L)
        if mult not in ("product", "quadratic"):
            raise ValueError("mult must be 'product' or 'quadratic'")
        F = 2 if mult == "quadratic" else A  # factors per output term
        if M is None:
            M = tuple(hermitian_min_padding(l, F) if (hermitian and d == dims - 1) else
                      (centered_min_padding(l, F) if (centered or hermitian) else F * l) for d, l in enumerate(L))
        M = (int(M),) if isinstance(M, int) else tuple(int(v) for v in M)
        self.L, self.M, self.A, self.B, self.dims = L, M, A, B, dims
        self.dtype_code = dtype_code(dtype)
        opt = _L.Options()
        _L.lib().hdconv_options_init(ctypes.byref(opt))
        opt.method = _METHODS[method]
        opt.flags = ((_L.PLAN_HOST_ONLY if host_only else 0) | (_L.PLAN_CENTERED if centered else 0) |
                     (_L.PLAN_HERMITIAN if hermitian else 0) | (_L.PLAN_NO_WORKSPACE if no_workspace else 0) |
                     (_L.PLAN_ACCUMULATE_OUTPUT if accumulate_output else 0))
        self.centered, self.hermitian = bool(centered), bool(hermitian)
        opt.conj_pairs = 0 if conj_pairs else -1
        # shape of the arrays passed in and out
        self.io_shape = L[:-1] + ((L[-1] + 1) // 2,) if hermitian else L
        self.copies, self.dist = int(copies), int(dist)
        opt.copies = self.copies
        opt.dist = self.dist
        self.mult = mult
        self._coef = None
        if mult == "quadratic":
            if coef is None:
                raise ValueError("a quadratic operator needs coef of shape (B, A, A)")
            flat = [float(coef[b][i][j]) for b in range(B) for i in range(A) for j in range(A)]
            self._coef = (ctypes.c_double * len(flat))(*flat)
            opt.mult = _L.MULT_QUADRATIC
            opt.mult_coef = ctypes.cast(self._coef, ctypes.POINTER(ctypes.c_double))
        self.strides = tuple(int(v) for v in strides) if strides else ()
        for d, v in enumerate(self.strides[:2]):
            opt.stride[d] = v
        # words one copy spans (strided: the first dimension's stride times its extent)
        if self.strides:
            self.span = self.io_shape[0] * self.strides[0]
        else:
            self.span = 1
            for v in self.io_shape:
                self.span *= v
        if dims > 3 or len(M) != dims:
            raise ValueError("L and M need 1 to 3 matching dimensions")
        for d, v in enumerate(_tup(m, dims)):
            opt.m[d] = v
        for d, v in enumerate(_tup(p, dims)):
            opt.p[d] = v
        for d, v in enumerate(_tup(D, dims)):
            opt.D[d] = v
        opt.tuner = {"heuristic": _L.TUNER_HEURISTIC, "exhaustive": _L.TUNER_EXHAUSTIVE,
                     "model": _L.TUNER_MODEL}[tuner]
        opt.tune_reps = int(tune_reps)
        opt.margin = float(margin)
        if tuner == "model" and model is None:
            from .tune import load_default_model
            model = load_default_model()
        self._model = model
        opt.model = ctypes.c_void_p(model.handle if model is not None else None)
        self._db = db_path.encode() if db_path else None
        opt.db_path = self._db
        for name, val in (("E_m", E_m), ("E_p", E_p), ("S", S), ("rows_per_block", rows_per_block),
                          ("twiddles", twiddles)):
            for d, v in enumerate(_tup(val, dims)):
                getattr(opt, name)[d] = v
        vs = variant if isinstance(variant, (list, tuple)) else [variant] * dims
        for d, v in enumerate(vs):
            opt.variant[d] = _VARIANTS[v]
        Ls = (ctypes.c_int64 * 3)(*(list(L) + [1] * (3 - dims)))
        Ms = (ctypes.c_int64 * 3)(*(list(M) + [1] * (3 - dims)))
        h = _L.lib().hdconv_plan_ex(Ls, Ms, A, B, dims, self.dtype_code, ctypes.byref(opt))
        if not h:
            code, msg = _L.last_error()
            raise _L.HdconvError(code, msg)
        self._h = h
        self.host_only = host_only

    # -- info -----------------------------------------------------------
    def info(self) -> dict:
        out = _L.PlanInfo()
        _L.check(_L.lib().hdconv_plan_info(self._h, ctypes.byref(out)))
        dims = []
        for d in range(out.dims):
            di = out.dim[d]
            dims.append({"L": di.L, "M": di.M, "m": di.m, "p": di.p, "n": di.n, "q": di.q, "D": di.D,
                         "variant": _L.VARIANT_NAMES[di.variant], "E_m": di.E_m, "E_p": di.E_p,
                         "S": di.S, "rows_per_block": di.rows_per_block, "tw_m": di.tw_m, "tw_p": di.tw_p,
                         "centered": bool(di.centered), "hermitian": di.centered == 2})
        return {"dims": dims, "A": out.A, "B": out.B, "dtype": "c64" if out.dtype == 0 else "c128",
                "method": {1: "hybrid", 2: "explicit"}.get(out.method, "auto"),
                "npad": list(out.npad)[: out.dims], "workspace_bytes": out.workspace_bytes,
                "table_bytes": out.table_bytes, "compulsory_bytes": out.compulsory_bytes,
                "traffic_bytes": out.traffic_bytes, "launches": out.launches,
                "tuner": {0: "heuristic", 1: "exhaustive", 2: "model"}.get(out.tuner, "?"),
                "tuned_candidates": out.tuned_candidates, "timed_candidates": out.timed_candidates,
                "tuned_ms": out.tuned_ms}

    # -- execution --------------------------------------------------------
    def _check_tensor(self, t, name):
        torch = _torch()
        want = torch.complex64 if self.dtype_code == _L.C64 else torch.complex128
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA (HIP) tensor" % name)
        if (self.copies > 1 and self.dist) or self.strides:
            need = (self.copies - 1) * (self.dist or self.span) + self.span
            if t.dtype != want or t.dim() != 1 or t.numel() < need or not t.is_contiguous():
                raise ValueError("%s must be a contiguous flat %s tensor of at least %d words" % (name, want, need))
            return
        shape = ((self.copies,) + self.io_shape) if self.copies > 1 else self.io_shape
        if t.dtype != want or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor of shape %s (got %s %s)"
                             % (name, want, shape, t.dtype, tuple(t.shape)))

    def execute(self, inputs, out, stream=None):
        """Run asynchronously on ``stream`` (default: torch's current stream).
        ``out``: one tensor, or a sequence of B tensors (B > 1)."""
        return self._run(_L.lib().hdconv_execute, inputs, out, stream)

    def execute_noalloc(self, inputs, out, stream=None):
        """As :meth:`execute`, with the library's static device scratch as
        the workspace (hdconv_execute_noalloc: nothing is allocated; calls
        that overlap on one device race on the scratch)."""
        return self._run(_L.lib().hdconv_execute_noalloc, inputs, out, stream)

    def _run(self, fn, inputs, out, stream):
        torch = _torch()
        if len(inputs) != self.A:
            raise ValueError("expected %d inputs" % self.A)
        for i, t in enumerate(inputs):
            self._check_tensor(t, "inputs[%d]" % i)
        outs_t = list(out) if isinstance(out, (list, tuple)) else [out]
        if len(outs_t) != self.B:
            raise ValueError("expected %d outputs" % self.B)
        for b, t in enumerate(outs_t):
            self._check_tensor(t, "out[%d]" % b)
        if stream is None:
            stream = torch.cuda.current_stream(outs_t[0].device)
        ins = (ctypes.c_void_p * self.A)(*[t.data_ptr() for t in inputs])
        outs = (ctypes.c_void_p * self.B)(*[t.data_ptr() for t in outs_t])
        _L.check(fn(self._h, ins, outs, ctypes.c_void_p(stream.cuda_stream)))
        return out

    def profile_begin(self, max_executes: int):
        """Record HIP events around each kernel of the next ``max_executes`` executes."""
        _L.check(_L.lib().hdconv_profile_begin(self._h, int(max_executes)))

    def profile_end(self) -> list:
        """Per-launch-slot timing since :meth:`profile_begin` (waits for the events)."""
        cap = 1024  # launch slots of one execute
        arr = (_L.KernelStat * cap)()
        n = ctypes.c_int(0)
        _L.check(_L.lib().hdconv_profile_end(self._h, arr, cap, ctypes.byref(n)))
        out = []
        for k in range(min(n.value, cap)):
            r = arr[k]
            out.append({"slot": k, "name": r.name.decode(), "launches": r.launches, "total_ms": r.total_ms,
                        "avg_ms": r.total_ms / r.launches if r.launches else float("nan"),
                        "bytes_per_launch": r.bytes_per_launch})
        return out

    def __call__(self, *inputs):
        torch = _torch()
        if self.B == 1:
            return self.execute(inputs, torch.empty_like(inputs[0]))
        return self.execute(inputs, [torch.empty_like(inputs[0]) for _ in range(self.B)])

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            _L.lib().hdconv_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class BatchPlan:
    """Many independent 1D convolutions of uneven length ``Ls`` (each padded to ``Ms``).

    Convolutions with the same planned shape form a group.  Ordinary batches
    with the heuristic tuner run as persistent kernel launches over device
    task tables, one per pass (``grouped=True``, tuned, centered and
    Hermitian batches: one set of launches per group on side streams); each
    execute is one hipGraph launch (from the second execute on, unless
    ``graph=False``).
    """

    def __init__(self, Ls, Ms=None, A: int = 2, B: int = 1, dtype="c64", graph: bool = True,
                 tuner: str = "heuristic", model=None, tune_reps: int = 5, margin: float = 0.05,
                 centered: bool = False, hermitian: bool = False, grouped: bool = False):
        Ls = [int(v) for v in Ls]
        if Ms is None:
            Ms = [hermitian_min_padding(v, A) if hermitian else
                  (centered_min_padding(v, A) if centered else A * v) for v in Ls]
        Ms = [int(v) for v in Ms]
        if len(Ms) != len(Ls):
            raise ValueError("Ls and Ms differ in length")
        self.Ls, self.Ms, self.A, self.B = Ls, Ms, A, B
        self.dtype_code = dtype_code(dtype)
        opt = _L.Options()
        _L.lib().hdconv_options_init(ctypes.byref(opt))
        opt.flags = ((0 if graph else _L.BATCH_NO_GRAPH) | (_L.PLAN_CENTERED if centered else 0) |
                     (_L.PLAN_HERMITIAN if hermitian else 0) | (_L.BATCH_GROUPED if grouped else 0))
        self.centered, self.hermitian = bool(centered), bool(hermitian)
        self.io_lengths = [(v + 1) // 2 for v in Ls] if hermitian else list(Ls)
        opt.tuner = {"heuristic": _L.TUNER_HEURISTIC, "exhaustive": _L.TUNER_EXHAUSTIVE,
                     "model": _L.TUNER_MODEL}[tuner]
        opt.tune_reps = int(tune_reps)
        opt.margin = float(margin)
        if tuner == "model" and model is None:
            from .tune import load_default_model
            model = load_default_model()
        self._model = model
        opt.model = ctypes.c_void_p(model.handle if model is not None else None)
        n = len(Ls)
        h = _L.lib().hdconv_plan_batched((ctypes.c_int64 * n)(*Ls), (ctypes.c_int64 * n)(*Ms), n, A, B, 1,
                                         self.dtype_code, ctypes.byref(opt))
        if not h:
            code, msg = _L.last_error()
            raise _L.HdconvError(code, msg)
        self._h = h

    def groups(self) -> list:
        cap = 256
        arr = (_L.DimInfo * cap)()
        cnt = (ctypes.c_int64 * cap)()
        ng = ctypes.c_int(0)
        _L.check(_L.lib().hdconv_batch_info(self._h, arr, cnt, cap, ctypes.byref(ng)))
        return [{"variant": _L.VARIANT_NAMES[arr[g].variant], "m": arr[g].m, "p": arr[g].p, "n": arr[g].n,
                 "q": arr[g].q, "E_m": arr[g].E_m, "E_p": arr[g].E_p, "S": arr[g].S,
                 "rows_per_block": arr[g].rows_per_block, "count": cnt[g], "Lmax": arr[g].L,
                 "centered": bool(arr[g].centered), "hermitian": arr[g].centered == 2}
                for g in range(min(ng.value, cap))]

    def stats(self) -> dict:
        """Launch shape: persistent (one launch) or grouped, and its sizes."""
        st = _L.BatchStats()
        _L.check(_L.lib().hdconv_batch_stats(self._h, ctypes.byref(st)))
        return {"persistent": bool(st.persistent), "grid": st.grid, "tasks": st.tasks, "lds_bytes": st.lds_bytes,
                "work_bytes": st.work_bytes}

    def bind(self, inputs, outputs) -> "BoundBatch":
        """Validate the tensors once and keep their device pointers: executes
        of the returned object pass the pointer tables straight to the
        library (the tensors must stay alive and in place meanwhile)."""
        torch = _torch()
        n = len(self.Ls)
        if len(inputs) != n or len(outputs) != n:
            raise ValueError("expected %d convolutions" % n)
        want = torch.complex64 if self.dtype_code == _L.C64 else torch.complex128
        ptrs = []
        for i, ins in enumerate(inputs):
            if len(ins) != self.A:
                raise ValueError("convolution %d needs %d inputs" % (i, self.A))
            for t in list(ins) + [outputs[i]]:
                if not t.is_cuda or t.dtype != want or t.numel() != self.io_lengths[i] or not t.is_contiguous():
                    raise ValueError("convolution %d: tensors must be contiguous %s CUDA vectors of length %d"
                                     % (i, want, self.io_lengths[i]))
            ptrs.extend(t.data_ptr() for t in ins)
        ins_c = (ctypes.c_void_p * len(ptrs))(*ptrs)
        outs_c = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outputs])
        return BoundBatch(self, ins_c, outs_c, outputs[0].device, (inputs, outputs))

    def execute(self, inputs, outputs, stream=None):
        """inputs: list (per convolution) of A tensors; outputs: list of tensors."""
        self.bind(inputs, outputs).execute(stream)
        return outputs

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            _L.lib().hdconv_batch_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class BoundBatch:
    """A batched plan with its tensors' pointer tables (see BatchPlan.bind)."""

    def __init__(self, plan, ins_c, outs_c, device, keep):
        self.plan, self._ins, self._outs, self.device, self._keep = plan, ins_c, outs_c, device, keep

    def execute(self, stream=None):
        if stream is None:
            stream = _torch().cuda.current_stream(self.device)
        _L.check(_L.lib().hdconv_execute_batched(self.plan._h, self._ins, self._outs,
                                                 ctypes.c_void_p(stream.cuda_stream)))


def convolve(*inputs, M=None, **kw):
    """One-shot convolution of equal-shape complex CUDA tensors (first L
    outputs; with ``centered`` / ``hermitian`` the centered or Hermitian
    convolution, the tensors then holding the stored halves; with ``copies``
    the leading dimension counts the copies; with ``mult="quadratic"``,
    ``B`` and ``coef``, the list of B outputs)."""
    L = tuple(inputs[0].shape)
    if kw.get("copies", 1) > 1:
        L = L[1:]
    if kw.get("hermitian"):
        # stored halves of Lh entries stand for the odd length 2 Lh - 1
        L = L[:-1] + (2 * L[-1] - 1,)
    with Plan(L, M, A=len(inputs), dtype=inputs[0].dtype, **kw) as p:
        out = p(*inputs)
        import torch
        torch.cuda.current_stream(inputs[0].device).synchronize()
    return out
