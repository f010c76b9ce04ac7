"""Python binding of ``libcomm.so``: contraction-only block-MM (B-CoMM) and
joint-MM (J-CoMM) updates for nonnegative CP and Tucker models under
beta-divergences, on MI355X (gfx950).

This module only marshals arguments: torch tensors on the GPU supply device
pointers and the current HIP stream; every step of the computation runs in the
library's HIP kernels.  The library must have been built
(``python -m paper_2602_14683_amd.build``); importing this module without it
raises an error rather than falling back to anything else.

Entry points (same names as the C ABI in ``include/comm.h``):
``cp_update``, ``tucker_update``, ``jcomm_outer``, ``beta_objective``,
``cp_jcomm_outer_coo``, ``jcomm_outer_batched`` (with :class:`Batch`).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcomm.so")

COMM_OK, COMM_EINVAL, COMM_EUNSUPPORTED, COMM_ENOMEM, COMM_EHIP = 0, 1, 2, 3, 4
COMM_CP, COMM_TUCKER = 0, 1
COMM_FP32 = 0
COMM_BF16 = 1
PRECISIONS = {"fp32": COMM_FP32, "bf16": COMM_BF16}
COMM_BATCH_GRAPH = 1
COMM_BATCH_GROUPED = 2
COMM_CACHE_AUTO = -1

EXPORTED = ["comm_create", "comm_destroy", "comm_last_error", "comm_workspace_bytes", "comm_profile_enable",
            "comm_profile_query", "comm_cp_update",
            "comm_tucker_update", "comm_jcomm_outer", "comm_jcomm_outer_noalloc", "comm_beta_objective",
            "comm_cp_jcomm_outer_coo",
            "comm_jcomm_outer_batched", "comm_coo_plan_create", "comm_coo_plan_destroy",
            "comm_cp_jcomm_outer_coo_plan", "comm_bcomm_sweep_extrap", "comm_jcomm_outer_extrap",
            "comm_cp_update_coo", "comm_beta_objective_coo", "comm_tucker_update_coo",
            "comm_tucker_jcomm_outer_coo", "comm_check", "comm_tune_jcomm", "comm_tune_lookup", "comm_tune_set"]


class CommError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


MAX_NDIM = 5  # COMM_MAX_NDIM
NOALLOC_SCRATCH_BYTES = 64 << 20  # COMM_NOALLOC_SCRATCH_BYTES


class Dense(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("dims", ctypes.c_int64 * MAX_NDIM), ("X", ctypes.c_void_p)]


class Model(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("rank", ctypes.c_int), ("core_dims", ctypes.c_int64 * MAX_NDIM),
                ("factors", ctypes.c_void_p * MAX_NDIM), ("core", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("eps", ctypes.c_double), ("eps_x", ctypes.c_double),
                ("inner_sweeps", ctypes.c_int), ("precision", ctypes.c_int), ("cache_pq", ctypes.c_int),
                ("check_inputs", ctypes.c_int)]


class Coo(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("dims", ctypes.c_int64 * MAX_NDIM), ("nnz", ctypes.c_int64),
                ("idx", ctypes.c_void_p * MAX_NDIM), ("val", ctypes.c_void_p)]


class Extrap(ctypes.Structure):
    _fields_ = [("alpha_nes", ctypes.c_double), ("c", ctypes.c_double), ("delta", ctypes.c_double)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("found", ctypes.c_int), ("cache_pq", ctypes.c_int), ("wshare", ctypes.c_int),
                ("tk_groups", ctypes.c_int), ("cp_tile", ctypes.c_int), ("variants", ctypes.c_int),
                ("ms", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("x", ctypes.POINTER(Dense)), ("model", ctypes.POINTER(Model)), ("opts", ctypes.POINTER(Opts)),
                ("obj_ref_dev", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load ``libcomm.so`` (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2602_14683_amd.build`")
    # torch ships its own HIP runtime; load it first so that the library binds to
    # the same runtime instance (same soname) instead of a second copy.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.comm_create.argtypes = [ctypes.c_int, ctypes.c_size_t, P(ctypes.c_void_p)]
    lib.comm_destroy.argtypes = [ctypes.c_void_p]
    lib.comm_last_error.restype = ctypes.c_char_p
    lib.comm_workspace_bytes.argtypes = [P(Dense), P(Model), P(Opts), ctypes.c_int]
    lib.comm_workspace_bytes.restype = ctypes.c_size_t
    lib.comm_cp_update.argtypes = [ctypes.c_void_p, P(Dense), P(Model), ctypes.c_int, P(Opts), ctypes.c_void_p]
    lib.comm_tucker_update.argtypes = [ctypes.c_void_p, P(Dense), P(Model), ctypes.c_int, P(Opts), ctypes.c_void_p]
    lib.comm_jcomm_outer.argtypes = [ctypes.c_void_p, P(Dense), P(Model), P(Opts), ctypes.c_void_p, ctypes.c_void_p]
    lib.comm_jcomm_outer_noalloc.argtypes = [ctypes.c_void_p, P(Dense), P(Model), P(Opts), ctypes.c_void_p,
                                             ctypes.c_void_p]
    lib.comm_beta_objective.argtypes = [ctypes.c_void_p, P(Dense), P(Model), P(Opts), ctypes.c_void_p,
                                        ctypes.c_void_p]
    lib.comm_cp_jcomm_outer_coo.argtypes = [ctypes.c_void_p, P(Coo), P(Model), P(Opts), ctypes.c_void_p,
                                            ctypes.c_void_p]
    lib.comm_jcomm_outer_batched.argtypes = [ctypes.c_void_p, P(Problem), ctypes.c_int, ctypes.c_int,
                                             ctypes.c_void_p]
    lib.comm_coo_plan_create.argtypes = [ctypes.c_void_p, P(Coo), P(ctypes.c_void_p), ctypes.c_void_p]
    lib.comm_coo_plan_destroy.argtypes = [ctypes.c_void_p]
    lib.comm_cp_jcomm_outer_coo_plan.argtypes = [ctypes.c_void_p, ctypes.c_void_p, P(Model), P(Opts),
                                                 ctypes.c_void_p, ctypes.c_void_p]
    lib.comm_bcomm_sweep_extrap.argtypes = [ctypes.c_void_p, P(Dense), P(Model), P(Model), P(Opts), P(Extrap),
                                            ctypes.c_void_p, ctypes.c_void_p]
    lib.comm_jcomm_outer_extrap.argtypes = [ctypes.c_void_p, P(Dense), P(Model), P(Model), P(Opts), P(Extrap),
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.comm_cp_update_coo.argtypes = [ctypes.c_void_p, P(Coo), P(Model), ctypes.c_int, P(Opts), ctypes.c_void_p]
    lib.comm_beta_objective_coo.argtypes = [ctypes.c_void_p, P(Coo), P(Model), P(Opts), ctypes.c_void_p,
                                            ctypes.c_void_p]
    lib.comm_tucker_update_coo.argtypes = [ctypes.c_void_p, P(Coo), P(Model), ctypes.c_int, P(Opts),
                                           ctypes.c_void_p]
    lib.comm_tucker_jcomm_outer_coo.argtypes = [ctypes.c_void_p, P(Coo), P(Model), P(Opts), ctypes.c_void_p,
                                                ctypes.c_void_p]
    lib.comm_check.argtypes = [ctypes.c_void_p]
    lib.comm_tune_jcomm.argtypes = [ctypes.c_void_p, P(Dense), P(Model), P(Opts), ctypes.c_int, P(ctypes.c_int),
                                    P(ctypes.c_double), ctypes.c_void_p]
    lib.comm_tune_lookup.argtypes = [ctypes.c_void_p, P(Dense), P(Model), P(Opts), P(TuneEntry)]
    lib.comm_tune_set.argtypes = [ctypes.c_void_p, P(Dense), P(Model), P(Opts), P(TuneEntry), ctypes.c_void_p]
    lib.comm_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.comm_profile_query.argtypes = [ctypes.c_void_p, P(ctypes.c_double), P(ctypes.c_int64), P(ctypes.c_int64)]
    for name in ["comm_create", "comm_destroy", "comm_profile_enable", "comm_profile_query", "comm_cp_update", "comm_tucker_update", "comm_jcomm_outer",
                 "comm_beta_objective", "comm_cp_jcomm_outer_coo", "comm_jcomm_outer_batched",
                 "comm_coo_plan_create", "comm_coo_plan_destroy", "comm_cp_jcomm_outer_coo_plan",
                 "comm_bcomm_sweep_extrap", "comm_jcomm_outer_extrap", "comm_cp_update_coo",
                 "comm_beta_objective_coo", "comm_tucker_update_coo", "comm_tucker_jcomm_outer_coo", "comm_check",
                 "comm_tune_jcomm", "comm_tune_lookup", "comm_tune_set"]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != COMM_OK:
        raise CommError(rc, load_library().comm_last_error().decode())


def _ptr(t, what: str) -> int:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t.data_ptr()


def _f32(t, what: str) -> int:
    import torch
    if t.dtype != torch.float32:
        raise TypeError(f"{what} must be float32")
    return _ptr(t, what)


def _stream(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dense(X) -> Dense:
    if X.dim() > MAX_NDIM:
        raise ValueError(f"tensors of order {X.dim()} exceed the largest supported order {MAX_NDIM}")
    d = Dense()
    d.ndim = X.dim()
    for n in range(X.dim()):
        d.dims[n] = X.shape[n]
    d.X = _f32(X, "X")
    return d


def _model(factors: Sequence, core=None) -> Model:
    m = Model()
    if core is None:
        m.kind = COMM_CP
        m.rank = int(factors[0].shape[1])
    else:
        m.kind = COMM_TUCKER
        m.rank = 0
        for n in range(core.dim()):
            m.core_dims[n] = core.shape[n]
        m.core = _f32(core, "core")
    if len(factors) > MAX_NDIM:
        raise ValueError(f"at most {MAX_NDIM} factors")
    for n, A in enumerate(factors):
        if A.dim() != 2:
            raise ValueError("factors must be matrices")
        m.factors[n] = _f32(A, f"factors[{n}]")
    return m


def _opts(beta: float, eps: float, eps_x: Optional[float], L: int = 1, cache_pq: "bool | str" = False,
          precision: str = "fp32", check_inputs: bool = False) -> Opts:
    o = Opts()
    o.check_inputs = 1 if check_inputs else 0
    o.beta = float(beta)
    o.eps = float(eps)
    o.eps_x = float(eps if eps_x is None else eps_x)
    o.inner_sweeps = int(L)
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
    o.precision = PRECISIONS[precision]
    if isinstance(cache_pq, str):
        if cache_pq != "auto":
            raise ValueError("cache_pq must be True, False or 'auto'")
        o.cache_pq = COMM_CACHE_AUTO
    else:
        o.cache_pq = 1 if cache_pq else 0
    return o


def _coo(idx: Sequence, val, dims: Sequence[int]) -> Coo:
    import torch
    if len(dims) > MAX_NDIM:
        raise ValueError(f"at most {MAX_NDIM} modes")
    c = Coo()
    c.ndim = len(dims)
    for n, dn in enumerate(dims):
        c.dims[n] = int(dn)
    c.nnz = int(val.numel())
    if len(idx) != len(dims):
        raise ValueError("one index tensor per mode")
    for n, ix in enumerate(idx):
        if ix.dtype != torch.int32:
            raise TypeError("idx must be int32")
        if ix.numel() != c.nnz:
            raise ValueError(f"idx[{n}] has {ix.numel()} entries, val {c.nnz}")
        c.idx[n] = _ptr(ix, f"idx[{n}]")
    c.val = _f32(val, "val")
    return c


class CooPlan:
    """Handle of a ``comm_coo_plan`` (device copies owned by the library)."""

    def __init__(self, lib, handle, dims, nnz):
        self._lib = lib
        self.handle = handle
        self.dims = dims
        self.nnz = nnz

    def close(self) -> None:
        if self.handle:
            _check(self._lib.comm_coo_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A problem list for :meth:`Context.jcomm_outer_batched`, marshalled once.

    Each item is a dict with the arguments of :meth:`Context.jcomm_outer`:
    ``X``, ``factors`` and optionally ``core``, ``beta``, ``L``, ``eps``,
    ``eps_x``, ``cache_pq``, ``precision``, ``check_inputs`` and ``obj_out`` (a float64 device view of one
    element).  The structures keep the tensors' device pointers, so the
    tensors must stay alive and in place while the batch is in use."""

    def __init__(self, items: Sequence[dict]):
        import torch
        self.items = list(items)
        n = len(self.items)
        self._dense = [None] * n
        self._model = [None] * n
        self._opts = [None] * n
        self.array = (Problem * max(n, 1))()
        for k, it in enumerate(self.items):
            d = _dense(it["X"])
            m = _model(it["factors"], it.get("core"))
            o = _opts(it.get("beta", 1.0), it.get("eps", 1e-12), it.get("eps_x"), it.get("L", 1),
                      it.get("cache_pq", False), it.get("precision", "fp32"), it.get("check_inputs", False))
            self._dense[k], self._model[k], self._opts[k] = d, m, o
            pr = self.array[k]
            pr.x = ctypes.pointer(d)
            pr.model = ctypes.pointer(m)
            pr.opts = ctypes.pointer(o)
            obj = it.get("obj_out")
            if obj is not None:
                if obj.dtype != torch.float64:
                    raise TypeError("obj_out must be float64")
                pr.obj_ref_dev = _ptr(obj, "obj_out")
            else:
                pr.obj_ref_dev = None

    def __len__(self) -> int:
        return len(self.items)


class Context:
    """A library context on one device; owns the scratch workspace.

    check_inputs=True sets comm_opts.check_inputs on every call: the data and
    parameters are verified on the device first (a synchronising debug mode)."""

    def __init__(self, device: int = 0, workspace_limit: int = 0, check_inputs: bool = False):
        self.check_inputs = bool(check_inputs)
        self._lib = load_library()
        h = ctypes.c_void_p()
        _check(self._lib.comm_create(int(device), int(workspace_limit), ctypes.byref(h)))
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(self._lib.comm_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def check(self) -> None:
        """comm_check: synchronise and raise CommError on an asynchronous device error."""
        _check(self._lib.comm_check(self._h))

    def _o(self, *args, **kw) -> Opts:
        o = _opts(*args, **kw)
        o.check_inputs = 1 if self.check_inputs else 0
        return o

    # ---------------------------------------------------------------- measurement

    def profile_enable(self, on: "bool | int" = True) -> None:
        """Time the fused dense pass launches: True (or 1) every launch, an
        integer k > 1 every k-th launch starting with the first, False (or 0) none."""
        every = int(on) if not isinstance(on, bool) else (1 if on else 0)
        _check(self._lib.comm_profile_enable(self._h, every))

    def profile_query(self):
        """(total kernel milliseconds, timed launches) of the fused dense pass since enable / last query."""
        ms, n, _ = self.profile_query_all()
        return ms, n

    def profile_query_all(self):
        """(total kernel milliseconds, timed launches, all pass launches) since enable / last query."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        seen = ctypes.c_int64()
        _check(self._lib.comm_profile_query(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(seen)))
        return ms.value, n.value, seen.value

    def workspace_bytes(self, dims: Sequence[int], rank: int = 0, core_dims: Optional[Sequence[int]] = None,
                        beta: float = 1.0, L: int = 1, cache_pq: "bool | str" = False, op: int = 1) -> int:
        """Workspace bytes of one call on a tensor of shape `dims` (op 0 update,
        1 jcomm_outer, 2 objective): CP of `rank`, or Tucker with `core_dims`.
        Needs no buffers; 0 if the arguments are invalid."""
        if len(dims) > MAX_NDIM:
            return 0
        d = Dense()
        d.ndim = len(dims)
        for n, v in enumerate(dims):
            d.dims[n] = int(v)
        m = Model()
        if core_dims is None:
            m.kind, m.rank = COMM_CP, int(rank)
        else:
            m.kind = COMM_TUCKER
            for n, v in enumerate(core_dims):
                m.core_dims[n] = int(v)
        o = self._o(beta, 1e-12, None, L, cache_pq)
        return int(self._lib.comm_workspace_bytes(ctypes.byref(d), ctypes.byref(m), ctypes.byref(o), int(op)))

    # ---------------------------------------------------------------- entry points

    def cp_update(self, X, factors, block: int = -1, beta: float = 1.0, eps: float = 1e-12,
                  eps_x: Optional[float] = None, stream=None, precision: str = "fp32") -> None:
        """B-CoMM block update(s) of a CP model in place (block -1: full sweep)."""
        d, m, o = _dense(X), _model(factors), self._o(beta, eps, eps_x, precision=precision)
        _check(self._lib.comm_cp_update(self._h, ctypes.byref(d), ctypes.byref(m), int(block), ctypes.byref(o),
                                        _stream(stream)))

    def tucker_update(self, X, core, factors, block: int = -2, beta: float = 1.0, eps: float = 1e-12,
                      eps_x: Optional[float] = None, stream=None, precision: str = "fp32") -> None:
        """B-CoMM block update(s) of a Tucker model in place (-1 core, n factor, -2 sweep)."""
        d, m, o = _dense(X), _model(factors, core), self._o(beta, eps, eps_x, precision=precision)
        _check(self._lib.comm_tucker_update(self._h, ctypes.byref(d), ctypes.byref(m), int(block),
                                            ctypes.byref(o), _stream(stream)))

    def jcomm_outer(self, X, factors, core=None, beta: float = 1.0, L: int = 1, eps: float = 1e-12,
                    eps_x: Optional[float] = None, cache_pq: "bool | str" = False, obj_out=None, stream=None,
                    precision: str = "fp32") -> None:
        """One J-CoMM outer iteration in place; F(reference) into obj_out[0] (float64) if given."""
        d, m, o = _dense(X), _model(factors, core), self._o(beta, eps, eps_x, L, cache_pq, precision)
        optr = None
        if obj_out is not None:
            import torch
            if obj_out.dtype != torch.float64:
                raise TypeError("obj_out must be float64")
            optr = _ptr(obj_out, "obj_out")
        _check(self._lib.comm_jcomm_outer(self._h, ctypes.byref(d), ctypes.byref(m), ctypes.byref(o), optr,
                                          _stream(stream)))

    def jcomm_outer_noalloc(self, X, factors, core=None, beta: float = 1.0, L: int = 1, eps: float = 1e-12,
                            eps_x: Optional[float] = None, cache_pq: "bool | str" = False, obj_out=None,
                            stream=None, precision: str = "fp32") -> None:
        """jcomm_outer with its workspace in the library's fixed per-GPU array
        (NOALLOC_SCRATCH_BYTES): no device allocation.  Calls that overlap on one
        GPU race; a problem that does not fit raises COMM_ENOMEM."""
        d, m, o = _dense(X), _model(factors, core), self._o(beta, eps, eps_x, L, cache_pq, precision)
        optr = None
        if obj_out is not None:
            import torch
            if obj_out.dtype != torch.float64:
                raise TypeError("obj_out must be float64")
            optr = _ptr(obj_out, "obj_out")
        _check(self._lib.comm_jcomm_outer_noalloc(self._h, ctypes.byref(d), ctypes.byref(m), ctypes.byref(o), optr,
                                                  _stream(stream)))

    def tune_jcomm(self, X, factors, core=None, beta: float = 1.0, L: int = 1, eps: float = 1e-12,
                   eps_x: Optional[float] = None, precision: str = "fp32", reps: int = 3, stream=None) -> dict:
        """Time the equivalent evaluations of a J-CoMM outer iteration (P~/Q~
        cached or recomputed; CP: modes 1 and 2 from one V pass or a pass each;
        Tucker: the mode-3 pair-group cap) on copies of the parameters and
        record the fastest in the context's autotune table.  The entry fixes
        the launch shapes of every J-CoMM call on the same problem, and the
        cache choice of ``cache_pq="auto"`` calls.  Returns ``{"cache_pq",
        "ms_recompute", "ms_cache"}`` (the fastest time of each cache choice,
        NaN when none ran) merged with :meth:`tune_entry`'s fields."""
        d, m, o = _dense(X), _model(factors, core), self._o(beta, eps, eps_x, L, False, precision)
        choice = ctypes.c_int(-1)
        ms = (ctypes.c_double * 2)()
        _check(self._lib.comm_tune_jcomm(self._h, ctypes.byref(d), ctypes.byref(m), ctypes.byref(o), int(reps),
                                         ctypes.byref(choice), ms, _stream(stream)))
        out = self.tune_entry(X, factors, core=core, beta=beta, L=L, eps=eps, eps_x=eps_x, precision=precision)
        out.update({"cache_pq": choice.value, "ms_recompute": ms[0], "ms_cache": ms[1]})
        return out

    def tune_entry(self, X, factors, core=None, beta: float = 1.0, L: int = 1, eps: float = 1e-12,
                   eps_x: Optional[float] = None, precision: str = "fp32") -> dict:
        """The autotune table's entry for a problem (``comm_tune_lookup``):
        ``{"found", "cache_pq", "wshare", "tk_groups", "variants", "ms"}``;
        without an entry, the defaults a call runs with."""
        d, m, o = _dense(X), _model(factors, core), self._o(beta, eps, eps_x, L, False, precision)
        e = TuneEntry()
        _check(self._lib.comm_tune_lookup(self._h, ctypes.byref(d), ctypes.byref(m), ctypes.byref(o),
                                          ctypes.byref(e)))
        return {"found": bool(e.found), "cache_pq": e.cache_pq, "wshare": e.wshare, "tk_groups": e.tk_groups,
                "cp_tile": e.cp_tile, "variants": e.variants, "ms": e.ms}

    def tune_set(self, X, factors, core=None, beta: float = 1.0, L: int = 1, eps: float = 1e-12,
                 eps_x: Optional[float] = None, precision: str = "fp32", cache_pq: int = 0, wshare: int = -1,
                 tk_groups: int = 0, cp_tile: int = 0, stream=None) -> None:
        """Record an autotune table entry directly (``comm_tune_set``)."""
        d, m, o = _dense(X), _model(factors, core), self._o(beta, eps, eps_x, L, False, precision)
        e = TuneEntry()
        e.cache_pq, e.wshare, e.tk_groups, e.cp_tile = int(cache_pq), int(wshare), int(tk_groups), int(cp_tile)
        _check(self._lib.comm_tune_set(self._h, ctypes.byref(d), ctypes.byref(m), ctypes.byref(o), ctypes.byref(e),
                                       _stream(stream)))

    def jcomm_outer_batched(self, batch: "Batch", graph: bool = False, stream=None, grouped: bool = False) -> None:
        """One J-CoMM outer iteration for every problem of `batch`, each with the
        result it would have alone; graph=True captures the batch into a HIP graph
        once and replays it while the same Batch object's problems are passed;
        grouped=True launches each kernel once for all problems that run it at
        the same point (dense order-3 problems)."""
        if not isinstance(batch, Batch):
            batch = Batch(batch)
        flags = (COMM_BATCH_GRAPH if graph else 0) | (COMM_BATCH_GROUPED if grouped else 0)
        _check(self._lib.comm_jcomm_outer_batched(self._h, batch.array, len(batch), flags, _stream(stream)))

    def bcomm_sweep_extrap(self, X, factors, prev, core=None, prev_core=None, beta: float = 1.0,
                           alpha_nes: float = 0.0, c: float = 1.0, delta: float = 1e-12, eps: float = 1e-12,
                           eps_x: Optional[float] = None, alpha_out=None, stream=None, precision: str = "fp32"):
        """Extrapolated B-CoMM sweep in place; ``prev`` (and ``prev_core``) hold the
        previous iterate and receive the one for the next call."""
        d, m, o = _dense(X), _model(factors, core), self._o(beta, eps, eps_x, precision=precision)
        pm = _model(prev, prev_core)
        e = Extrap(float(alpha_nes), float(c), float(delta))
        aptr = _f32(alpha_out, "alpha_out") if alpha_out is not None else None
        _check(self._lib.comm_bcomm_sweep_extrap(self._h, ctypes.byref(d), ctypes.byref(m), ctypes.byref(pm),
                                                 ctypes.byref(o), ctypes.byref(e), aptr, _stream(stream)))

    def jcomm_outer_extrap(self, X, factors, prev, core=None, prev_core=None, beta: float = 1.0, L: int = 1,
                           alpha_nes: float = 0.0, c: float = 1.0, delta: float = 1e-12, eps: float = 1e-12,
                           eps_x: Optional[float] = None, cache_pq: "bool | str" = False, obj_out=None, alpha_out=None,
                           stream=None, precision: str = "fp32"):
        """J-CoMM outer iteration from the extrapolated reference, in place."""
        d, m = _dense(X), _model(factors, core)
        o = self._o(beta, eps, eps_x, L, cache_pq, precision)
        pm = _model(prev, prev_core)
        e = Extrap(float(alpha_nes), float(c), float(delta))
        optr = _ptr(obj_out, "obj_out") if obj_out is not None else None
        aptr = _f32(alpha_out, "alpha_out") if alpha_out is not None else None
        _check(self._lib.comm_jcomm_outer_extrap(self._h, ctypes.byref(d), ctypes.byref(m), ctypes.byref(pm),
                                                 ctypes.byref(o), ctypes.byref(e), optr, aptr, _stream(stream)))

    def beta_objective(self, X, factors, core=None, beta: float = 1.0, eps: float = 1e-12,
                       eps_x: Optional[float] = None, out=None, stream=None, precision: str = "fp32"):
        """D_beta(X, Xhat) in float64, written to out[0] (allocated if None)."""
        import torch
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=X.device)
        d, m, o = _dense(X), _model(factors, core), self._o(beta, eps, eps_x, precision=precision)
        _check(self._lib.comm_beta_objective(self._h, ctypes.byref(d), ctypes.byref(m), ctypes.byref(o),
                                             _ptr(out, "out"), _stream(stream)))
        return out

    def cp_jcomm_outer_coo(self, idx: Sequence, val, dims: Sequence[int], factors, L: int = 1,
                           eps: float = 1e-12, obj_out=None, stream=None, beta: float = 1.0) -> None:
        """One J-CoMM outer iteration on COO data (idx: per-mode int32 tensors);
        beta in (0, 2) (beta = 1: orders 2 to 4, closed-form denominators;
        beta != 1: orders 3 to 5, dense denominators)."""
        c = _coo(idx, val, dims)
        m, o = _model(factors), self._o(beta, eps, None, L)
        optr = _ptr(obj_out, "obj_out") if obj_out is not None else None
        _check(self._lib.comm_cp_jcomm_outer_coo(self._h, ctypes.byref(c), ctypes.byref(m), ctypes.byref(o), optr,
                                                 _stream(stream)))

    def cp_update_coo(self, idx: Sequence, val, dims: Sequence[int], factors, block: int = -1, beta: float = 1.0,
                      eps: float = 1e-12, stream=None) -> None:
        """B-CoMM block update(s) of a CP model on COO data, beta in (0, 2)."""
        c = _coo(idx, val, dims)
        m, o = _model(factors), self._o(beta, eps, None)
        _check(self._lib.comm_cp_update_coo(self._h, ctypes.byref(c), ctypes.byref(m), int(block), ctypes.byref(o),
                                            _stream(stream)))

    def beta_objective_coo(self, idx: Sequence, val, dims: Sequence[int], factors, core=None, beta: float = 1.0,
                           eps: float = 1e-12, out=None, stream=None):
        """D_beta over every cell of COO data (float64 device scalar), beta in (0, 2), CP or Tucker."""
        import torch
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=val.device)
        c = _coo(idx, val, dims)
        m, o = _model(factors, core), self._o(beta, eps, None)
        _check(self._lib.comm_beta_objective_coo(self._h, ctypes.byref(c), ctypes.byref(m), ctypes.byref(o),
                                                 _ptr(out, "out"), _stream(stream)))
        return out

    def tucker_update_coo(self, idx: Sequence, val, dims: Sequence[int], core, factors, block: int = -2,
                          beta: float = 1.0, eps: float = 1e-12, stream=None) -> None:
        """B-CoMM block update(s) of a Tucker model on COO data, beta in (0, 2) (-1 core, n factor, -2 sweep)."""
        c = _coo(idx, val, dims)
        m, o = _model(factors, core), self._o(beta, eps, None)
        _check(self._lib.comm_tucker_update_coo(self._h, ctypes.byref(c), ctypes.byref(m), int(block),
                                                ctypes.byref(o), _stream(stream)))

    def tucker_jcomm_outer_coo(self, idx: Sequence, val, dims: Sequence[int], core, factors, beta: float = 1.0,
                               L: int = 1, eps: float = 1e-12, obj_out=None, stream=None) -> None:
        """One J-CoMM outer iteration of a Tucker model on COO data, beta in (0, 2)."""
        c = _coo(idx, val, dims)
        m, o = _model(factors, core), self._o(beta, eps, None, L)
        optr = _ptr(obj_out, "obj_out") if obj_out is not None else None
        _check(self._lib.comm_tucker_jcomm_outer_coo(self._h, ctypes.byref(c), ctypes.byref(m), ctypes.byref(o),
                                                     optr, _stream(stream)))

    def coo_plan(self, idx: Sequence, val, dims: Sequence[int], stream=None) -> "CooPlan":
        """Sorted device copies of a COO tensor for repeated beta = 1 J-CoMM iterations."""
        c = _coo(idx, val, dims)
        h = ctypes.c_void_p()
        _check(self._lib.comm_coo_plan_create(self._h, ctypes.byref(c), ctypes.byref(h), _stream(stream)))
        return CooPlan(self._lib, h, tuple(int(d) for d in dims), int(val.numel()))

    def cp_jcomm_outer_coo_plan(self, plan: "CooPlan", factors, L: int = 1, eps: float = 1e-12, obj_out=None,
                                stream=None) -> None:
        """cp_jcomm_outer_coo on a planned tensor."""
        m, o = _model(factors), self._o(1.0, eps, None, L)
        optr = _ptr(obj_out, "obj_out") if obj_out is not None else None
        _check(self._lib.comm_cp_jcomm_outer_coo_plan(self._h, plan.handle, ctypes.byref(m), ctypes.byref(o), optr,
                                                      _stream(stream)))


_default_ctx = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


def cp_update(X, factors, block=-1, beta=1.0, eps=1e-12, eps_x=None, stream=None):
    default_context().cp_update(X, factors, block, beta, eps, eps_x, stream)


def tucker_update(X, core, factors, block=-2, beta=1.0, eps=1e-12, eps_x=None, stream=None):
    default_context().tucker_update(X, core, factors, block, beta, eps, eps_x, stream)


def jcomm_outer(X, factors, core=None, beta=1.0, L=1, eps=1e-12, eps_x=None, cache_pq=False, obj_out=None,
                stream=None):
    default_context().jcomm_outer(X, factors, core, beta, L, eps, eps_x, cache_pq, obj_out, stream)


def beta_objective(X, factors, core=None, beta=1.0, eps=1e-12, eps_x=None, out=None, stream=None):
    return default_context().beta_objective(X, factors, core, beta, eps, eps_x, out, stream)


def cp_jcomm_outer_coo(idx, val, dims, factors, L=1, eps=1e-12, obj_out=None, stream=None):
    default_context().cp_jcomm_outer_coo(idx, val, dims, factors, L, eps, obj_out, stream)


def jcomm_outer_batched(batch, graph=False, stream=None, grouped=False):
    default_context().jcomm_outer_batched(batch, graph, stream, grouped)
