"""givscore: scores of every (child, parent set) family of m variables by the
Givens-rotation walk over QR decompositions, as hand-written HIP kernels for
MI355X (gfx950).

This module is a thin binding over the C ABI in include/givscore.h: it marshals
torch device tensors into pointers and the current HIP stream; every step of the
computation runs in libgivscore.so.  PyTorch only provides device memory and
streams.

    X = torch.as_tensor(data, dtype=torch.float64, device="cuda")   # (n, m)
    table = score_all(X)               # (m * 2^(m-1),) float32 BIC, FP32 walk
    rss = score_all(X, what="rss", precision="fp64")

Table order: index(c, S) = c * 2^(m-1) + compress(S, c), see family_index().
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._abi import (BatchData, ReduceOut, GS_EINVAL, GS_ENOTFINITE, GS_ERANGE, GS_ERANK, GS_MAX_M, GS_OK,
                   GS_OUT_BIC, GS_OUT_RSS, GivScoreError, PlanInfo, check, last_error, lib)

__all__ = [
    "Plan", "Batch", "score_all", "score_all_many", "score_reduce", "score_beta", "count_writes", "score_backward", "givscore", "GivScore", "qr_r0", "num_families", "family_index", "upsilon", "GivScoreError",
    "GS_OK", "GS_EINVAL", "GS_ERANK", "GS_ENOTFINITE", "GS_ERANGE", "GS_MAX_M", "lib", "last_error",
]


def num_families(m: int) -> int:
    r = lib().gs_num_families(m)
    if r < 0:
        raise GivScoreError(GS_EINVAL, f"m={m} out of range")
    return int(r)


def family_index(m: int, child: int, parent_mask: int) -> int:
    r = lib().gs_family_index(m, child, parent_mask)
    if r < 0:
        raise GivScoreError(GS_EINVAL, "bad family")
    return int(r)


def upsilon(m: int) -> list[int]:
    """The paper's swap sequence (1-based), from the library's planner."""
    n = check(lib().gs_upsilon(m, None, 0))
    buf = (ctypes.c_int32 * max(1, n))()
    check(lib().gs_upsilon(m, buf, n))
    return list(buf[:n])


class Plan:
    """Library-owned plan for m variables (segment split and walk program)."""

    def __init__(self, m: int, k: int = 0, ks: int = 0):
        h = ctypes.c_void_p()
        check(lib().gs_plan_tuned(m, k, ks, ctypes.byref(h)))
        self._h = h
        self.m = m
        self._many_count = 0
        self._reuse = False

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan destroyed")
        return self._h

    @property
    def info(self) -> dict:
        inf = PlanInfo()
        check(lib().gs_plan_get_info(self.handle, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in PlanInfo._fields_}

    def workspace_bytes(self, n: int, backward: bool = False) -> int:
        """Device bytes the plan holds after a call with n rows."""
        b = ctypes.c_int64()
        check(lib().gs_plan_workspace_bytes(self.handle, n, 1 if backward else 0, ctypes.byref(b)))
        return int(b.value)

    def count_emissions(self) -> np.ndarray:
        """Host simulation of the walk: how often each table entry would be written."""
        counts = np.zeros(num_families(self.m), dtype=np.int32)
        check(lib().gs_plan_count_emissions(
            self.handle, counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), counts.size))
        return counts

    def status(self) -> int:
        """Wait for the last call and return its device status code (0, GS_ERANK,
        GS_ENOTFINITE, GS_ERANGE)."""
        return int(lib().gs_sync_status(self.handle))

    def many_status(self) -> list[int]:
        """Per-dataset status codes of the plan's last score_all_many call (waits)."""
        cnt = self._many_count
        st = (ctypes.c_int * max(cnt, 1))()
        lib().gs_many_status(self.handle, st)
        return [int(st[i]) for i in range(cnt)]

    def vif(self) -> np.ndarray:
        """Variance inflation factors of the columns of the last call's data."""
        out = np.zeros(self.m, dtype=np.float64)
        check(lib().gs_column_vif(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set_reuse(self, enable: bool = True):
        """Let backward calls take R0 and the segment anchors from the plan's last call on
        the same X (same pointer, n, row stride and walk precision; gs_plan_set_reuse)
        instead of forming them again.  X must still hold the same values."""
        check(lib().gs_plan_set_reuse(self.handle, 1 if enable else 0))
        self._reuse = bool(enable)

    def set_timing(self, enable: bool = True):
        check(lib().gs_set_timing(self.handle, 1 if enable else 0))

    def timing(self):
        """Mean ms of (R0 QR, anchors, walk, whole call) over the recorded calls."""
        ms = (ctypes.c_double * 4)()
        cnt = ctypes.c_int64()
        check(lib().gs_get_timing(self.handle, ms, ctypes.byref(cnt)))
        return list(ms), int(cnt.value)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().gs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_X(X, m_expected=None):
    import torch
    if not isinstance(X, torch.Tensor) or X.device.type != "cuda":
        raise TypeError("X must be a torch tensor on a HIP device")
    if X.dtype != torch.float64 or X.dim() != 2:
        raise TypeError("X must be a 2-D float64 tensor (n, m)")
    if X.stride(1) != 1:
        raise ValueError("X must have unit column stride (row-major)")
    n, m = X.shape
    if m_expected is not None and m != m_expected:
        raise ValueError("X has a different m than the plan")
    return n, m, X.stride(0)


def _stream(dev):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def qr_r0(X, plan: Plan | None = None):
    """R factor (m x m, FP64, non-negative diagonal) of the QR decomposition of X."""
    import torch
    n, m, ldx = _check_X(X, plan.m if plan else None)
    plan = plan or Plan(m)
    R = torch.empty((m, m), dtype=torch.float64, device=X.device)
    with torch.cuda.device(X.device):
        check(lib().gs_qr_r0(plan.handle, ctypes.c_void_p(X.data_ptr()), n, m, ldx,
                             ctypes.c_void_p(R.data_ptr()), _stream(X.device)))
    return R


def score_all(X, plan: Plan | None = None, what: str = "bic", precision: str = "fp32", out=None,
              check_status: bool = True):
    """All m * 2^(m-1) family scores of X (device tensor (n, m) float64).

    what: "bic" or "rss".  precision: "fp32" (FP32 walk, FP32 table) or "fp64"
    (FP64 walk, FP64 table).  With check_status the call waits for the device and
    raises GivScoreError on rank-deficient or non-finite X."""
    import torch
    n, m, ldx = _check_X(X, plan.m if plan else None)
    plan = plan or Plan(m)
    w = {"bic": GS_OUT_BIC, "rss": GS_OUT_RSS}[what]
    dtype = {"fp32": torch.float32, "fp64": torch.float64}[precision]
    N = num_families(m)
    if out is None:
        out = torch.empty(N, dtype=dtype, device=X.device)
    elif out.dtype != dtype or out.numel() != N or not out.is_contiguous() or out.device != X.device:
        raise ValueError("out must be a contiguous tensor of m*2^(m-1) elements of the right dtype")
    fn = lib().gs_score_all if precision == "fp32" else lib().gs_score_all_f64
    with torch.cuda.device(X.device):
        check(fn(plan.handle, ctypes.c_void_p(X.data_ptr()), n, m, ldx,
                 ctypes.c_void_p(out.data_ptr()), w, _stream(X.device)))
        if check_status:
            check(plan.status())
    return out


def score_all_many(Xs, plan: Plan | None = None, what: str = "bic", outs=None,
                   in_flight: int = 3, check_status: bool = True):
    """FP32 score tables of many datasets of one shape (gs_score_all_many): up to
    in_flight of them in progress at once on the plan's internal streams, forked from
    and joined to the current stream.  Xs: list of (n, m) float64 device tensors with
    the same n, m and row stride.  Returns the list of tables (float32, m * 2^(m-1)),
    each bit-identical to score_all on its dataset.  With check_status the call waits
    and raises GivScoreError naming the first dataset whose status is not GS_OK."""
    import torch
    if not Xs:
        raise ValueError("Xs is empty")
    n, m, ldx = _check_X(Xs[0], plan.m if plan else None)
    for X in Xs:
        if _check_X(X, m) != (n, m, ldx) or X.device != Xs[0].device:
            raise ValueError("every dataset needs the same shape, row stride and device")
    plan = plan or Plan(m)
    w = {"bic": GS_OUT_BIC, "rss": GS_OUT_RSS}[what]
    N = num_families(m)
    if outs is None:
        outs = [torch.empty(N, dtype=torch.float32, device=Xs[0].device) for _ in Xs]
    elif len(outs) != len(Xs) or any(o.dtype != torch.float32 or o.numel() != N or
                                     not o.is_contiguous() or o.device != Xs[0].device
                                     for o in outs):
        raise ValueError("outs must hold one contiguous float32 tensor of m*2^(m-1) "
                         "elements per dataset")
    cnt = len(Xs)
    xp = (ctypes.c_void_p * cnt)(*[X.data_ptr() for X in Xs])
    op = (ctypes.c_void_p * cnt)(*[o.data_ptr() for o in outs])
    with torch.cuda.device(Xs[0].device):
        check(lib().gs_score_all_many(plan.handle, cnt, xp, n, ldx, op, w, in_flight,
                                      _stream(Xs[0].device)))
        plan._many_count = cnt
        if check_status:
            st = (ctypes.c_int * cnt)()
            check(lib().gs_many_status(plan.handle, st))
    return outs


def score_reduce(X, plan: Plan | None = None, top_k: int = 0, check_status: bool = True):
    """Per-child results of the FP32 BIC walk without the score table (gs_score_reduce):
    dict of device tensors best_score (m,) float32, best_parents (m,) int32 parent masks,
    logsumexp (m,) float64 = ln sum_S exp(-BIC(c, S)), and with top_k > 0 top_score
    (m, top_k) float32 ascending and top_parents (m, top_k) int32."""
    import torch
    n, m, ldx = _check_X(X, plan.m if plan else None)
    plan = plan or Plan(m)
    dev = X.device
    res = {"best_score": torch.empty(m, dtype=torch.float32, device=dev),
           "best_parents": torch.empty(m, dtype=torch.int32, device=dev),
           "logsumexp": torch.empty(m, dtype=torch.float64, device=dev)}
    o = ReduceOut()
    o.best_score = res["best_score"].data_ptr()
    o.best_parents = res["best_parents"].data_ptr()
    o.logsumexp = res["logsumexp"].data_ptr()
    o.top_k = int(top_k)
    if top_k > 0:
        res["top_score"] = torch.empty((m, top_k), dtype=torch.float32, device=dev)
        res["top_parents"] = torch.empty((m, top_k), dtype=torch.int32, device=dev)
        o.top_score = res["top_score"].data_ptr()
        o.top_parents = res["top_parents"].data_ptr()
    with torch.cuda.device(dev):
        check(lib().gs_score_reduce(plan.handle, ctypes.c_void_p(X.data_ptr()), n, m, ldx,
                                    ctypes.byref(o), _stream(dev)))
        if check_status:
            check(plan.status())
    return res


def score_beta(X, plan: Plan | None = None, out=None, check_status: bool = True):
    """Regression coefficients of every family (gs_score_beta): a (m * 2^(m-1), m) float64
    device tensor in table order, row index(c, S) holding beta_v for v in S and zeros
    elsewhere.  m <= 22."""
    import torch
    n, m, ldx = _check_X(X, plan.m if plan else None)
    plan = plan or Plan(m)
    N = num_families(m)
    if out is None:
        out = torch.empty((N, m), dtype=torch.float64, device=X.device)
    elif out.shape != (N, m) or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous (m*2^(m-1), m) float64 tensor")
    with torch.cuda.device(X.device):
        check(lib().gs_score_beta(plan.handle, ctypes.c_void_p(X.data_ptr()), n, m, ldx,
                                  ctypes.c_void_p(out.data_ptr()), _stream(X.device)))
        if check_status:
            check(plan.status())
    return out


def count_writes(X, plan: Plan | None = None, out=None):
    """Testing: how often the FP32 walk writes each table entry (int32 device tensor;
    a correct plan gives all ones).  Same kernels and store path as score_all."""
    import torch
    n, m, ldx = _check_X(X, plan.m if plan else None)
    plan = plan or Plan(m)
    N = num_families(m)
    if out is None:
        out = torch.zeros(N, dtype=torch.int32, device=X.device)
    elif out.dtype != torch.int32 or out.numel() != N or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor of m*2^(m-1) elements")
    else:
        out.zero_()
    with torch.cuda.device(X.device):
        check(lib().gs_count_writes(plan.handle, ctypes.c_void_p(X.data_ptr()), n, m, ldx,
                                    ctypes.c_void_p(out.data_ptr()), _stream(X.device)))
        check(plan.status())
    return out


def score_backward(X, dscores, plan: Plan | None = None, what: str = "bic",
                   precision: str = "fp32", out=None, check_status: bool = True,
                   reuse_front: bool | None = None):
    """d(loss)/dX (n, m) float64 from dscores = d(loss)/d(score) for every family.

    precision "fp32" replays and undoes the FP32 walk (dscores float32); "fp64" the FP64
    walk (dscores float64).  The anchor and R0 QR adjoints run in FP64.  reuse_front
    (None: the plan's setting, see Plan.set_reuse) takes R0 and the anchors from the
    plan's last call on the same X, which must still hold the same values."""
    import torch
    n, m, ldx = _check_X(X, plan.m if plan else None)
    plan = plan or Plan(m)
    w = {"bic": GS_OUT_BIC, "rss": GS_OUT_RSS}[what]
    dtype = {"fp32": torch.float32, "fp64": torch.float64}[precision]
    N = num_families(m)
    if (not isinstance(dscores, torch.Tensor) or dscores.dtype != dtype
            or dscores.numel() != N or dscores.device != X.device):
        raise ValueError(f"dscores must be a {dtype} device tensor of m*2^(m-1) elements")
    dscores = dscores.contiguous()
    if out is None:
        out = torch.empty((n, m), dtype=torch.float64, device=X.device)
    elif out.shape != (n, m) or out.dtype != torch.float64 or out.stride(1) != 1:
        raise ValueError("out must be an (n, m) float64 tensor with unit column stride")
    fn = lib().gs_score_backward if precision == "fp32" else lib().gs_score_backward_f64
    override = reuse_front is not None and bool(reuse_front) != plan._reuse
    with torch.cuda.device(X.device):
        if override:
            check(lib().gs_plan_set_reuse(plan.handle, 1 if reuse_front else 0))
        try:
            check(fn(plan.handle, ctypes.c_void_p(X.data_ptr()), n, m, ldx,
                     ctypes.c_void_p(dscores.data_ptr()), w, ctypes.c_void_p(out.data_ptr()),
                     out.stride(0), _stream(X.device)))
        finally:
            if override:
                lib().gs_plan_set_reuse(plan.handle, 1 if plan._reuse else 0)
        if check_status:
            check(plan.status())
    return out


class Batch:
    """Many datasets scored together: one launch per stage for the whole batch
    (gs_score_batched), optionally replayed from a captured hipGraph.

        b = Batch([(m0, n0), (m1, n1), ...])
        tables = b.score([X0, X1, ...])          # list of float32 device tensors
    """

    def __init__(self, shapes, k=None):
        shapes = [(int(m), int(n)) for m, n in shapes]
        cnt = len(shapes)
        ms = (ctypes.c_int * cnt)(*[m for m, _ in shapes])
        ns = (ctypes.c_int64 * cnt)(*[n for _, n in shapes])
        ks = None if k is None else (ctypes.c_int * cnt)(*(k if hasattr(k, "__len__") else [k] * cnt))
        h = ctypes.c_void_p()
        check(lib().gs_batch_create(cnt, ms, ns, ks, ctypes.byref(h)))
        self._h = h
        self.shapes = shapes
        self._keep = None

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch destroyed")
        return self._h

    @property
    def info(self) -> dict:
        w, s, f = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(lib().gs_batch_info(self.handle, ctypes.byref(w), ctypes.byref(s), ctypes.byref(f)))
        return {"total_waves": w.value, "total_segments": s.value, "total_families": f.value}

    def score(self, Xs, what: str = "bic", outs=None, use_graph: bool = True,
              check_status: bool = True):
        """Score tables (float32, FP32 walk) of every dataset in Xs (device float64
        tensors of the shapes given at creation)."""
        import torch
        if len(Xs) != len(self.shapes):
            raise ValueError("one tensor per dataset")
        w = {"bic": GS_OUT_BIC, "rss": GS_OUT_RSS}[what]
        dev = Xs[0].device
        if outs is None:
            outs = [torch.empty(num_families(m), dtype=torch.float32, device=dev)
                    for m, _ in self.shapes]
        data = (BatchData * len(Xs))()
        for i, (X, (m, n)) in enumerate(zip(Xs, self.shapes)):
            nn, mm, ldx = _check_X(X, m)
            if nn != n or X.device != dev:
                raise ValueError(f"dataset {i}: expected ({n}, {m}) on {dev}")
            o = outs[i]
            if o.dtype != torch.float32 or o.numel() != num_families(m) or not o.is_contiguous():
                raise ValueError(f"dataset {i}: bad output tensor")
            data[i].X, data[i].ldx, data[i].scores = X.data_ptr(), ldx, o.data_ptr()
        with torch.cuda.device(dev):
            check(lib().gs_score_batched(self.handle, data, w, 1 if use_graph else 0, _stream(dev)))
            self._keep = (list(Xs), outs)  # the tables hold these pointers
            if check_status:
                bad = [(i, c) for i, c in enumerate(self.status()) if c != GS_OK]
                if bad:
                    raise GivScoreError(bad[0][1], f"dataset {bad[0][0]} (of {len(bad)} failed)")
        return outs

    def status(self) -> list[int]:
        """Wait for the last call; per-dataset GS_OK, GS_ERANK, GS_ENOTFINITE or
        GS_ERANGE."""
        st = (ctypes.c_int * len(self.shapes))()
        r = lib().gs_batch_status(self.handle, st)
        if r not in (GS_OK, GS_ERANK, GS_ENOTFINITE, GS_ERANGE):
            check(r)
        return list(st)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().gs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_function():
    import torch

    class GivScore(torch.autograd.Function):
        """scores = score_all(X) with a hand-written backward (gs_score_backward)."""

        @staticmethod
        def forward(ctx, X, plan, what, precision):
            scores = score_all(X, plan=plan, what=what, precision=precision)
            ctx.save_for_backward(X)
            ctx.plan, ctx.what, ctx.precision = plan, what, precision
            return scores

        @staticmethod
        def backward(ctx, dscores):
            (X,) = ctx.saved_tensors
            dtype = torch.float32 if ctx.precision == "fp32" else torch.float64
            # autograd has checked that X was not modified since the forward, so R0 and
            # the anchors that the forward left in the plan can be reused when nothing
            # else has run on the plan since
            dX = score_backward(X, dscores.to(dtype).contiguous(), plan=ctx.plan, what=ctx.what,
                                precision=ctx.precision, reuse_front=True)
            return dX, None, None, None

    return GivScore


_GIVSCORE_FN = None


def __getattr__(name):
    global _GIVSCORE_FN
    if name == "GivScore":
        if _GIVSCORE_FN is None:
            _GIVSCORE_FN = _make_function()
        return _GIVSCORE_FN
    raise AttributeError(name)


def givscore(X, plan: Plan | None = None, what: str = "bic", precision: str = "fp32"):
    """Differentiable scores of every family of X (torch.autograd)."""
    n, m, _ = _check_X(X, plan.m if plan else None)
    plan = plan or Plan(m)
    return __getattr__("GivScore").apply(X, plan, what, precision)
