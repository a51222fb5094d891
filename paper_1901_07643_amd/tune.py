"""Autotuning of the segment size k by measurement on the device.

The walk of m variables is split into 2^(m-k) segments of 2^k - k - 1 Givens
steps each (Sec. 6).  Small k means many segments, each with its own O(m^3)
anchor QR; large k means fewer, longer walks (fewer waves to balance, and more
FP32 rounding from the FP64 start).  The best k depends on m, on n only through
the R0 QR, and for a batch on the mix of sizes, so it is chosen by timing the
real calls on synthetic data of the requested shapes.

    k = tune_plan(26, 5000)                 # best k for one dataset shape
    caps = tune_batch([(m0, n0), ...])      # best common cap on k for a batch

Results are kept in a per-process cache keyed by shape and, when GS_TUNE_CACHE names a
file (or the default ~/.cache/givscore/tune.json is writable), in a JSON file keyed by
the GPU architecture, the library build and the shapes, so that later processes on the
same kind of device skip the timing.  GS_TUNE_CACHE=off disables the file.
"""
from __future__ import annotations

import hashlib
import json
import os

_CACHE: dict = {}


def _cache_path():
    p = os.environ.get("GS_TUNE_CACHE")
    if p == "off":
        return None
    return p or os.path.join(os.path.expanduser("~"), ".cache", "givscore", "tune.json")


def _file_key(key, device) -> str:
    """Stable text key: architecture, library build, and the in-process key."""
    import torch

    from ._abi import LIB_PATH
    props = torch.cuda.get_device_properties(device or "cuda")
    arch = getattr(props, "gcnArchName", props.name)
    try:
        st = os.stat(LIB_PATH)
        build = f"{st.st_size}:{int(st.st_mtime)}"
    except OSError:
        build = "?"
    return hashlib.sha256(repr((arch, build, key)).encode()).hexdigest()[:32]


def _file_get(key, device):
    path = _cache_path()
    if not path:
        return None
    try:
        with open(path) as f:
            val = json.load(f).get(_file_key(key, device))
    except (OSError, ValueError):
        return None
    return val


def _file_put(key, device, value) -> None:
    path = _cache_path()
    if not path:
        return
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        try:
            with open(path) as f:
                data = json.load(f)
        except (OSError, ValueError):
            data = {}
        data[_file_key(key, device)] = value
        tmp = f"{path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(data, f)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home: the in-process cache still holds the result

# FP32 accuracy limit on the walk length from its FP64 start (see the plan defaults)
K_MAX_FP32 = 13


def _timed(fn, reps: int, warmup: int = 1) -> float:
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def k_candidates(m: int, ks: int = 5, kmax: int = K_MAX_FP32) -> list[int]:
    """Segment sizes worth trying for m variables: ks .. min(m, kmax), at most 16
    middle variables."""
    ks = min(ks, m)
    return [k for k in range(ks, min(m, kmax) + 1) if k - ks <= 16]


def tune_plan(m: int, n: int, candidates=None, reps: int = 5, device=None, seed: int = 0,
              what: str = "bic") -> int:
    """The k (inner block 5) with the shortest gs_score_all call for an (n, m)
    dataset, timed on seeded Gaussian data on the device."""
    import torch

    from . import Plan, score_all
    key = ("plan", m, n, what, tuple(candidates) if candidates else None)
    if key in _CACHE:
        return _CACHE[key]
    hit = _file_get(key, device)
    if isinstance(hit, int):
        _CACHE[key] = hit
        return hit
    dev = torch.device(device or "cuda")
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.randn((n, m), generator=g, dtype=torch.float64).to(dev)
    best, best_ms = None, float("inf")
    out = None
    for k in candidates or k_candidates(m):
        plan = Plan(m, k, 5 if m >= 5 else 0)
        out = score_all(X, plan=plan, what=what, out=out)
        ms = _timed(lambda: score_all(X, plan=plan, what=what, out=out, check_status=False), reps)
        if ms < best_ms:
            best, best_ms = k, ms
        plan.close()
    _CACHE[key] = best
    _file_put(key, device, best)
    return best


def batch_k(shapes, cap: int) -> list[int]:
    """Per-dataset k for a common cap: k = min(m, cap), at least the inner block."""
    return [max(5, min(m, cap)) for m, _ in shapes]


def tune_batch(shapes, caps=None, reps: int = 5, device=None, seed: int = 0,
               what: str = "bic", use_graph: bool = True):
    """Best common cap on k for a batch of (m, n) shapes, timed as graph replays of
    gs_score_batched on seeded Gaussian data.  Returns (cap, {cap: ms})."""
    import torch

    from . import Batch, num_families
    shapes = [(int(m), int(n)) for m, n in shapes]
    key = ("batch", tuple(shapes), what, tuple(caps) if caps else None)
    if key in _CACHE:
        return _CACHE[key]
    hit = _file_get(key, device)
    if isinstance(hit, list) and len(hit) == 2 and isinstance(hit[1], dict):
        val = (int(hit[0]), {int(c): float(t) for c, t in hit[1].items()})
        _CACHE[key] = val
        return val
    dev = torch.device(device or "cuda")
    g = torch.Generator(device="cpu").manual_seed(seed)
    Xs = [torch.randn((n, m), generator=g, dtype=torch.float64).to(dev) for m, n in shapes]
    outs = [torch.empty(num_families(m), dtype=torch.float32, device=dev) for m, _ in shapes]
    mmax = max(m for m, _ in shapes)
    times = {}
    for cap in caps or range(5, min(mmax, K_MAX_FP32) + 1):
        b = Batch(shapes, k=batch_k(shapes, cap))
        b.score(Xs, what=what, outs=outs, use_graph=use_graph)
        times[cap] = _timed(lambda: b.score(Xs, what=what, outs=outs, use_graph=use_graph,
                                            check_status=False), reps)
        b.close()
    best = min(times, key=times.get)
    _CACHE[key] = (best, times)
    _file_put(key, device, [best, {str(c): t for c, t in times.items()}])
    return best, times


def clear_cache():
    _CACHE.clear()


__all__ = ["tune_plan", "tune_batch", "batch_k", "k_candidates", "clear_cache"]
