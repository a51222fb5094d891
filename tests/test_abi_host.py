"""Host-side checks of libgivscore (no GPU needed): the library loads, exports every
symbol its header declares, validates arguments before touching the device, and its
integer planner covers every family exactly once."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle import walk as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gs():
    import paper_1901_07643_amd as g
    g.lib()
    return g


def test_header_symbols_exported(gs):
    hdr = open(os.path.join(ROOT, "include", "givscore.h")).read()
    names = set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(gs_\w+)\s*\(", hdr, re.M))
    assert {"gs_plan", "gs_score_all", "gs_score_all_f64", "gs_qr_r0"} <= names
    L = ctypes.CDLL(gs._abi.LIB_PATH)
    for n in sorted(names):
        assert hasattr(L, n), f"{n} declared in the header but not exported"


def test_family_index_matches_oracle(gs):
    rng = np.random.default_rng(0)
    for m in [1, 2, 5, 13, 26, 30]:
        for _ in range(200):
            c = int(rng.integers(0, m))
            mask = int(rng.integers(0, 1 << m)) & ~(1 << c)
            assert gs.family_index(m, c, mask) == oracle.family_index(m, c, mask)
        assert gs.num_families(m) == m * 2 ** (m - 1)
    with pytest.raises(gs.GivScoreError):
        gs.family_index(5, 2, 0b100)
    with pytest.raises(gs.GivScoreError):
        gs.num_families(31)


@pytest.mark.parametrize("m", range(1, 15))
def test_upsilon_matches_reference(gs, m):
    assert gs.upsilon(m) == W.greedy_swaps(m)


def test_plan_argument_errors(gs):
    with pytest.raises(gs.GivScoreError) as e:
        gs.Plan(0)
    assert e.value.code == gs.GS_EINVAL
    for m, k, ks in [(31, 0, 0), (10, 3, 5), (10, 11, 5), (30, 30, 5), (8, 8, 7)]:
        with pytest.raises(gs.GivScoreError):
            gs.Plan(m, k, ks)


def test_score_argument_errors_before_device_work(gs):
    L = gs.lib()
    p = gs.Plan(6)
    fake = ctypes.c_void_p(4096)
    # n <= m, ldx < m, m mismatch, bad output selector, misaligned output, NULL data
    assert L.gs_score_all(p.handle, fake, 6, 6, 6, fake, 0, None) == gs.GS_EINVAL
    assert L.gs_score_all(p.handle, fake, 50, 6, 5, fake, 0, None) == gs.GS_EINVAL
    assert L.gs_score_all(p.handle, fake, 50, 7, 7, fake, 0, None) == gs.GS_EINVAL
    assert L.gs_score_all(p.handle, fake, 50, 6, 6, fake, 7, None) == gs.GS_EINVAL
    assert L.gs_score_all(p.handle, fake, 50, 6, 6, ctypes.c_void_p(4100), 0, None) == gs.GS_EINVAL
    assert L.gs_score_all_f64(p.handle, None, 50, 6, 6, fake, 0, None) == gs.GS_EINVAL
    assert L.gs_qr_r0(None, fake, 50, 6, 6, fake, None) == gs.GS_EINVAL
    assert "plan" in gs.last_error()


def _plans():
    out = []
    for m in range(1, 15):
        for ks in range(1, min(6, m) + 1):
            for k in sorted({ks, min(m, ks + 1), min(m, ks + 3), m}):
                if k - ks <= 16:
                    out.append((m, k, ks))
    return out


def test_many_argument_errors_before_device_work(gs):
    """gs_score_all_many rejects bad arguments before it touches the device (the
    pointers here are never dereferenced)."""
    L = gs.lib()
    p = gs.Plan(6)
    vp = ctypes.c_void_p
    xs = (vp * 2)(4096, 8192)
    outs = (vp * 2)(4096, 8192)
    bad = (vp * 2)(4096, 4100)  # second table not 16-byte aligned
    assert L.gs_score_all_many(p.handle, 0, xs, 50, 6, outs, 0, 2, None) == gs.GS_EINVAL
    assert L.gs_score_all_many(p.handle, 2, xs, 50, 6, outs, 0, 0, None) == gs.GS_EINVAL
    assert L.gs_score_all_many(p.handle, 2, xs, 50, 6, outs, 0, 9, None) == gs.GS_EINVAL
    assert L.gs_score_all_many(p.handle, 2, None, 50, 6, outs, 0, 2, None) == gs.GS_EINVAL
    assert L.gs_score_all_many(p.handle, 2, xs, 50, 6, None, 0, 2, None) == gs.GS_EINVAL
    assert L.gs_score_all_many(p.handle, 2, xs, 50, 6, bad, 0, 2, None) == gs.GS_EINVAL
    assert L.gs_score_all_many(p.handle, 2, xs, 6, 6, outs, 0, 2, None) == gs.GS_EINVAL
    assert L.gs_score_all_many(p.handle, 2, xs, 50, 6, outs, 7, 2, None) == gs.GS_EINVAL
    assert L.gs_score_all_many(None, 2, xs, 50, 6, outs, 0, 2, None) == gs.GS_EINVAL
    st = (ctypes.c_int * 2)()
    assert L.gs_many_status(p.handle, st) == gs.GS_EINVAL  # no call has run
    assert L.gs_many_status(None, st) == gs.GS_EINVAL


def test_backward_argument_errors_before_device_work(gs):
    """gs_score_backward rejects a NULL or misaligned dscores (the line loads of the
    walk adjoint are 16 bytes wide) before it touches the device."""
    L = gs.lib()
    p = gs.Plan(6)
    vp = ctypes.c_void_p
    for fn in (L.gs_score_backward, L.gs_score_backward_f64):
        assert fn(p.handle, vp(4096), 50, 6, 6, None, 0, vp(8192), 6, None) == gs.GS_EINVAL
        assert fn(p.handle, vp(4096), 50, 6, 6, vp(4100), 0, vp(8192), 6, None) == gs.GS_EINVAL
        assert "16-byte aligned" in gs.last_error()
        assert fn(p.handle, vp(4096), 50, 6, 6, vp(4096), 0, vp(8200), 6, None) == gs.GS_EINVAL


def test_reuse_switch(gs):
    """gs_plan_set_reuse only sets a flag of the plan (no device work)."""
    L = gs.lib()
    assert L.gs_plan_set_reuse(None, 1) == gs.GS_EINVAL
    p = gs.Plan(6)
    assert L.gs_plan_set_reuse(p.handle, 1) == gs.GS_OK
    p.set_reuse(False)
    assert p._reuse is False


@pytest.mark.parametrize("m,k,ks", _plans())
def test_plan_covers_every_family_once(gs, m, k, ks):
    p = gs.Plan(m, k, ks)
    info = p.info
    q = k - ks
    assert info["num_segments"] == 2 ** (m - k) and info["sub_per_segment"] == 2 ** q
    # Givens steps of the two-level walk = the optimum 2^k - k - 1 of one segment
    steps = (2 ** q - 1) * ks + (2 ** q - q - 1) + 2 ** q * W.swap_count(ks)
    assert steps == info["swaps_per_segment"] == W.swap_count(k)
    c = p.count_emissions()
    assert c.size == m * 2 ** (m - 1) and (c == 1).all()


@pytest.mark.slow
@pytest.mark.parametrize("m,k,ks", [(18, 13, 5), (20, 7, 5), (16, 16, 6), (22, 9, 5)])
def test_plan_covers_every_family_once_large(gs, m, k, ks):
    c = gs.Plan(m, k, ks).count_emissions()
    assert (c == 1).all()


def test_default_plans(gs):
    for m, k, ks in [(8, 5, 5), (14, 5, 5), (20, 7, 5), (26, 13, 5), (30, 13, 5), (3, 3, 3)]:
        inf = gs.Plan(m).info
        assert (inf["k"], inf["ks"]) == (k, ks)


def test_batch_planning_host(gs):
    """Batch creation is host-only: sizes add up over the per-dataset plans."""
    from datagen import bootstrap_batch
    shapes = [(X.shape[1], X.shape[0]) for X in bootstrap_batch(count=32)]
    b = gs.Batch(shapes)
    inf = b.info
    waves = segs = 0
    for m, _ in shapes:
        pi = gs.Plan(m, 0, 5).info
        waves += pi["num_waves"]
        segs += pi["num_segments"]
    assert inf == {"total_waves": waves, "total_segments": segs,
                   "total_families": sum(m * 2 ** (m - 1) for m, _ in shapes)}
    assert b.status() == [gs.GS_OK] * len(shapes)  # nothing enqueued yet
    b.close()


def test_batch_argument_errors(gs):
    L = gs.lib()
    h = ctypes.c_void_p()
    i32, i64 = ctypes.c_int, ctypes.c_int64
    for ms, ns in [([4], [100]), ([31], [100]), ([8], [8]), ([8, 9], [100, 5])]:
        cnt = len(ms)
        r = L.gs_batch_create(cnt, (i32 * cnt)(*ms), (i64 * cnt)(*ns), None, ctypes.byref(h))
        assert r == gs.GS_EINVAL, (ms, ns)
    assert L.gs_batch_create(0, (i32 * 1)(8), (i64 * 1)(100), None, ctypes.byref(h)) == gs.GS_EINVAL
    # bad k for one dataset
    assert L.gs_batch_create(1, (i32 * 1)(8), (i64 * 1)(100), (i32 * 1)(3),
                             ctypes.byref(h)) == gs.GS_EINVAL
    b = gs.Batch([(8, 100)])
    fake = ctypes.c_void_p(4096)
    d = (gs._abi.BatchData * 1)()
    d[0].X, d[0].ldx, d[0].scores = 4096, 7, 4096  # ldx < m
    assert L.gs_score_batched(b.handle, d, 0, 0, None) == gs.GS_EINVAL
    d[0].ldx, d[0].scores = 8, 4100  # misaligned table
    assert L.gs_score_batched(b.handle, d, 0, 0, None) == gs.GS_EINVAL
    d[0].scores = 4096
    assert L.gs_score_batched(b.handle, d, 5, 0, None) == gs.GS_EINVAL  # bad what
    assert L.gs_score_batched(None, d, 0, 0, None) == gs.GS_EINVAL
    del fake
    b.close()


def test_workspace_cap_forces_enomem_before_the_device(gs, monkeypatch):
    """GS_WORKSPACE_LIMIT below the plan's workspace: gs_score_all and gs_score_backward
    fail with GS_ENOMEM during argument processing, before any device call (the data
    pointers here are never dereferenced)."""
    m, n = 12, 300
    p = gs.Plan(m)
    need = p.workspace_bytes(n)
    need_bw = p.workspace_bytes(n, backward=True)
    assert 0 < need < need_bw
    info = p.info
    # anchors of every segment (FP64 slots), their tails, two TSQR buffers: a lower bound
    assert need >= info["num_segments"] * (info["k"] + 1) * 32 * 8 + 2 * ((n + 127) // 128) * m * m * 8
    fake = ctypes.c_void_p(0x100000)
    L = gs.lib()
    monkeypatch.setenv("GS_WORKSPACE_LIMIT", str(need - 1))
    assert L.gs_score_all(p.handle, fake, n, m, m, fake, gs.GS_OK, None) == gs._abi.GS_ENOMEM
    assert "GS_WORKSPACE_LIMIT" in gs.last_error()
    monkeypatch.setenv("GS_WORKSPACE_LIMIT", str(need_bw - 1))
    assert L.gs_score_backward(p.handle, fake, n, m, m, fake, 0, fake, m, None) == gs._abi.GS_ENOMEM
    monkeypatch.setenv("GS_WORKSPACE_LIMIT", "not-a-number")
    assert L.gs_score_all(p.handle, fake, n, m, m, fake, 0, None) == gs.GS_EINVAL
