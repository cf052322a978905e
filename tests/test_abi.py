"""The C-ABI library loads and exports every entry point its header declares
(no GPU work: nothing is called)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tabi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tabi_\w+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("tabi_pack", "tabi_pack_many"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2602_07782_amd as tabi
    if not os.path.exists(tabi.LIB_PATH):
        pytest.fail("libtabi_hip.so is not built; run `python -m paper_2602_07782_amd.build`")
    L = ctypes.CDLL(tabi.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(tabi.EXPORTS) <= set(declared_functions())


def test_binding_fails_loudly_without_library(monkeypatch):
    import paper_2602_07782_amd as tabi
    monkeypatch.setattr(tabi, "_lib", None)
    monkeypatch.setattr(tabi, "LIB_PATH", "/nonexistent/libtabi_hip.so")
    with pytest.raises(RuntimeError):
        tabi.lib()


def test_lds_plan_is_host_only():
    import paper_2602_07782_amd as tabi
    if not os.path.exists(tabi.LIB_PATH):
        pytest.skip("library not built")
    b = tabi.lib().tabi_pack_lds_bytes(2000, 2048, 2)
    assert b > 4 * 2050


def test_padding_limit_and_arena_sizing_are_host_only():
    """Padding above TABI_MAX_PADDING is refused before any device work, and
    the stored-profile arena is part of the batched work space."""
    import paper_2602_07782_amd as tabi
    if not os.path.exists(tabi.LIB_PATH):
        pytest.skip("library not built")
    L = tabi.lib()
    hdr = open(os.path.join(ROOT, "include", "tabi.h")).read()
    maxp = int(re.search(r"#define TABI_MAX_PADDING (\d+)", hdr).group(1))
    ws = L.tabi_pack_many_workspace_bytes
    ws.restype = ctypes.c_int64
    assert ws(4, 8000, 2000, 2048, maxp, 2) > 0
    assert ws(4, 8000, 2000, 2048, maxp + 1, 2) == -1
    full = ws(4, 8000, 2000, 2048, 2, 2)
    tabi.debug_set_profile_cap(0)
    try:
        none = ws(4, 8000, 2000, 2048, 2, 2)
    finally:
        tabi.debug_set_profile_cap(-1)
    # 8 scale slots x 8000 charts x 96 words + 8 x 4 x 4 x 2050 words
    assert full - none >= 4 * (8 * 8000 * 96 + 8 * 4 * 4 * 2050)


def test_serving_context_refuses_bad_arguments_on_the_host():
    """Configuration and request checks of the serving context come before
    any HIP call, so they run without a GPU."""
    import paper_2602_07782_amd as tabi
    if not os.path.exists(tabi.LIB_PATH):
        pytest.skip("library not built")
    L = tabi.lib()
    h = ctypes.c_void_p()
    for bad in [tabi.CtxConfig(3, 2, 4, 16, 1 << 30, 1 << 20),     # quality
                tabi.CtxConfig(2, 33, 4, 16, 1 << 30, 1 << 20),    # padding
                tabi.CtxConfig(2, 2, 0, 16, 1 << 30, 1 << 20),     # streams
                tabi.CtxConfig(2, 2, 4, 0, 1 << 30, 1 << 20),      # batch
                tabi.CtxConfig(2, 2, 4, 16, 1000, 1 << 20),        # device budget
                tabi.CtxConfig(2, 2, 4, 16, 1 << 30, 100)]:        # staging
        assert L.tabi_ctx_create(ctypes.byref(bad), ctypes.byref(h)) == tabi.TABI_EINVAL
        assert not h.value
    assert L.tabi_ctx_create(None, ctypes.byref(h)) == tabi.TABI_EINVAL
    i32, i64 = ctypes.c_int32(), ctypes.c_int64()
    assert L.tabi_submit(None, None, None, 1, 64, 64, None, None, None, ctypes.byref(i32),
                         ctypes.byref(i64)) == tabi.TABI_EINVAL
    assert L.tabi_repack(None, 0, None, 1, None, None, None, None, None,
                         ctypes.byref(i64)) == tabi.TABI_EINVAL
    assert L.tabi_poll(None, 0, None, 0, ctypes.byref(i32)) == tabi.TABI_EINVAL
    assert L.tabi_ctx_destroy(None) == tabi.TABI_EINVAL


def test_timing_stage_mask_is_checked_on_the_host():
    """tabi_timing_stages takes a non-empty mask of the six stages (host
    state only: no device work)."""
    import paper_2602_07782_amd as tabi
    if not os.path.exists(tabi.LIB_PATH):
        pytest.skip("library not built")
    L = tabi.lib()
    hdr = open(os.path.join(ROOT, "include", "tabi.h")).read()
    einval = int(re.search(r"TABI_EINVAL = (-?\d+)", hdr).group(1))
    assert L.tabi_timing_stages(0) == einval
    assert L.tabi_timing_stages(1 << 6) == einval
    assert L.tabi_timing_stages(1 << tabi.STAGES.index("pack")) == 0
    tabi.timing_stages(None)  # every stage again
    with pytest.raises(RuntimeError):
        tabi._check(L.tabi_timing_stages(0))
