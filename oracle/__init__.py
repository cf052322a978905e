"""ctypes binding of the TABI oracle (plain C, host only).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  The GPU library
never uses it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libtabi_oracle.so")
SRC = os.path.join(HERE, "tabi_oracle.c")

I32P = ctypes.POINTER(ctypes.c_int32)
U8P = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (host only)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class OrcChart(ctypes.Structure):
    _fields_ = [("valid", ctypes.c_int32), ("rot", ctypes.c_int32), ("flipx", ctypes.c_int32),
                ("flipy", ctypes.c_int32), ("xmin", ctypes.c_int64), ("ymin", ctypes.c_int64),
                ("W", ctypes.c_int64), ("H", ctypes.c_int64), ("K", ctypes.c_int32),
                ("ylo", ctypes.c_int64 * 10), ("yhi", ctypes.c_int64 * 10),
                ("xlo", ctypes.c_int64 * 10), ("xhi", ctypes.c_int64 * 10),
                ("obb", ctypes.c_int32), ("obb_m", ctypes.c_int32),
                ("C", ctypes.c_int64), ("S", ctypes.c_int64), ("a", ctypes.c_int64),
                ("b", ctypes.c_int64), ("e", ctypes.c_int64), ("f", ctypes.c_int64),
                ("area2", ctypes.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        L.tabi_oracle_pack.argtypes = [I32P, I32P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, I32P, U8P,
                                       ctypes.POINTER(ctypes.c_float), I32P]
        L.tabi_oracle_feasible.argtypes = [I32P, I32P, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, I32P, U8P, I32P]
        L.tabi_oracle_order.argtypes = [I32P, I32P, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, I32P, I32P]
        L.tabi_oracle_pairs.argtypes = [I32P, I32P, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, I32P, U8P]
        L.orc_prep_chart.argtypes = [I32P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(OrcChart)]
        L.orc_prep_chart_loops.argtypes = [I32P, I32P, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(OrcChart)]
        L.orc_prep_chart_ex.argtypes = [I32P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(OrcChart)]
        i32 = ctypes.c_int32
        L.tabi_oracle_pack_hybrid.argtypes = [I32P, I32P, i32, i32, i32, i32, i32, i32, I32P, U8P,
                                              I32P, I32P]
        L.tabi_oracle_feasible_hybrid.argtypes = [I32P, I32P, i32, i32, i32, i32, i32, i32, i32,
                                                  I32P, I32P, U8P, I32P, I32P]
        L.orc_prerotate.argtypes = [I32P, ctypes.c_int32, I32P, I32P]
        L.tabi_oracle_pack_prerotate.argtypes = [I32P, I32P, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                 I32P, U8P, U8P, ctypes.POINTER(ctypes.c_float),
                                                 I32P]
        L.tabi_oracle_pack_loops.argtypes = [I32P, I32P, I32P, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, I32P,
                                             U8P, ctypes.POINTER(ctypes.c_float), I32P]
        L.tabi_oracle_pack_method.argtypes = [I32P, I32P, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32, I32P, U8P,
                                              ctypes.POINTER(ctypes.c_float), I32P]
        L.orc_profiles.argtypes = [ctypes.POINTER(OrcChart), ctypes.c_int32, I32P, I32P,
                                   I32P, I32P, I32P, I32P]
        L.orc_row_proxies.argtypes = [ctypes.POINTER(OrcChart), ctypes.c_int32, I32P, I32P, I32P,
                                      I32P, I32P]
        L.orc_knee_update.argtypes = [I32P, ctypes.c_int32, ctypes.c_int32, I32P, I32P]
        L.orc_quality.argtypes = [ctypes.c_int32, ctypes.c_int32, I32P, I32P]
        L.orc_interlock.argtypes = [I32P, ctypes.c_int32, ctypes.c_int32, I32P, ctypes.c_int32,
                                    ctypes.c_int32]
        _lib = L
    return _lib


def _p32(a):
    return a.ctypes.data_as(I32P)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def pack(inp):
    """Whole pack -> (out_xy int32[n,2], out_orient uint8[n], scale float, k int)."""
    n = inp.n
    xy, off = _c(inp.xy, np.int32), _c(inp.offsets, np.int32)
    oxy = np.zeros(max(2 * n, 1), np.int32)
    ori = np.zeros(max(n, 1), np.uint8)
    sc = ctypes.c_float(0)
    kk = ctypes.c_int32(0)
    rc = lib().tabi_oracle_pack(_p32(xy), _p32(off), n, inp.atlas_w, inp.atlas_h, inp.padding,
                                inp.quality, _p32(oxy), ori.ctypes.data_as(U8P),
                                ctypes.byref(sc), ctypes.byref(kk))
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")
    return oxy[:2 * n].reshape(n, 2), ori[:n], float(sc.value), int(kk.value)


FULL, TIGHT_ONLY, BALANCED_ONLY = 0, 1, 2


def pack_method(inp, K, topt, variant):
    """Whole pack with the method's knobs (K slices, t_opt percent or -1 for
    the paper's setting, variant) -> as pack()."""
    n = inp.n
    xy, off = _c(inp.xy, np.int32), _c(inp.offsets, np.int32)
    oxy = np.zeros(max(2 * n, 1), np.int32)
    ori = np.zeros(max(n, 1), np.uint8)
    sc = ctypes.c_float(0)
    kk = ctypes.c_int32(0)
    rc = lib().tabi_oracle_pack_method(_p32(xy), _p32(off), n, inp.atlas_w, inp.atlas_h,
                                       inp.padding, int(K), int(topt), int(variant), _p32(oxy),
                                       ori.ctypes.data_as(U8P), ctypes.byref(sc),
                                       ctypes.byref(kk))
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")
    return oxy[:2 * n].reshape(n, 2), ori[:n], float(sc.value), int(kk.value)


def pack_hybrid(inp, K=10, topt=-1):
    """Whole pack with the hybrid tail -> (xy, orient, per-chart k, head k)."""
    n = inp.n
    xy, off = _c(inp.xy, np.int32), _c(inp.offsets, np.int32)
    oxy = np.zeros(max(2 * n, 1), np.int32)
    ori = np.zeros(max(n, 1), np.uint8)
    ks = np.zeros(max(n, 1), np.int32)
    kk = ctypes.c_int32(0)
    rc = lib().tabi_oracle_pack_hybrid(_p32(xy), _p32(off), n, inp.atlas_w, inp.atlas_h,
                                       inp.padding, int(K), int(topt), _p32(oxy),
                                       ori.ctypes.data_as(U8P), _p32(ks), ctypes.byref(kk))
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")
    return oxy[:2 * n].reshape(n, 2), ori[:n], ks[:n], int(kk.value)


def feasible_hybrid(inp, k, K=10, topt=0):
    """One candidate k of the hybrid pack -> (ok, xs, ys, mir (sorted order),
    t0, kt)."""
    n = inp.n
    xy, off = _c(inp.xy, np.int32), _c(inp.offsets, np.int32)
    xs = np.zeros(max(n, 1), np.int32)
    ys = np.zeros(max(n, 1), np.int32)
    mir = np.zeros(max(n, 1), np.uint8)
    t0, kt = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = lib().tabi_oracle_feasible_hybrid(_p32(xy), _p32(off), n, inp.atlas_w, inp.atlas_h,
                                           inp.padding, int(K), int(topt), int(k), _p32(xs),
                                           _p32(ys), mir.ctypes.data_as(U8P), ctypes.byref(t0),
                                           ctypes.byref(kt))
    if rc < 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")
    return bool(rc), xs[:n], ys[:n], mir[:n], int(t0.value), int(kt.value)


def prerotate(verts_q8):
    """Pre-rotation of one chart: (rotated Q8 vertices (m,2), direction m)."""
    v = _c(verts_q8, np.int32).reshape(-1)
    out = np.zeros_like(v)
    m = ctypes.c_int32(0)
    lib().orc_prerotate(_p32(v), int(v.shape[0] // 2), _p32(out), ctypes.byref(m))
    return out.reshape(-1, 2), int(m.value)


def pack_prerotate(inp):
    """Whole pack after pre-rotation -> (xy, orient, scale, k, directions)."""
    n = inp.n
    xy, off = _c(inp.xy, np.int32), _c(inp.offsets, np.int32)
    oxy = np.zeros(max(2 * n, 1), np.int32)
    ori = np.zeros(max(n, 1), np.uint8)
    dirs = np.zeros(max(n, 1), np.uint8)
    sc = ctypes.c_float(0)
    kk = ctypes.c_int32(0)
    rc = lib().tabi_oracle_pack_prerotate(_p32(xy), _p32(off), n, inp.atlas_w, inp.atlas_h,
                                          inp.padding, inp.quality, _p32(oxy),
                                          ori.ctypes.data_as(U8P), dirs.ctypes.data_as(U8P),
                                          ctypes.byref(sc), ctypes.byref(kk))
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")
    return oxy[:2 * n].reshape(n, 2), ori[:n], float(sc.value), int(kk.value), dirs[:n]


def pack_loops(inp):
    """Whole pack of a LoopsInput (charts of several loops) -> as pack()."""
    n = inp.n
    xy = _c(inp.xy, np.int32)
    lo, cl = _c(inp.loop_offsets, np.int32), _c(inp.chart_loops, np.int32)
    oxy = np.zeros(max(2 * n, 1), np.int32)
    ori = np.zeros(max(n, 1), np.uint8)
    sc = ctypes.c_float(0)
    kk = ctypes.c_int32(0)
    rc = lib().tabi_oracle_pack_loops(_p32(xy), _p32(lo), _p32(cl), n, inp.atlas_w, inp.atlas_h,
                                      inp.padding, inp.quality, _p32(oxy),
                                      ori.ctypes.data_as(U8P), ctypes.byref(sc), ctypes.byref(kk))
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")
    return oxy[:2 * n].reshape(n, 2), ori[:n], float(sc.value), int(kk.value)


def prep_chart_loops(loops_q8, K):
    """Proxy record of a chart of several loops (list of (m,2) Q8 arrays)."""
    v = np.ascontiguousarray(np.concatenate([np.asarray(L).reshape(-1) for L in loops_q8]),
                             np.int32)
    lofs = np.zeros(len(loops_q8) + 1, np.int32)
    lofs[1:] = np.cumsum([len(L) for L in loops_q8])
    ch = OrcChart()
    lib().orc_prep_chart_loops(_p32(v), _p32(lofs), len(loops_q8), int(K), ctypes.byref(ch))
    return ch


def prep_chart_ex(verts_q8, K, use_obb):
    v = _c(verts_q8, np.int32).reshape(-1)
    ch = OrcChart()
    lib().orc_prep_chart_ex(_p32(v), int(v.shape[0] // 2), int(K), int(use_obb), ctypes.byref(ch))
    return ch


def feasible(inp, k):
    n = inp.n
    xy, off = _c(inp.xy, np.int32), _c(inp.offsets, np.int32)
    oxy = np.zeros(max(2 * n, 1), np.int32)
    ori = np.zeros(max(n, 1), np.uint8)
    rows = ctypes.c_int32(0)
    rc = lib().tabi_oracle_feasible(_p32(xy), _p32(off), n, inp.atlas_w, inp.atlas_h, inp.padding,
                                    inp.quality, int(k), _p32(oxy), ori.ctypes.data_as(U8P),
                                    ctypes.byref(rows))
    if rc < 0:
        raise ValueError("bad arguments")
    return bool(rc), oxy[:2 * n].reshape(n, 2), ori[:n], int(rows.value)


def order(inp):
    n = inp.n
    xy, off = _c(inp.xy, np.int32), _c(inp.offsets, np.int32)
    perm = np.zeros(max(n, 1), np.int32)
    khi = ctypes.c_int32(0)
    rc = lib().tabi_oracle_order(_p32(xy), _p32(off), n, inp.atlas_w, inp.atlas_h, inp.quality,
                                 _p32(perm), ctypes.byref(khi))
    if rc != 0:
        raise ValueError("bad arguments")
    return perm[:n], int(khi.value)


def pairs(inp, k):
    n = inp.n
    xy, off = _c(inp.xy, np.int32), _c(inp.offsets, np.int32)
    cd = np.zeros(max(n, 1), np.int32)
    fl = np.zeros(max(n, 1), np.uint8)
    rc = lib().tabi_oracle_pairs(_p32(xy), _p32(off), n, inp.padding, inp.quality, int(k),
                                 _p32(cd), fl.ctypes.data_as(U8P))
    if rc != 0:
        raise ValueError("bad arguments")
    return cd[:n], fl[:n]


def quality(q, n):
    K, t = ctypes.c_int32(0), ctypes.c_int32(0)
    lib().orc_quality(q, n, ctypes.byref(K), ctypes.byref(t))
    return int(K.value), int(t.value)


def prep_chart(verts_q8, K):
    """verts_q8: (m,2) int array.  Returns an OrcChart (valid == 0 if degenerate)."""
    v = _c(np.asarray(verts_q8).reshape(-1), np.int32)
    ch = OrcChart()
    lib().orc_prep_chart(_p32(v), int(v.shape[0] // 2), int(K), ctypes.byref(ch))
    return ch


def profiles(ch, k):
    """Undilated per-texel profiles of a prepped chart at k: (top, bot, left, right)."""
    W, H = int(ch.W), int(ch.H)
    w = -(-k * W // 16384)
    h = -(-k * H // 16384)
    top = np.zeros(max(w, 1), np.int32)
    bot = np.zeros(max(w, 1), np.int32)
    left = np.zeros(max(h, 1), np.int32)
    right = np.zeros(max(h, 1), np.int32)
    ww, hh = ctypes.c_int32(0), ctypes.c_int32(0)
    lib().orc_profiles(ctypes.byref(ch), int(k), ctypes.byref(ww), ctypes.byref(hh), _p32(top),
                       _p32(bot), _p32(left), _p32(right))
    assert ww.value == w and hh.value == h
    return top[:w], bot[:w], left[:h], right[:h]


def row_proxies(ch, k):
    """Undilated per-proxy row bounds at k: (la, ra) local AABBs, (lo, ro) OBB."""
    h = -(-k * int(ch.H) // 16384)
    out = [np.zeros(max(h, 1), np.int32) for _ in range(4)]
    hh = ctypes.c_int32(0)
    lib().orc_row_proxies(ctypes.byref(ch), int(k), ctypes.byref(hh), *[_p32(a) for a in out])
    assert hh.value == h
    return tuple(a[:h] for a in out)


def knee_update(F, direction, left, right):
    """Alg. 4 on frontline F: returns (active, left, right)."""
    f = _c(F, np.int32)
    lft, rgt = ctypes.c_int32(left), ctypes.c_int32(right)
    act = lib().orc_knee_update(_p32(f), f.shape[0], int(direction), ctypes.byref(lft),
                                ctypes.byref(rgt))
    return bool(act), int(lft.value), int(rgt.value)


def interlock(rightA, wdA, leftB, d):
    rA = _c(rightA, np.int32)
    lB = _c(leftB, np.int32)
    return int(lib().orc_interlock(_p32(rA), rA.shape[0], int(wdA), _p32(lB), lB.shape[0], int(d)))


def correct(pairs_arr, y):
    """Alg. 1 fixpoint: pairs_arr (m,3) int rows (A, B, flags); returns new y."""
    pa = _c(np.asarray(pairs_arr).reshape(-1), np.int32)
    yy = _c(y, np.int32).copy()
    L = lib()
    L.orc_correct.argtypes = [ctypes.c_int32, I32P, I32P]
    L.orc_correct(int(pa.shape[0] // 3), _p32(pa) if pa.size else None, _p32(yy))
    return yy
