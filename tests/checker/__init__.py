"""ctypes binding of the brute-force raster checker (test infrastructure).

The checker is independent of both the oracle and the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "raster_check.c")
LIB = os.path.join(HERE, "libraster_check.so")

I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)
U8P = ctypes.POINTER(ctypes.c_uint8)

_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-shared", "-fPIC", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        L.tabi_check_raster.argtypes = [I64P, I64P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int64, U8P,
                                        ctypes.POINTER(ctypes.c_long)]
        L.tabi_check_raster.restype = ctypes.c_long
        L.tabi_check_layout.argtypes = [I32P, I32P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, I32P, U8P, ctypes.c_int32, I64P]
        L.tabi_check_layout.restype = ctypes.c_long
        L.tabi_check_layout_ks.argtypes = [I32P, I32P, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_int32, I32P, U8P, I32P, I64P]
        L.tabi_check_layout_ks.restype = ctypes.c_long
        _lib = L
    return _lib


def raster(X, Y, bx, by, bw, bh):
    """Coverage mask (bh, bw) of a Q14 polygon, window origin (bx, by)."""
    X = np.ascontiguousarray(X, np.int64)
    Y = np.ascontiguousarray(Y, np.int64)
    mask = np.zeros((bh, bw), np.uint8)
    out = ctypes.c_long(0)
    lib().tabi_check_raster(X.ctypes.data_as(I64P), Y.ctypes.data_as(I64P), X.shape[0], bx, by,
                            bw, bh, mask.ctypes.data_as(U8P), ctypes.byref(out))
    return mask, int(out.value)


def check_layout(inp, out_xy, out_orient, k):
    """Returns dict(overlap, outside, covered, empty)."""
    xy = np.ascontiguousarray(inp.xy, np.int32)
    off = np.ascontiguousarray(inp.offsets, np.int32)
    oxy = np.ascontiguousarray(np.asarray(out_xy).reshape(-1), np.int32)
    ori = np.ascontiguousarray(out_orient, np.uint8)
    st = np.zeros(4, np.int64)
    lib().tabi_check_layout(xy.ctypes.data_as(I32P), off.ctypes.data_as(I32P), inp.n, inp.atlas_w,
                            inp.atlas_h, inp.padding, oxy.ctypes.data_as(I32P),
                            ori.ctypes.data_as(U8P), int(k), st.ctypes.data_as(I64P))
    return dict(overlap=int(st[0]), outside=int(st[1]), covered=int(st[2]), empty=int(st[3]))


def check_layout_ks(inp, out_xy, out_orient, ks):
    """check_layout with a scale ks[c]/64 of its own for every chart."""
    xy = np.ascontiguousarray(inp.xy, np.int32)
    off = np.ascontiguousarray(inp.offsets, np.int32)
    oxy = np.ascontiguousarray(np.asarray(out_xy).reshape(-1), np.int32)
    ori = np.ascontiguousarray(out_orient, np.uint8)
    kk = np.ascontiguousarray(ks, np.int32)
    st = np.zeros(4, np.int64)
    lib().tabi_check_layout_ks(xy.ctypes.data_as(I32P), off.ctypes.data_as(I32P), inp.n,
                               inp.atlas_w, inp.atlas_h, inp.padding, oxy.ctypes.data_as(I32P),
                               ori.ctypes.data_as(U8P), kk.ctypes.data_as(I32P),
                               st.ctypes.data_as(I64P))
    return dict(overlap=int(st[0]), outside=int(st[1]), covered=int(st[2]), empty=int(st[3]))


def atlas_polygons(inp, out_xy, out_orient, k):
    """Exact Q14 atlas polygons (list of (m,2) int64) from the output contract.

    bit0 quarter turn (u,v) -> (h0 - v, u); bit1 / bit2 mirror inside the
    chart box in x / y; scale by k (Q8 -> Q14 at k/64); bit3 mirror inside the
    scaled texel box; translate by the output texel position.
    """
    polys = []
    for c in range(inp.n):
        P = inp.chart(c).astype(np.int64)
        u = P[:, 0] - P[:, 0].min()
        v = P[:, 1] - P[:, 1].min()
        w0, h0 = int(u.max()), int(v.max())
        o = int(out_orient[c])
        if o & 1:
            u, v = h0 - v, u
            W, H = h0, w0
        else:
            W, H = w0, h0
        if o & 2:
            u = W - u
        if o & 4:
            v = H - v
        U, V = k * u, k * v
        wt = -(-k * W // 16384)
        if o & 8:
            U = 16384 * wt - U
        polys.append(np.stack([16384 * int(out_xy[c][0]) + U, 16384 * int(out_xy[c][1]) + V], 1))
    return polys
