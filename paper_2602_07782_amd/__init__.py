"""MI355X (gfx950) implementation of TABI atlas packing.

Thin ctypes binding over the C ABI in ``include/tabi.h``.  Every step of the
packing path runs in the HIP kernels of ``libtabi_hip.so``; this module only
allocates output tensors with PyTorch (device memory and streams) and passes
raw pointers.  There is no CPU fallback: without the built library every call
raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtabi_hip.so")

TABI_OK, TABI_EINVAL, TABI_ENOMEM, TABI_EHIP, TABI_ETOOBIG, TABI_ENOTRESIDENT = 0, -1, -2, -3, -4, -5
ERRORS = {TABI_EINVAL: "invalid argument", TABI_ENOMEM: "out of device memory",
          TABI_EHIP: "HIP runtime error",
          TABI_ETOOBIG: "input exceeds the work space available to it",
          TABI_ENOTRESIDENT: "atlas records no longer resident"}


class TabiError(RuntimeError):
    def __init__(self, code, detail=""):
        super().__init__(f"tabi error {code}: {ERRORS.get(code, 'unknown')} {detail}".strip())
        self.code = code


class Charts(ctypes.Structure):
    _fields_ = [("xy", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("total_verts", ctypes.c_int32)]


class ChartsLoops(ctypes.Structure):
    _fields_ = [("xy", ctypes.c_void_p), ("loop_offsets", ctypes.c_void_p),
                ("chart_loops", ctypes.c_void_p), ("total_loops", ctypes.c_int32)]


class Method(ctypes.Structure):
    _fields_ = [("slices", ctypes.c_int32), ("topt_percent", ctypes.c_int32),
                ("variant", ctypes.c_int32)]


FULL, TIGHT_ONLY, BALANCED_ONLY = 0, 1, 2


class CtxConfig(ctypes.Structure):
    _fields_ = [("quality", ctypes.c_int32), ("padding", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("staging_bytes", ctypes.c_int64)]


class Done(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("atlas_id", ctypes.c_int32),
                ("status", ctypes.c_int32), ("batch", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("latency_ms", ctypes.c_double), ("submit_ms", ctypes.c_double),
                ("done_ms", ctypes.c_double)]


_lib = None
EXPORTS = ["tabi_pack", "tabi_pack_loops", "tabi_pack_prerotate", "tabi_pack_hybrid", "tabi_pack_method", "tabi_pack_many_method", "tabi_pack_noalloc",
           "tabi_pack_many", "tabi_pack_many_ws", "tabi_submit_with", "tabi_pack_many_workspace_bytes",
           "tabi_record_bytes", "tabi_prep_records", "tabi_splice_records",
           "tabi_pack_many_records", "tabi_debug_order", "tabi_debug_pairs",
           "tabi_debug_feasible", "tabi_debug_phase_clock", "tabi_strerror", "tabi_last_hip_error", "tabi_pack_lds_bytes",
           "tabi_timing_enable", "tabi_timing_stages", "tabi_timing_read", "tabi_timing_reset",
           "tabi_debug_set_stage_cap", "tabi_debug_set_pack_lds", "tabi_debug_set_profile_cap", "tabi_tune_many",
           "tabi_many_shape", "tabi_many_shape_count", "tabi_debug_set_many_shape",
           "tabi_shutdown", "tabi_ctx_create", "tabi_ctx_destroy", "tabi_submit", "tabi_repack",
           "tabi_poll", "tabi_ctx_stats"]
STAGES = ["prep", "sort", "setup", "profile", "pack", "select"]


def lib():
    """Load libtabi_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2602_07782_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        L.tabi_pack.argtypes = [ctypes.POINTER(Charts), i32, i32, i32, i32, i32, vp, vp, vp, vp]
        L.tabi_pack_noalloc.argtypes = [ctypes.POINTER(Charts), i32, i32, i32, i32, i32, vp, vp,
                                        vp, vp]
        L.tabi_pack_loops.argtypes = [ctypes.POINTER(ChartsLoops), i32, i32, i32, i32, i32, vp,
                                      vp, vp, vp]
        L.tabi_pack_hybrid.argtypes = [ctypes.POINTER(Charts), i32, i32, i32, i32,
                                       ctypes.POINTER(Method), vp, vp, vp, vp, vp]
        L.tabi_pack_prerotate.argtypes = [ctypes.POINTER(Charts), i32, i32, i32, i32, i32, vp,
                                          vp, vp, vp, vp, vp]
        L.tabi_pack_method.argtypes = [ctypes.POINTER(Charts), i32, i32, i32, i32,
                                       ctypes.POINTER(Method), vp, vp, vp, vp]
        L.tabi_pack_many_method.argtypes = [vp, vp, vp, i32, vp, i32, i32, i32, i32,
                                            ctypes.POINTER(Method), vp, vp, vp, vp]
        L.tabi_pack_many.argtypes = [vp, vp, vp, i32, vp, i32, i32, i32, i32, i32, vp, vp, vp, vp]
        L.tabi_pack_many_workspace_bytes.argtypes = [i32, i32, i32, i32, i32, i32]
        L.tabi_pack_many_workspace_bytes.restype = ctypes.c_int64
        L.tabi_pack_many_ws.argtypes = [vp, vp, vp, i32, vp, i32, i32, i32, i32, i32, vp, vp, vp,
                                        vp, ctypes.c_int64, vp]
        L.tabi_record_bytes.restype = ctypes.c_int64
        L.tabi_prep_records.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp]
        L.tabi_splice_records.argtypes = [vp, vp, i32, vp, vp]
        L.tabi_pack_many_records.argtypes = [vp, vp, i32, vp, i32, i32, i32, i32, i32, vp, vp, vp,
                                             vp]
        L.tabi_debug_order.argtypes = [ctypes.POINTER(Charts), i32, i32, i32, i32, i32, vp, vp, vp]
        L.tabi_debug_pairs.argtypes = [ctypes.POINTER(Charts), i32, i32, i32, i32, vp, vp, vp]
        L.tabi_debug_feasible.argtypes = [ctypes.POINTER(Charts), i32, i32, i32, i32, i32, i32,
                                          vp, vp, vp, vp, vp]
        L.tabi_strerror.restype = ctypes.c_char_p
        L.tabi_last_hip_error.restype = ctypes.c_char_p
        L.tabi_pack_lds_bytes.argtypes = [i32, i32, i32]
        L.tabi_pack_lds_bytes.restype = ctypes.c_int64
        L.tabi_timing_enable.argtypes = [ctypes.c_int]
        L.tabi_timing_stages.argtypes = [ctypes.c_uint32]
        L.tabi_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int32), i32]
        L.tabi_timing_reset.restype = None
        L.tabi_debug_set_stage_cap.argtypes = [i32]
        L.tabi_debug_set_pack_lds.argtypes = [i32]
        L.tabi_debug_set_profile_cap.argtypes = [ctypes.c_int64]
        L.tabi_tune_many.argtypes = [vp, vp, vp, i32, vp, i32, i32, i32, i32, i32, vp, vp, vp, i32,
                                     vp, vp, vp]
        L.tabi_many_shape.argtypes = [i32, i32, vp]
        L.tabi_many_shape_count.restype = i32
        L.tabi_debug_set_many_shape.argtypes = [i32, i32]
        L.tabi_ctx_create.argtypes = [ctypes.POINTER(CtxConfig), ctypes.POINTER(vp)]
        L.tabi_ctx_destroy.argtypes = [vp]
        L.tabi_submit.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp,
                                  ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64)]
        L.tabi_repack.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp, vp,
                                  ctypes.POINTER(ctypes.c_int64)]
        L.tabi_submit_with.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, vp, vp, vp,
                                       ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64)]
        L.tabi_poll.argtypes = [vp, i32, ctypes.POINTER(Done), i32, ctypes.POINTER(i32)]
        L.tabi_ctx_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), i32]
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _check(rc):
    if rc != TABI_OK:
        detail = lib().tabi_last_hip_error().decode() if rc == TABI_EHIP else ""
        raise TabiError(rc, detail)


def _dev_i32(a, device):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=torch.int32)
    else:
        import numpy as np
        t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(device)
    return t.contiguous()


def _charts(xy, offsets):
    n = int(offsets.numel()) - 1
    c = Charts(_ptr(xy).value, _ptr(offsets).value, int(xy.numel() // 2))
    return c, n


def pack(xy, offsets, atlas_w, atlas_h, padding, quality, stream=None, device="cuda"):
    """tabi_pack.  xy: int32[2V] (Q8), offsets: int32[n+1] (device tensors or
    arrays).  Returns (out_xy int32[n,2], out_orient uint8[n], out_scale
    float32[1]) on the device; enqueued on `stream` (default: current)."""
    torch = _torch()
    xy = _dev_i32(xy, device)
    offsets = _dev_i32(offsets, device)
    ch, n = _charts(xy, offsets)
    out_xy = torch.empty((max(n, 0), 2), dtype=torch.int32, device=xy.device)
    out_or = torch.empty(max(n, 0), dtype=torch.uint8, device=xy.device)
    out_sc = torch.empty(1, dtype=torch.float32, device=xy.device)
    _check(lib().tabi_pack(ctypes.byref(ch), n, int(atlas_w), int(atlas_h), int(padding),
                           int(quality), _ptr(out_xy), _ptr(out_or), _ptr(out_sc), _stream(stream)))
    return out_xy, out_or, out_sc


def pack_loops(xy, loop_offsets, chart_loops, atlas_w, atlas_h, padding, quality, stream=None,
               device="cuda"):
    """tabi_pack_loops: charts of one or more boundary loops (loop l:
    vertices [loop_offsets[l], loop_offsets[l+1]), chart c: loops
    [chart_loops[c], chart_loops[c+1])).  Returns as pack()."""
    torch = _torch()
    xy = _dev_i32(xy, device)
    lo = _dev_i32(loop_offsets, device)
    cl = _dev_i32(chart_loops, device)
    n = int(cl.numel()) - 1
    ch = ChartsLoops(_ptr(xy).value, _ptr(lo).value, _ptr(cl).value, int(lo.numel()) - 1)
    out_xy = torch.empty((max(n, 0), 2), dtype=torch.int32, device=xy.device)
    out_or = torch.empty(max(n, 0), dtype=torch.uint8, device=xy.device)
    out_sc = torch.empty(1, dtype=torch.float32, device=xy.device)
    _check(lib().tabi_pack_loops(ctypes.byref(ch), n, int(atlas_w), int(atlas_h), int(padding),
                                 int(quality), _ptr(out_xy), _ptr(out_or), _ptr(out_sc),
                                 _stream(stream)))
    return out_xy, out_or, out_sc


def pack_hybrid(xy, offsets, atlas_w, atlas_h, padding, slices=10, topt_percent=-1,
                stream=None, device="cuda"):
    """tabi_pack_hybrid: the full method with the hybrid tail.  Returns
    (out_xy int32[n,2], out_orient uint8[n], out_chart_scale float32[n],
    out_scale float32[1]) on the device."""
    torch = _torch()
    xy = _dev_i32(xy, device)
    offsets = _dev_i32(offsets, device)
    ch, n = _charts(xy, offsets)
    out_xy = torch.empty((max(n, 0), 2), dtype=torch.int32, device=xy.device)
    out_or = torch.empty(max(n, 0), dtype=torch.uint8, device=xy.device)
    out_ks = torch.empty(max(n, 0), dtype=torch.float32, device=xy.device)
    out_sc = torch.empty(1, dtype=torch.float32, device=xy.device)
    m = Method(int(slices), int(topt_percent), 0)
    _check(lib().tabi_pack_hybrid(ctypes.byref(ch), n, int(atlas_w), int(atlas_h), int(padding),
                                  ctypes.byref(m), _ptr(out_xy), _ptr(out_or), _ptr(out_ks),
                                  _ptr(out_sc), _stream(stream)))
    return out_xy, out_or, out_ks, out_sc


def pack_prerotate(xy, offsets, atlas_w, atlas_h, padding, quality, stream=None, device="cuda",
                   in_place=False):
    """tabi_pack_prerotate: every chart turned to its least-area box over 64
    directions, then packed.  Returns (turned xy int32[2V], direction uint8[n],
    out_xy, out_orient, out_scale) on the device; with in_place the turned
    vertices overwrite `xy` (a device int32 tensor)."""
    torch = _torch()
    xy = _dev_i32(xy, device)
    offsets = _dev_i32(offsets, device)
    ch, n = _charts(xy, offsets)
    rxy = xy if in_place else torch.empty_like(xy)
    out_dir = torch.empty(max(n, 0), dtype=torch.uint8, device=xy.device)
    out_xy = torch.empty((max(n, 0), 2), dtype=torch.int32, device=xy.device)
    out_or = torch.empty(max(n, 0), dtype=torch.uint8, device=xy.device)
    out_sc = torch.empty(1, dtype=torch.float32, device=xy.device)
    _check(lib().tabi_pack_prerotate(ctypes.byref(ch), n, int(atlas_w), int(atlas_h),
                                     int(padding), int(quality), _ptr(rxy), _ptr(out_dir),
                                     _ptr(out_xy), _ptr(out_or), _ptr(out_sc), _stream(stream)))
    return rxy, out_dir, out_xy, out_or, out_sc


def pack_method(xy, offsets, atlas_w, atlas_h, padding, slices, topt_percent, variant,
                stream=None, device="cuda"):
    """tabi_pack_method: the method's knobs (local AABBs per axis, t_opt in
    percent or -1 for the paper's setting, variant FULL / TIGHT_ONLY /
    BALANCED_ONLY) instead of a quality preset.  Returns as pack()."""
    torch = _torch()
    xy = _dev_i32(xy, device)
    offsets = _dev_i32(offsets, device)
    ch, n = _charts(xy, offsets)
    out_xy = torch.empty((max(n, 0), 2), dtype=torch.int32, device=xy.device)
    out_or = torch.empty(max(n, 0), dtype=torch.uint8, device=xy.device)
    out_sc = torch.empty(1, dtype=torch.float32, device=xy.device)
    m = Method(int(slices), int(topt_percent), int(variant))
    _check(lib().tabi_pack_method(ctypes.byref(ch), n, int(atlas_w), int(atlas_h), int(padding),
                                  ctypes.byref(m), _ptr(out_xy), _ptr(out_or), _ptr(out_sc),
                                  _stream(stream)))
    return out_xy, out_or, out_sc


def pack_noalloc_into(xy, offsets, n, atlas_w, atlas_h, padding, quality, out_xy, out_orient,
                      out_scale, stream=None):
    """tabi_pack_noalloc on caller tensors (device int32 xy / offsets, outputs
    int32[n,2], uint8[n], float32[1]): the library allocates nothing."""
    ch = Charts(_ptr(xy).value, _ptr(offsets).value, int(xy.numel() // 2))
    _check(lib().tabi_pack_noalloc(ctypes.byref(ch), int(n), int(atlas_w), int(atlas_h),
                                   int(padding), int(quality), _ptr(out_xy), _ptr(out_orient),
                                   _ptr(out_scale), _stream(stream)))


def pack_into(xy, offsets, n, atlas_w, atlas_h, padding, quality, out_xy, out_orient, out_scale,
              stream=None):
    """tabi_pack on caller-provided device tensors (no allocation here)."""
    ch = Charts(_ptr(xy).value, _ptr(offsets).value, int(xy.numel() // 2))
    _check(lib().tabi_pack(ctypes.byref(ch), int(n), int(atlas_w), int(atlas_h), int(padding),
                           int(quality), _ptr(out_xy), _ptr(out_orient), _ptr(out_scale),
                           _stream(stream)))


class Batch:
    """A flattened batch of atlases resident on the device (inputs of
    tabi_pack_many), with the host-side shape the library sizes itself by."""

    def __init__(self, inputs, device="cuda"):
        import numpy as np
        torch = _torch()
        xs, offs, aoff, wh = [], [0], [0], []
        for inp in inputs:
            xs.append(np.asarray(inp.xy, np.int32))
            o = np.asarray(inp.offsets, np.int64)
            offs.extend((o[1:] + offs[-1]).tolist())
            aoff.append(aoff[-1] + inp.n)
            wh.extend([inp.atlas_w, inp.atlas_h])
        self.count = len(inputs)
        self.total = aoff[-1]
        self.max_charts = max([inp.n for inp in inputs], default=0)
        self.max_side = max([max(inp.atlas_w, inp.atlas_h) for inp in inputs], default=1)
        pads = {inp.padding for inp in inputs}
        quals = {inp.quality for inp in inputs}
        if len(pads) > 1 or len(quals) > 1:
            raise ValueError("one padding and one quality per batch")
        self.padding = pads.pop() if pads else 0
        self.quality = quals.pop() if quals else 2
        self.xy = _dev_i32(np.concatenate(xs) if xs else np.zeros(0, np.int32), device)
        self.voff = _dev_i32(np.asarray(offs, np.int64), device)
        self.aoff = _dev_i32(np.asarray(aoff, np.int64), device)
        self.wh = _dev_i32(np.asarray(wh, np.int64), device)
        self.out_xy = torch.empty((self.total, 2), dtype=torch.int32, device=self.xy.device)
        self.out_orient = torch.empty(self.total, dtype=torch.uint8, device=self.xy.device)
        self.out_scale = torch.empty(self.count, dtype=torch.float32, device=self.xy.device)
        self.workspace = None

    def tune(self, stream=None, reps=2):
        """tabi_tune_many on this batch: times every candidate batched shape
        and keeps the fastest for this quality on the device.  Returns
        {"shape": (first-round slots, rounds at that size, largest slots,
        threads, LDS cap), "ms": [per shape]}."""
        n = int(lib().tabi_many_shape_count())
        shape = (ctypes.c_int32 * 5)()
        ms = (ctypes.c_float * n)()
        _check(lib().tabi_tune_many(_ptr(self.xy), _ptr(self.voff), _ptr(self.aoff), self.count,
                                    _ptr(self.wh), self.total, self.max_charts, self.max_side,
                                    self.padding, self.quality, _ptr(self.out_xy),
                                    _ptr(self.out_orient), _ptr(self.out_scale), int(reps), shape,
                                    ms, _stream(stream)))
        return {"shape": tuple(int(v) for v in shape), "ms": [round(float(v), 4) for v in ms]}

    def workspace_bytes(self):
        return int(lib().tabi_pack_many_workspace_bytes(self.count, self.total, self.max_charts,
                                                        self.max_side, self.padding, self.quality))

    def run(self, stream=None, use_workspace=False):
        """Enqueue tabi_pack_many (or tabi_pack_many_ws on a kept work space)."""
        args = (_ptr(self.xy), _ptr(self.voff), _ptr(self.aoff), self.count, _ptr(self.wh),
                self.total, self.max_charts, self.max_side, self.padding, self.quality,
                _ptr(self.out_xy), _ptr(self.out_orient), _ptr(self.out_scale))
        if use_workspace:
            torch = _torch()
            nb = self.workspace_bytes()
            if self.workspace is None or self.workspace.numel() < nb:
                self.workspace = torch.empty(nb, dtype=torch.uint8, device=self.xy.device)
            _check(lib().tabi_pack_many_ws(*args, _ptr(self.workspace), ctypes.c_int64(nb),
                                           _stream(stream)))
        else:
            _check(lib().tabi_pack_many(*args, _stream(stream)))
        return self.out_xy, self.out_orient, self.out_scale

    def run_method(self, slices, topt_percent, variant, stream=None):
        """Enqueue tabi_pack_many_method: the batch with the method's knobs."""
        m = Method(int(slices), int(topt_percent), int(variant))
        _check(lib().tabi_pack_many_method(_ptr(self.xy), _ptr(self.voff), _ptr(self.aoff),
                                           self.count, _ptr(self.wh), self.total,
                                           self.max_charts, self.max_side, self.padding,
                                           ctypes.byref(m), _ptr(self.out_xy),
                                           _ptr(self.out_orient), _ptr(self.out_scale),
                                           _stream(stream)))
        return self.out_xy, self.out_orient, self.out_scale


def many_shape(quality, count=256):
    """Current batched shape (first-round slots, rounds at that size, largest
    slots per round, threads, LDS cap) on this device for a batch of `count`
    atlases."""
    shape = (ctypes.c_int32 * 5)()
    _check(lib().tabi_many_shape(int(quality), int(count), shape))
    return tuple(int(v) for v in shape)


def debug_set_many_shape(quality, index):
    """Force candidate batched shape `index` (-1: default); results are unchanged."""
    _check(lib().tabi_debug_set_many_shape(int(quality), int(index)))


def pack_many(inputs, stream=None, device="cuda", use_workspace=False):
    """tabi_pack_many over a list of AtlasInput-like objects.  Returns
    (out_xy int32[N,2], out_orient uint8[N], out_scale float32[count]) with
    charts in the order of the inputs."""
    return Batch(inputs, device).run(stream, use_workspace)


def debug_order(xy, offsets, atlas_w, atlas_h, padding, quality, stream=None, device="cuda"):
    torch = _torch()
    xy = _dev_i32(xy, device)
    offsets = _dev_i32(offsets, device)
    ch, n = _charts(xy, offsets)
    perm = torch.empty(n, dtype=torch.int32, device=xy.device)
    khi = torch.empty(1, dtype=torch.int32, device=xy.device)
    _check(lib().tabi_debug_order(ctypes.byref(ch), n, int(atlas_w), int(atlas_h), int(padding),
                                  int(quality), _ptr(perm), _ptr(khi), _stream(stream)))
    return perm, khi


def debug_pairs(xy, offsets, padding, quality, k, stream=None, device="cuda"):
    torch = _torch()
    xy = _dev_i32(xy, device)
    offsets = _dev_i32(offsets, device)
    ch, n = _charts(xy, offsets)
    cd = torch.empty(n, dtype=torch.int32, device=xy.device)
    fl = torch.empty(n, dtype=torch.uint8, device=xy.device)
    _check(lib().tabi_debug_pairs(ctypes.byref(ch), n, int(padding), int(quality), int(k),
                                  _ptr(cd), _ptr(fl), _stream(stream)))
    return cd, fl


def debug_feasible(xy, offsets, atlas_w, atlas_h, padding, quality, k, stream=None,
                   device="cuda"):
    torch = _torch()
    xy = _dev_i32(xy, device)
    offsets = _dev_i32(offsets, device)
    ch, n = _charts(xy, offsets)
    out_xy = torch.empty((n, 2), dtype=torch.int32, device=xy.device)
    out_or = torch.empty(n, dtype=torch.uint8, device=xy.device)
    feas = torch.empty(1, dtype=torch.int32, device=xy.device)
    rows = torch.empty(1, dtype=torch.int32, device=xy.device)
    _check(lib().tabi_debug_feasible(ctypes.byref(ch), n, int(atlas_w), int(atlas_h),
                                     int(padding), int(quality), int(k), _ptr(out_xy),
                                     _ptr(out_or), _ptr(feas), _ptr(rows), _stream(stream)))
    return out_xy, out_or, feas, rows


def debug_phase_clock(slots=64):
    """tabi_debug_phase_clock: per-slot phase clock sums of the last single
    pack (the diagnostic library only).  Returns an int64 array [slots, 11]."""
    import numpy as np
    out = np.zeros((slots, 11), np.int64)
    L = lib()
    L.tabi_debug_phase_clock.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    n = L.tabi_debug_phase_clock(out.ctypes.data_as(ctypes.c_void_p), int(slots))
    if n < 0:
        _check(n)
    return out[:n]


def timing_enable(on=True):
    lib().tabi_timing_enable(1 if on else 0)


def timing_stages(stages=None):
    """Bracket only these stages (names of STAGES; None: all) while timing is on."""
    names = STAGES if stages is None else stages
    _check(lib().tabi_timing_stages(sum(1 << STAGES.index(s) for s in names)))


def timing_reset():
    lib().tabi_timing_reset()


def timing_read():
    """{stage: (total_ms, launches)} since the last reset (waits for events)."""
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_int32 * len(STAGES))()
    _check(lib().tabi_timing_read(ms, n, len(STAGES)))
    return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(STAGES)}


# ---- resident per-chart proxy records (incremental re-packs) -----------------
def record_bytes():
    return int(lib().tabi_record_bytes())


def prep_records(xy, vert_offsets, atlas_offsets, quality, stream=None, device="cuda"):
    """Proxy records (uint8 tensor [N, record_bytes]) of every chart of the
    atlases delimited by atlas_offsets."""
    torch = _torch()
    xy = _dev_i32(xy, device)
    vert_offsets = _dev_i32(vert_offsets, device)
    atlas_offsets = _dev_i32(atlas_offsets, device)
    N = int(vert_offsets.numel()) - 1
    count = int(atlas_offsets.numel()) - 1
    rec = torch.empty((max(N, 0), record_bytes()), dtype=torch.uint8, device=xy.device)
    _check(lib().tabi_prep_records(_ptr(xy), _ptr(vert_offsets), _ptr(atlas_offsets), count, N,
                                   int(quality), _ptr(rec), _stream(stream)))
    return rec


def splice_records(records, index, new_records, stream=None):
    """records[index[i]] = new_records[i] on the device (keeps input indices)."""
    idx = _dev_i32(index, records.device)
    m = int(idx.numel())
    if m != int(new_records.shape[0]):
        raise ValueError("index and new_records differ in length")
    _check(lib().tabi_splice_records(_ptr(records), _ptr(idx), m, _ptr(new_records),
                                     _stream(stream)))


def pack_many_records(records, atlas_offsets, atlas_wh, max_charts, max_side, padding, quality,
                      out_xy, out_orient, out_scale, stream=None):
    """tabi_pack_many_records into caller-provided device tensors."""
    count = int(atlas_offsets.numel()) - 1
    N = int(records.shape[0])
    _check(lib().tabi_pack_many_records(_ptr(records), _ptr(atlas_offsets), count, _ptr(atlas_wh),
                                        N, int(max_charts), int(max_side), int(padding),
                                        int(quality), _ptr(out_xy), _ptr(out_orient),
                                        _ptr(out_scale), _stream(stream)))


def shutdown():
    """tabi_shutdown: return the library's pooled work space to the device
    (waits for the device); later calls still work."""
    _check(lib().tabi_shutdown())


def debug_set_stage_cap(entries):
    """Cap the pack kernel's per-row staging (-1 = default); results are unchanged."""
    _check(lib().tabi_debug_set_stage_cap(int(entries)))


def debug_set_pack_lds(nbytes):
    """Cap the pack kernel's row shared memory (-1 = default); results are unchanged."""
    _check(lib().tabi_debug_set_pack_lds(int(nbytes)))


def debug_set_profile_cap(words):
    """Size of the stored-profile arena in words (-1 = default, 0 = none);
    results are unchanged."""
    _check(lib().tabi_debug_set_profile_cap(int(words)))


CTX_STATS = ["launches", "finished", "failed", "evicted", "resident", "device_bytes_used",
             "device_bytes_peak", "queued", "in_flight", "cross_slot_waits", "peak_in_flight"]


def _hptr(a):
    """Host address of a C-contiguous numpy array."""
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


class ServeContext:
    """tabi_ctx: continuous batching of pack requests with resident proxies.
    Chart data are host numpy arrays (copied at submission); each request's
    outputs are host numpy arrays filled when tabi_poll reports it done."""

    def __init__(self, quality=2, padding=2, streams=4, max_batch=256, device_bytes=16 << 30,
                 staging_bytes=64 << 20):
        cfg = CtxConfig(int(quality), int(padding), int(streams), int(max_batch),
                        int(device_bytes), int(staging_bytes))
        h = ctypes.c_void_p()
        _check(lib().tabi_ctx_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self.outputs = {}  # ticket -> (xy, orient, scale): kept alive until reported

    def _outs(self, n):
        import numpy as np
        return (np.empty((n, 2), np.int32), np.empty(n, np.uint8), np.empty(1, np.float32))

    def submit(self, xy, offsets, atlas_w, atlas_h, padding=None, quality=None):
        """New atlas; returns (atlas_id, ticket).  padding / quality: the
        request's own (tabi_submit_with), else the context's."""
        import numpy as np
        xy = np.ascontiguousarray(xy, np.int32)
        off = np.ascontiguousarray(offsets, np.int32)
        n = off.size - 1
        o = self._outs(n)
        aid, t = ctypes.c_int32(), ctypes.c_int64()
        if padding is None and quality is None:
            _check(lib().tabi_submit(self.h, _hptr(xy), _hptr(off), n, int(atlas_w),
                                     int(atlas_h), _hptr(o[0]), _hptr(o[1]), _hptr(o[2]),
                                     ctypes.byref(aid), ctypes.byref(t)))
        else:
            _check(lib().tabi_submit_with(self.h, _hptr(xy), _hptr(off), n, int(atlas_w),
                                          int(atlas_h), int(padding), int(quality),
                                          _hptr(o[0]), _hptr(o[1]), _hptr(o[2]),
                                          ctypes.byref(aid), ctypes.byref(t)))
        self.outputs[t.value] = o
        return aid.value, t.value

    def repack(self, atlas_id, replaced, xy, offsets, n):
        """Re-pack of resident atlas `atlas_id` (n charts) with charts
        `replaced` (increasing indices) replaced by the CSR (xy, offsets)."""
        import numpy as np
        idx = np.ascontiguousarray(replaced, np.int32)
        xy = np.ascontiguousarray(xy, np.int32)
        off = np.ascontiguousarray(offsets, np.int32)
        o = self._outs(n)
        t = ctypes.c_int64()
        _check(lib().tabi_repack(self.h, int(atlas_id), _hptr(idx), int(idx.size), _hptr(xy),
                                 _hptr(off), _hptr(o[0]), _hptr(o[1]), _hptr(o[2]),
                                 ctypes.byref(t)))
        self.outputs[t.value] = o
        return t.value

    def poll(self, wait=False, max_done=4096):
        """Finished requests: list of (ticket, atlas_id, status, batch,
        latency_ms, (xy, orient, scale) or None)."""
        buf = (Done * max_done)()
        k = ctypes.c_int32()
        _check(lib().tabi_poll(self.h, 1 if wait else 0, buf, max_done, ctypes.byref(k)))
        out = []
        for d in buf[:k.value]:
            o = self.outputs.pop(d.ticket)
            out.append((d.ticket, d.atlas_id, d.status, d.batch, d.latency_ms,
                        o if d.status == TABI_OK else None))
        return out

    def stats(self):
        v = (ctypes.c_int64 * len(CTX_STATS))()
        _check(lib().tabi_ctx_stats(self.h, v, len(CTX_STATS)))
        return dict(zip(CTX_STATS, list(v)))

    def close(self):
        if self.h:
            h, self.h = self.h, None
            _check(lib().tabi_ctx_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
