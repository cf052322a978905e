"""GPU parity of the pre-rotation of UV charts to their tight boxes (Sec. 5,
experimental setup): tabi_pack_prerotate against the oracle, bit for bit
(turned vertices, directions, positions, orientation bits, scale)."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

from cases import small_input
from paper_2602_07782_amd import synth

pytestmark = pytest.mark.gpu
Q = 256


@pytest.fixture(scope="module")
def tabi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_07782_amd as t
    t.lib()
    return t


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _turned(orc, inp):
    polys, dirs = [], []
    for c in range(inp.n):
        r, m = orc.prerotate(inp.chart(c))
        polys.append(r)
        dirs.append(m)
    rxy = np.concatenate([p.reshape(-1) for p in polys]) if polys else np.zeros(0, np.int32)
    return rxy.astype(np.int32), np.array(dirs, np.uint8)


def _check(tabi, orc, inp, label, in_place=False):
    _say("prerotate parity:", label, "n =", inp.n, "V =", len(inp.xy) // 2)
    import torch
    src = torch.from_numpy(np.ascontiguousarray(inp.xy, np.int32)).to("cuda:0")
    rxy, dirs, xy, ori, sc = tabi.pack_prerotate(src, inp.offsets, inp.atlas_w, inp.atlas_h,
                                                 inp.padding, inp.quality, device="cuda:0",
                                                 in_place=in_place)
    erxy, edirs = _turned(orc, inp)
    assert np.array_equal(rxy.cpu().numpy(), erxy), (label, np.argwhere(rxy.cpu().numpy() != erxy)[:4])
    assert np.array_equal(dirs.cpu().numpy(), edirs), label
    oxy, oor, osc, ok, odirs = orc.pack_prerotate(inp)
    assert np.array_equal(odirs, edirs)
    assert float(sc.cpu().numpy()[0]) == osc, label
    assert np.array_equal(xy.cpu().numpy(), oxy), label
    assert np.array_equal(ori.cpu().numpy(), oor), label
    if in_place:
        assert np.array_equal(src.cpu().numpy(), erxy)
    return ok


@pytest.mark.parametrize("seed", range(12))
def test_prerotate_parity_small(tabi, orc, seed):
    _check(tabi, orc, small_input(9700 + seed), f"small {seed}")


def test_prerotate_in_place(tabi, orc):
    _check(tabi, orc, small_input(9750, n=20), "in place", in_place=True)


@pytest.mark.parametrize("name,inst", [("stars64", 1), ("mixed2k", 0), ("mixed2k", 3)])
def test_prerotate_parity_configs(tabi, orc, name, inst):
    _check(tabi, orc, synth.make_input(name, inst), f"{name}/{inst}")


def test_prerotate_turned_rectangles_and_long_charts(tabi, orc):
    """Rectangles turned by searched angles come back to them; charts of
    several hundred vertices span several 64-vertex chunks with a ragged tail."""
    polys, want = [], []
    for i, m0 in enumerate([0, 1, 7, 8, 23, 40, 63, 32]):
        th = m0 * math.pi / 128
        w, h = (30 + 3 * i) * Q, (10 + i) * Q
        P = np.array([(0, 0), (w, 0), (w, h), (0, h)], float)
        R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        polys.append(np.rint(P @ R.T + np.array([5000 + 9000 * i, 3000])).astype(np.int64))
        want.append(m0)
    rng = np.random.default_rng(9760)
    for nv in (64, 65, 127, 300, 1000):
        ang = np.sort(rng.uniform(0, 2 * np.pi, nv))
        rad = rng.uniform(0.6, 1.0, nv) * 20 * Q
        polys.append(np.stack([4000 + rad * np.cos(ang) * 1.8, 6000 + rad * np.sin(ang)],
                              1).astype(np.int64))
        want.append(None)
    xy, off = synth.pack_csr(polys)
    inp = synth.AtlasInput(xy, off, 256, 256, 2, 2)
    _check(tabi, orc, inp, "rectangles + long charts")
    _, dirs = _turned(orc, inp)
    for c, m0 in enumerate(want):
        if m0 is not None:
            assert dirs[c] == m0, c


def test_prerotate_degenerate_and_empty(tabi, orc):
    """Charts the pack rejects are copied unchanged (direction 0) and the
    pack reports them (-1); no charts at all gives scale 1."""
    big = 1 << 22
    polys = [np.array([(0, 0), (3000, 0), (3000, 2000), (0, 2000)], np.int64),
             np.array([(0, 0), (big, 0), (big, 300), (0, 300)], np.int64)]
    xy, off = synth.pack_csr(polys)
    inp = synth.AtlasInput(xy, off, 64, 64, 1, 2)
    rxy, dirs, oxy, ori, sc = tabi.pack_prerotate(inp.xy, inp.offsets, 64, 64, 1, 2,
                                                  device="cuda:0")
    assert np.array_equal(rxy.cpu().numpy()[8:], np.asarray(inp.xy)[8:])
    assert list(dirs.cpu().numpy()) == [0, 0]
    assert float(sc.cpu().numpy()[0]) == -1.0 == orc.pack_prerotate(inp)[2]
    empty = tabi.pack_prerotate(np.zeros(0, np.int32), np.zeros(1, np.int32), 64, 64, 1, 2,
                                device="cuda:0")
    assert float(empty[4].cpu().numpy()[0]) == 1.0


def test_prerotate_tss_recipe_parity(tabi, orc):
    """The paper leaves TSS charts unturned, but the entry point must still
    agree with the oracle on them (axis-aligned clipped patches)."""
    _check(tabi, orc, synth.make_tss(0, n=600, atlas=1024), "tss 600")
