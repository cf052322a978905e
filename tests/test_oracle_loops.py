"""Charts of several boundary loops (mesh charts with holes, charts of
several islands) in the oracle: holes change neither a chart's proxies nor
the packing, only the area that bounds the scale (outer less holes,
exactly); islands are all bounded, which the raster check of every loop
under its chart's transform confirms (no overlap, nothing outside)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2602_07782_amd import synth


def _shoelace2(P):
    P = np.asarray(P, np.int64)
    x, y = P[:, 0], P[:, 1]
    return abs(int(np.dot(x, np.roll(y, -1)) - np.dot(np.roll(x, -1), y)))


def _outer_input(L, outers):
    xy, off = synth.pack_csr(outers)
    return synth.AtlasInput(xy, off, L.atlas_w, L.atlas_h, L.padding, L.quality)


@pytest.mark.parametrize("seed", range(6))
def test_holes_change_nothing_but_the_area(orc, seed):
    L, outers = synth.make_loops(60, 256, 256, 2, 2, 600 + seed, hole_frac=1.0, island_frac=0.0)
    assert any(L.chart_loops[c + 1] - L.chart_loops[c] > 1 for c in range(L.n))
    got = orc.pack_loops(L)
    want = orc.pack(_outer_input(L, outers))
    assert got[3] == want[3]
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    for c in range(0, L.n, 7):
        loops = L.loops(c)
        a = orc.prep_chart_loops(loops, 10)
        b = orc.prep_chart(loops[0], 10)
        assert a.area2 == _shoelace2(loops[0]) - sum(_shoelace2(h) for h in loops[1:])
        for f in ("W", "H", "rot", "flipx", "flipy", "obb_m", "a", "b", "e", "f"):
            assert getattr(a, f) == getattr(b, f), f
        assert list(a.ylo) == list(b.ylo) and list(a.xhi) == list(b.xhi)


def _check_islands(chk, L, xy, ori, k):
    """Every loop rasterised under its chart's output transform (the box
    of all its loops); footprints grown by the gutter must not overlap and
    charts must stay inside the atlas."""
    T = 16384
    Wd, Hd, p = L.atlas_w + L.padding, L.atlas_h + L.padding, L.padding
    grid = np.zeros((Hd + 2, Wd + 2), np.int32)
    outside = 0
    for c in range(L.n):
        loops = [np.asarray(x, np.int64) for x in L.loops(c)]
        allp = np.concatenate(loops)
        x0, y0 = allp.min(0)
        w0, h0 = (allp.max(0) - allp.min(0)).tolist()
        o = int(ori[c])
        W, H = (h0, w0) if o & 1 else (w0, h0)
        wt = -(-k * W // T)
        mask = np.zeros((-(-k * H // T) + 1, wt + 1), np.uint8)
        for P in loops:
            u, v = P[:, 0] - x0, P[:, 1] - y0
            if o & 1:
                u, v = h0 - v, u
            if o & 2:
                u = W - u
            if o & 4:
                v = H - v
            U, V = k * u, k * v
            if o & 8:
                U = T * wt - U
            m, _ = chk.raster(U, V, 0, 0, mask.shape[1], mask.shape[0])
            mask |= m
        jj, ii = np.nonzero(mask)
        X, Y = int(xy[c][0]) + ii, int(xy[c][1]) + jj
        outside += int(np.sum((X < 0) | (X >= L.atlas_w) | (Y < 0) | (Y >= L.atlas_h)))
        fp = np.zeros_like(grid)
        for dy in range(p + 1):
            for dx in range(p + 1):
                ok = (Y + dy < grid.shape[0]) & (X + dx < grid.shape[1]) & (X >= 0) & (Y >= 0)
                fp[Y[ok] + dy, X[ok] + dx] = 1
        grid += fp
    return int(np.sum(grid > 1)), outside


@pytest.mark.parametrize("seed", range(4))
def test_island_charts_give_valid_layouts(orc, chk, seed):
    L, _ = synth.make_loops(50, 256, 256, 2, 2, 700 + seed, hole_frac=0.0, island_frac=1.0)
    assert sum(L.chart_loops[c + 1] - L.chart_loops[c] > 1 for c in range(L.n)) > 20
    xy, ori, sc, k = orc.pack_loops(L)
    assert k > 0
    overlap, outside = _check_islands(chk, L, xy, ori, k)
    assert overlap == 0 and outside == 0


def test_a_loop_of_two_vertices_makes_the_chart_degenerate(orc):
    good = np.array([[0, 0], [2560, 0], [2560, 2560], [0, 2560]], np.int64)
    L = synth.loops_csr([[good], [good + 5000, np.array([[1, 1], [5, 5]], np.int64)]],
                        64, 64, 1, 2)
    xy, ori, sc, k = orc.pack_loops(L)
    assert sc == -1.0 and np.all(xy == -1)


def test_slices_between_islands_take_the_slice_box(orc):
    """Two 10x10-texel islands 80 texels apart: the x-slices that meet
    neither (the gap) are read as the whole slice box, [0, H] in v; the
    slices over the islands are the islands' own ranges."""
    a = np.array([[0, 0], [2560, 0], [2560, 2560], [0, 2560]], np.int64)
    b = a + [25600, 12800]  # 100 texels right, 50 texels down
    rec = orc.prep_chart_loops([a, b], 10)
    H = int(rec.H)
    W = int(rec.W)
    assert rec.rot == 1  # 110 x 60 texels: turned to stand upright
    # after the turn the islands are stacked in v; the y-slices (rows) in the
    # gap take the whole slice box in u
    inner = [j for j in range(10) if j * H // 10 >= 12 * 256 and (j + 1) * H // 10 <= 98 * 256]
    assert inner, inner
    for j in inner:
        assert (rec.xlo[j], rec.xhi[j]) == (0, W), j
    xy, ori, sc, k = orc.pack_loops(synth.loops_csr([[a, b]], 128, 128, 1, 2))
    assert k > 0
