"""Pins of the oracle's hybrid tail (Sec. 4.4 "Performance Optimization"):
after the t_opt switch the remaining charts are folded all at once by prefix
sums of their offsets (grown width less the compacting distance to the next
chart) modulo the atlas width, downscaled until every row fits, placed in the
one left-to-right : two right-to-left alternation and pushed up; the
candidate scale is the one with the largest area-weighted final scale.

What fixes it independently of the code under test:
  * with t_opt = 0 there is no tail and the result is the plain pack;
  * identical rectangles folded entirely by prefix sums have a closed form
    (rows from integer division, the tail scale from the row counts, flat
    rows pushed on a brute-force frontline of texel columns);
  * the tail's rows, its scale and its offsets follow from the compacting
    distances of the pinned pair diagnostic at the head scale and below;
  * the chosen scale maximises sum(area * k) over the feasible candidates
    (areas by the shoelace formula here), ties to the larger k;
  * every layout is valid by the independent rasteriser, each chart at its
    own scale.
"""
from __future__ import annotations

import numpy as np
import pytest

from cases import small_input
from paper_2602_07782_amd import synth

T = 16384


def _area2(P):
    P = np.asarray(P, np.int64)
    x, y = P[:, 0], P[:, 1]
    return abs(int(np.dot(x, np.roll(y, -1)) - np.dot(np.roll(x, -1), y)))


def _dims(P):
    e = np.ptp(np.asarray(P, np.int64), axis=0)
    return int(min(e)), int(max(e))  # W <= H after the quarter turn


@pytest.mark.parametrize("seed", range(10))
def test_no_tail_is_the_plain_pack(orc, seed):
    inp = small_input(9500 + seed, n=30)
    xy, ori, ks, k = orc.pack_hybrid(inp, 10, 0)
    pxy, pori, psc, pk = orc.pack_method(inp, 10, 0, orc.FULL)
    assert k == pk and np.array_equal(xy, pxy) and np.array_equal(ori, pori)
    assert np.all(ks == (k if k > 0 else 0))


def _rect_hybrid_closed_form(n, a, b, Wa, Ha, p):
    """All charts tail (t_opt = 100): returns (k, kt, positions, mirror bits)."""
    Wd, Hd = Wa + p, Ha + p
    best = None
    for k in range(64, 0, -1):
        wd = -(-k * a // T) + p
        rows = [j * wd // Wd for j in range(n)]
        counts = np.bincount(rows)
        kt = 0
        for kk in range(k, 0, -1):
            if all(c * (-(-kk * a // T) + p) <= Wd for c in counts if c):
                kt = kk
                break
        if kt == 0:
            continue
        w, h = -(-kt * a // T) + p, -(-kt * b // T) + p
        F = np.zeros(Wd, np.int64)
        xs, ys, mir, r_ord = [0] * n, [0] * n, [0] * n, -1
        prev = None
        t = 0
        for j in range(n):
            if rows[j] != prev:
                prev, t = rows[j], 0
                r_ord += 1
            lr = r_ord % 3 == 0
            x = t * w if lr else Wd - t * w - w
            xs[j], mir[j] = x, 0 if lr else 1
            t += 1
        # flat rows pushed row by row on a frontline of texel columns
        for r in sorted(set(rows)):
            js = [j for j in range(n) if rows[j] == r]
            for j in js:
                ys[j] = int(F[xs[j]:xs[j] + w].max())
            for j in js:
                F[xs[j]:xs[j] + w] = np.maximum(F[xs[j]:xs[j] + w], ys[j] + h)
        if F.max() > Hd:
            continue
        if best is None or kt > best[1]:
            best = (k, kt, xs, ys, mir)
    return best


@pytest.mark.parametrize("a,b,n,Wa,Ha,p", [
    (256 * 3, 256 * 5, 37, 40, 60, 1), (1000, 1900, 50, 64, 90, 2), (700, 3000, 25, 50, 200, 3),
    (256 * 2, 256 * 7, 120, 64, 300, 0), (900, 1300, 80, 100, 100, 2)])
def test_identical_rectangles_all_tail_closed_form(orc, chk, a, b, n, Wa, Ha, p):
    inp = synth.rect_input(n, a, b, Wa, Ha, p, q=2, seed=n)
    want = _rect_hybrid_closed_form(n, a, b, Wa, Ha, p)
    xy, ori, ks, k = orc.pack_hybrid(inp, 10, 100)
    assert want is not None and k == want[0]
    assert np.all(ks == want[1])
    perm, _ = orc.order(inp)
    assert np.array_equal(perm, np.arange(n))
    for j in range(n):
        assert tuple(xy[j]) == (want[2][j], want[3][j]), j
        assert bool(ori[j] & 8) == bool(want[4][j]), j
    st = chk.check_layout_ks(inp, xy, ori, ks)
    assert st["overlap"] == 0 and st["outside"] == 0


def _tail_structure(orc, inp, k, t0, K=10):
    """Rows, tail scale and in-row offsets of the tail from the pair
    diagnostic: returns (rows, kt, X) over the tail charts t0.. in sorted
    order."""
    perm, _ = orc.order(inp)
    n, Wd, p = inp.n, inp.atlas_w + inp.padding, inp.padding
    dims = [_dims(inp.chart(int(c))) for c in perm]
    cd_k, _ = orc.pairs(inp, k)
    P, rows = 0, []
    for j in range(t0, n):
        rows.append(P // Wd)
        P += (-(-k * dims[j][0] // T) + p) - (cd_k[j + 1] if j + 1 < n else 0)
    for kt in range(k, 0, -1):
        cd, _ = orc.pairs(inp, kt)
        X, x, ok = [], 0, True
        for i, j in enumerate(range(t0, n)):
            wd = -(-kt * dims[j][0] // T) + p
            if i > 0:
                x = 0 if rows[i] != rows[i - 1] else x + (-(-kt * dims[j - 1][0] // T) + p) - cd[j]
            X.append(x)
            ok &= x + wd <= Wd
        if ok:
            return rows, kt, X
    return rows, 0, None


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("topt", [5, 20])
def test_tail_rows_scale_and_offsets(orc, seed, topt):
    inp = small_input(9600 + seed, n=60, W=128, q=2)
    perm, _ = orc.order(inp)
    dims = [_dims(inp.chart(int(c))) for c in perm]
    seen = 0
    for k in range(64, 0, -4):
        ok, xs, ys, mir, t0, kt = orc.feasible_hybrid(inp, k, 10, topt)
        if t0 >= inp.n:
            continue
        # the switch: the tail's first chart is shorter than t_opt of the height
        assert 100 * -(-k * dims[t0][1] // T) < topt * inp.atlas_h
        rows, kt_want, X = _tail_structure(orc, inp, k, t0)
        assert kt == kt_want or (not ok and kt_want == 0), (k, kt, kt_want)
        if not ok or kt_want == 0:
            continue
        seen += 1
        Wd, p = inp.atlas_w + inp.padding, inp.padding
        order, r_prev = -1, None
        for i, j in enumerate(range(t0, inp.n)):
            if rows[i] != r_prev:
                r_prev, order = rows[i], order + 1
            wd = -(-kt * dims[j][0] // T) + p
            lr = order % 3 == 0
            assert xs[j] == (X[i] if lr else Wd - X[i] - wd), (k, j)
            assert mir[j] == (0 if lr else 1)
    if seen == 0:
        pytest.skip("no candidate scale with a feasible tail for this input")


@pytest.mark.parametrize("seed", [0, 1, 8, 9])
@pytest.mark.parametrize("topt", [10, 30, 100])
def test_choice_maximises_area_weighted_scale(orc, chk, seed, topt):
    """Seeds 0 (t_opt 30, 100), 8 (100) and 9 (30) are inputs where a head
    scale below the largest feasible one wins on the area-weighted scale."""
    inp = small_input(9650 + seed, n=50, W=128, q=2)
    perm, _ = orc.order(inp)
    areas = [_area2(inp.chart(int(c))) for c in perm]
    best = None
    for k in range(64, 0, -1):
        ok, xs, ys, mir, t0, kt = orc.feasible_hybrid(inp, k, 10, topt)
        if not ok:
            continue
        obj = k * sum(areas[:t0]) + kt * sum(areas[t0:])
        if best is None or obj > best[0]:
            best = (obj, k, t0, kt)
    xy, ori, ks, k = orc.pack_hybrid(inp, 10, topt)
    assert best is not None and k == best[1]
    rank = np.empty(inp.n, int)
    rank[perm] = np.arange(inp.n)
    for c in range(inp.n):
        assert ks[c] == (k if rank[c] < best[2] else best[3]), c
    st = chk.check_layout_ks(inp, xy, ori, ks)
    assert st["overlap"] == 0 and st["outside"] == 0


@pytest.mark.parametrize("topt", [1, 2, 5])
def test_mixed2k_hybrid_layout_is_valid(orc, chk, topt):
    inp = synth.make_input("mixed2k", 0)
    xy, ori, ks, k = orc.pack_hybrid(inp, 10, topt)
    assert k > 0 and ks.min() >= 1 and ks.max() == k
    st = chk.check_layout_ks(inp, xy, ori, ks)
    assert st["overlap"] == 0 and st["outside"] == 0


def test_degenerate_and_empty(orc):
    empty = synth.AtlasInput(np.zeros(0, np.int32), np.zeros(1, np.int32), 64, 64, 1, 2)
    assert orc.pack_hybrid(empty, 10, 5)[3] == 64
    two = synth.AtlasInput(np.array([0, 0, 100, 100], np.int32), np.array([0, 2], np.int32),
                           64, 64, 1, 2)
    xy, ori, ks, k = orc.pack_hybrid(two, 10, 5)
    assert k == -1 and np.all(xy == -1) and np.all(ks == 0)
    big = synth.rect_input(1, 100 * 256, 100 * 256, 1, 1, 0)
    xy, ori, ks, k = orc.pack_hybrid(big, 10, 5)
    assert k == 0 and np.all(xy == -1)
