"""Pins of the method's knobs and ablation variants in the oracle (Sec. 5
"Ablations", Tab. ablationBalancedTight; App. D local-AABB count and t_opt
tables): the presets are their knob settings, balanced-only packs the
charts' boxes, tight-only has a closed form on identical rectangles, a t_opt
of 100 % folds every row like tight-only, and every variant's layout is
valid by the independent rasteriser."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from cases import small_input
from paper_2602_07782_amd import synth

T = 16384


def _same(a, b):
    assert a[2] == b[2] and a[3] == b[3], (a[2:], b[2:])
    assert np.array_equal(a[0], b[0]), np.argwhere(a[0] != b[0])[:5]
    assert np.array_equal(a[1], b[1]), np.argwhere(a[1] != b[1])[:5]


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("q", [0, 1, 2])
def test_presets_are_their_knobs(orc, seed, q):
    inp = small_input(8100 + seed, q=q)
    K, topt = orc.quality(q, inp.n)
    _same(orc.pack(inp), orc.pack_method(inp, K, topt, orc.FULL))
    if q == 2:  # the paper's t_opt setting spelled as -1
        _same(orc.pack(inp), orc.pack_method(inp, 10, -1, orc.FULL))


def _boxes(inp):
    """Each chart replaced by its axis-aligned bounding box (same Q8 extents)."""
    polys = []
    for c in range(inp.n):
        P = inp.chart(c).astype(np.int64)
        (x0, y0), (x1, y1) = P.min(0), P.max(0)
        polys.append(np.array([(x0, y0), (x1, y0), (x1, y1), (x0, y1)], np.int64))
    xy, off = synth.pack_csr(polys)
    return synth.AtlasInput(xy, off, inp.atlas_w, inp.atlas_h, inp.padding, 2)


@pytest.mark.parametrize("seed", range(12))
def test_balanced_only_packs_the_boxes(orc, seed):
    """Without tightening every chart is represented by its box: the
    balanced-only pack of the polygons equals the full method's pack of their
    bounding rectangles, whose proxies are exactly their boxes (and no
    feasible box packing exceeds the rectangles' area bound)."""
    inp = small_input(8200 + seed)
    got = orc.pack_method(inp, 10, -1, orc.BALANCED_ONLY)
    _same(got, orc.pack(_boxes(inp)))
    assert not np.any(got[1] & 6)  # no reflections


@pytest.mark.parametrize("a,b,n,Wa,Ha,p", [
    (256 * 3, 256 * 5, 37, 40, 40, 1), (1000, 1900, 50, 64, 90, 2), (700, 3000, 25, 50, 128, 3),
    (512, 512, 9, 9, 9, 1), (256 * 2, 256 * 7, 120, 64, 300, 0)])
def test_tight_only_identical_rectangles_closed_form(orc, a, b, n, Wa, Ha, p):
    """Static folding on identical rectangles: row r holds M = floor(W' /
    (w + p)) boxes, left to right when r = 0 mod 3 and right to left (mirror
    bit set) otherwise, each row pushed flat onto the last."""
    inp = synth.rect_input(n, a, b, Wa, Ha, p, q=2, seed=n)
    Wd, Hd = Wa + p, Ha + p

    def fits(k):
        w, h = -(-k * a // T), -(-k * b // T)
        M = Wd // (w + p)
        return M >= 1 and -(-n // M) * (h + p) <= Hd
    ks = [k for k in range(1, 65) if fits(k)]
    xy, ori, sc, k = orc.pack_method(inp, 10, -1, orc.TIGHT_ONLY)
    assert k == (max(ks) if ks else 0)
    if k:
        w, h = -(-k * a // T), -(-k * b // T)
        M = Wd // (w + p)
        for t in range(n):
            r, m = divmod(t, M)
            x = m * (w + p) if r % 3 == 0 else Wd - (m + 1) * (w + p)
            assert tuple(xy[t]) == (x, r * (h + p)), t
            assert bool(ori[t] & 8) == (r % 3 != 0), t


@pytest.mark.parametrize("seed", range(10))
def test_topt_100_folds_like_tight_only(orc, seed):
    """With t_opt = 100 % the switch to static rows happens before the first
    row (its tallest chart is shorter than the atlas), so the method equals
    tight-only."""
    inp = small_input(8300 + seed, n=20, q=2)
    perm, khi = orc.order(inp)
    Hmax = max(int(np.ptp(inp.chart(c), axis=0).max()) for c in range(inp.n))
    if -(-khi * Hmax // T) >= inp.atlas_h:
        pytest.skip("a chart as tall as the atlas at the top scale")
    for K in (2, 10):
        _same(orc.pack_method(inp, K, 100, orc.FULL), orc.pack_method(inp, K, 5, orc.TIGHT_ONLY))


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("K,topt", [(2, 0), (5, 1), (10, 2), (10, 5)])
def test_every_variant_gives_a_valid_layout(orc, chk, variant, K, topt):
    for seed in range(3):
        inp = small_input(8400 + seed)
        xy, ori, sc, k = orc.pack_method(inp, K, topt, variant)
        if k > 0:
            st = chk.check_layout(inp, xy, ori, k)
            assert st["overlap"] == 0 and st["outside"] == 0, (variant, K, topt, seed)


def test_invalid_knobs_are_refused(orc):
    inp = small_input(8500)
    for K, topt, v in [(0, 0, 0), (11, 0, 0), (10, 101, 0), (10, 0, 3), (10, 0, -1)]:
        with pytest.raises(ValueError):
            orc.pack_method(inp, K, topt, v)


def test_report_mean_stretch_by_variant(orc):
    """Reported, not asserted: the paper finds the full method's mean L2
    stretch below both single-component variants (Sec. 5 ablation table);
    this prints the same comparison on synthetic sets (stretch = 64 / k)."""
    sets = [synth.make_input("stars64", i) for i in range(4)]
    sets += [small_input(8600 + s, n=24) for s in range(8)]
    res = {}
    for name, v in (("full", 0), ("tight_only", 1), ("balanced_only", 2)):
        ks = [orc.pack_method(inp, 10, -1, v)[3] for inp in sets]
        assert all(k > 0 for k in ks)
        res[name] = float(np.mean([64.0 / k for k in ks]))
    print("mean L2 stretch by variant:", res, file=sys.stderr)
