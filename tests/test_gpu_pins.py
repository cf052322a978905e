"""The oracle's hand-built pin cases run through the HIP library: closed
forms (single chart, identical rectangles, exact tiling), the knee
thresholds at +-1 Q8 unit, the tail's one-to-two direction alternation, the
orientation rules (App. A "Computing Chart Orientations"), the compaction
choice (Sec. 4.2 "Placing Rows"), the sort's tie-breaks and the degenerate
inputs.  Each case checks the GPU against the closed form or the hand-derived
answer directly, and against the oracle bit for bit."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from cases import small_input
from paper_2602_07782_amd import synth

pytestmark = pytest.mark.gpu
T = 16384
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


def _pack(tabi, inp):
    xy, ori, sc = tabi.pack(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h, inp.padding,
                            inp.quality, device="cuda:0")
    sc = float(sc.cpu().numpy()[0])
    return xy.cpu().numpy(), ori.cpu().numpy(), sc, int(round(sc * 64)) if sc > 0 else 0


def _same_as_oracle(orc, inp, got):
    oxy, oor, osc, ok = orc.pack(inp)
    assert got[2] == osc
    assert np.array_equal(got[0], oxy) and np.array_equal(got[1], oor)


def _feasible(tabi, inp, k):
    xy, ori, feas, rows = tabi.debug_feasible(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h,
                                              inp.padding, inp.quality, k, device="cuda:0")
    return int(feas.cpu().numpy()[0]), xy.cpu().numpy(), ori.cpu().numpy()


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(30))
def test_single_chart_closed_form(tabi, orc, seed):
    rng = np.random.default_rng(seed)
    inp0 = small_input(6000 + seed, n=1)
    Wa, Ha = int(rng.integers(4, 200)), int(rng.integers(4, 200))
    p = int(rng.integers(0, 4))
    inp = synth.AtlasInput(inp0.xy, inp0.offsets, Wa, Ha, p, int(rng.integers(0, 3)))
    _say("single chart closed form, seed", seed, (Wa, Ha, p))
    P = inp.chart(0)
    W, H = sorted(int(e) for e in P.max(axis=0) - P.min(axis=0))
    ks = [k for k in range(1, 65) if -(-k * W // T) <= Wa and -(-k * H // T) <= Ha]
    got = _pack(tabi, inp)
    assert got[3] == (max(ks) if ks else 0)
    if got[3]:
        assert tuple(got[0][0]) == (0, 0)
    _same_as_oracle(orc, inp, got)


@pytest.mark.parametrize("a,b,n,Wa,Ha,p", [
    (256 * 3, 256 * 5, 37, 40, 40, 1), (1000, 1900, 50, 64, 90, 2), (2048, 2048, 64, 64, 64, 0),
    (256 * 6, 256 * 6, 36, 36, 36, 0), (700, 3000, 25, 50, 128, 3), (512, 512, 9, 9, 9, 1),
    (256 * 2, 256 * 7, 300, 200, 200, 2)])
def test_identical_rectangles_closed_form(tabi, orc, a, b, n, Wa, Ha, p):
    inp = synth.rect_input(n, a, b, Wa, Ha, p, q=2, seed=n)
    _say("identical rectangles", (a, b, n, Wa, Ha, p))
    Wd, Hd = Wa + p, Ha + p

    def fits(k):
        w, h = -(-k * a // T), -(-k * b // T)
        M = Wd // (w + p)
        return M >= 1 and -(-n // M) * (h + p) <= Hd
    ks = [k for k in range(1, 65) if fits(k)]
    got = _pack(tabi, inp)
    assert got[3] == (max(ks) if ks else 0)
    if got[3]:
        k = got[3]
        w, h = -(-k * a // T), -(-k * b // T)
        M = Wd // (w + p)
        for t in range(n):
            assert tuple(got[0][t]) == ((t % M) * (w + p), (t // M) * (h + p)), t
    _same_as_oracle(orc, inp, got)


def test_exact_tiling_reaches_full_scale(tabi, orc):
    inp = synth.rect_input(24, 2560, 3840, 6 * 12 - 2, 4 * 17 - 2, 2)
    got = _pack(tabi, inp)
    assert got[3] == 64 and got[2] == 1.0
    _same_as_oracle(orc, inp, got)


# ---------------------------------------------------------------------------
# knees (>= 10 % of the atlas height and >= 20 % of the taller chart) and
# the tail's alternation
# ---------------------------------------------------------------------------
def _knee_input(tall_h_q8, short_h_q8, Ha):
    polys = [np.array([[0, 0], [20 * 256, 0], [20 * 256, tall_h_q8], [0, tall_h_q8]])]
    for i in range(30):
        ox = 1000 * (i + 1)
        polys.append(np.array([[ox, 0], [ox + 10 * 256, 0], [ox + 10 * 256, short_h_q8],
                               [ox, short_h_q8]]))
    xy, off = synth.pack_csr(polys)
    return synth.AtlasInput(xy, off, 100, Ha, 0, 2)


@pytest.mark.parametrize("tall,short,Ha,knee", [
    (60 * 256, 48 * 256, 100, True), (60 * 256, 48 * 256 + 1, 100, False),
    (40 * 256, 28 * 256, 120, True), (40 * 256, 28 * 256, 121, False)])
def test_knee_thresholds(tabi, orc, tall, short, Ha, knee):
    inp = _knee_input(tall, short, Ha)
    ok, xy, ori = _feasible(tabi, inp, 64)
    # row 0: the tall chart and 8 short ones; a knee starts row 1 at x = 20
    assert (int(xy[9][0]) == 20) == knee
    ook, oxy, oori, _ = orc.feasible(inp, 64)
    assert ok == int(ook) and np.array_equal(xy, oxy) and np.array_equal(ori, oori)


def test_tail_rows_follow_one_to_two_alternation(tabi, orc):
    n, a, b = 60, 256 * 2, 256 * 3
    inp = synth.rect_input(n, a, b, 20, 200, 0, q=0, seed=1)
    ok, xy, ori = _feasible(tabi, inp, 64)
    assert ok == 1
    for r in range(6):
        assert bool(ori[r * 10] & 8) == (r % 3 != 0), r
    ook, oxy, oori, _ = orc.feasible(inp, 64)
    assert np.array_equal(xy, oxy) and np.array_equal(ori, oori)


# ---------------------------------------------------------------------------
# orientation (App. A): the chart's reflection bits in a single-chart pack
# ---------------------------------------------------------------------------
def poly(*pts):
    return np.array(pts, np.int64)


def _orient_bits(tabi, orc, P, K):
    q = {2: 0, 5: 1, 10: 2}[K]
    xy, off = synth.pack_csr([P])
    inp = synth.AtlasInput(xy, off, 64, 64, 0, q)
    got = _pack(tabi, inp)
    _same_as_oracle(orc, inp, got)
    o = int(got[1][0])
    return (o & 1, (o >> 2) & 1, (o >> 1) & 1)  # rot, flipy, flipx


ORIENT_CASES = [
    # apex up: flip y; apex down: keep; rectangle: keep
    (poly((0, 4000), (3000, 4000), (1500, 0)), 10, (0, 1, 0)),
    (poly((0, 0), (3000, 0), (1500, 4000)), 10, (0, 0, 0)),
    (poly((0, 0), (3000, 0), (3000, 4000), (0, 4000)), 10, (0, 0, 0)),
    # left notch of width c: reflect in x iff c * H/2 > 10 % of W * H (c > 200)
    (poly((199, 0), (1000, 0), (1000, 2000), (0, 2000), (0, 1001), (199, 1001)), 2, (0, 0, 0)),
    (poly((200, 0), (1000, 0), (1000, 2000), (0, 2000), (0, 1001), (200, 1001)), 2, (0, 0, 0)),
    (poly((201, 0), (1000, 0), (1000, 2000), (0, 2000), (0, 1001), (201, 1001)), 2, (0, 0, 1)),
    # midline rule, K = 2
    (poly((0, 0), (1000, 0), (1000, 2000), (501, 2000), (501, 1700), (0, 1700)), 2, (0, 0, 1)),
    (poly((0, 0), (1000, 0), (1000, 1700), (499, 1700), (499, 2000), (0, 2000)), 2, (0, 0, 0)),
    # midline rule, K = 5 (the middle slice split between the halves)
    (poly((0, 0), (1000, 0), (1000, 2000), (601, 2000), (601, 1700), (399, 1700), (399, 2000),
          (0, 2000)), 5, (0, 0, 0)),
    (poly((0, 0), (1000, 0), (1000, 2000), (401, 2000), (401, 1700), (199, 1700), (199, 2000),
          (0, 2000)), 5, (0, 0, 1)),
    (poly((0, 0), (1000, 0), (1000, 2000), (801, 2000), (801, 1800), (601, 1800), (601, 1700),
          (399, 1700), (399, 2000), (0, 2000)), 5, (0, 0, 0)),
    # L, U and diagonal charts
    (poly((0, 0), (1200, 0), (1200, 2100), (3000, 2100), (3000, 5000), (0, 5000)), 10, (0, 1, 0)),
    (poly((1800, 0), (3000, 0), (3000, 5000), (0, 5000), (0, 2100), (1800, 2100)), 10, (0, 1, 1)),
    (poly((0, 0), (900, 0), (900, 3000), (2100, 3000), (2100, 0), (3000, 0), (3000, 5000),
          (0, 5000)), 10, (0, 1, 0)),
    (poly((0, 0), (400, 0), (3000, 4600), (3000, 5000), (2600, 5000), (0, 400)), 10, (0, 0, 1)),
]


@pytest.mark.parametrize("i", range(len(ORIENT_CASES)))
def test_orientation_rules(tabi, orc, i):
    P, K, want = ORIENT_CASES[i]
    assert _orient_bits(tabi, orc, P, K) == want


# ---------------------------------------------------------------------------
# compaction choice and sort ties
# ---------------------------------------------------------------------------
def _slanted_row(n, Wa, p):
    a, W, H = 3 * Q, 17 * Q, 40 * Q
    P = [np.array([[a + 20000 * i, 0], [W + 20000 * i, 0], [W - a + 20000 * i, H],
                   [20000 * i, H]]) for i in range(n)]
    xy, off = synth.pack_csr(P)
    return synth.AtlasInput(xy, off, Wa, 4000, p, 2)


@pytest.mark.parametrize("extra", [0, 1])
def test_compaction_only_when_it_fits_more(tabi, orc, extra):
    p, n, m = 3, 12, 3
    probe = _slanted_row(n, 100, p)
    cd, _ = tabi.debug_pairs(probe.xy, probe.offsets, p, 2, 64, device="cuda:0")
    cd = cd.cpu().numpy()
    wd, c = 17 + p, int(cd[1])
    assert c > 0 and np.all(cd[1:] == c) and m * c < wd
    Wd = m * wd if extra == 0 else m * (wd - c) + wd
    inp = _slanted_row(n, Wd - p, p)
    ok, xy, ori = _feasible(tabi, inp, 64)
    step = wd - c if extra else wd
    assert [int(xy[t][0]) for t in range(m + extra)] == [t * step for t in range(m + extra)]
    assert int(xy[m + extra][1]) > 0
    ook, oxy, oori, _ = orc.feasible(inp, 64)
    assert np.array_equal(xy, oxy) and np.array_equal(ori, oori)


def test_sort_breaks_height_ties_by_width(tabi, orc):
    widths, heights = [3, 7, 5, 7, 2], [10, 10, 10, 10, 12]
    P = [np.array([[1000 * i, 0], [1000 * i + w * Q, 0], [1000 * i + w * Q, h * Q],
                   [1000 * i, h * Q]]) for i, (w, h) in enumerate(zip(widths, heights))]
    xy, off = synth.pack_csr(P)
    perm, _ = tabi.debug_order(xy, off, 64, 64, 0, 2, device="cuda:0")
    assert list(perm.cpu().numpy()) == [4, 1, 3, 2, 0]


# ---------------------------------------------------------------------------
# degenerate inputs and the coordinate range
# ---------------------------------------------------------------------------
def test_degenerate_inputs_and_coordinate_range(tabi, orc):
    big = (1 << 22) - 1
    cases = [
        (np.array([0, 0, 100, 100], np.int32), -1.0),                      # 2 vertices
        (np.array([0, 0, 100, 0, 200, 0], np.int32), -1.0),                # zero height
        (np.array([0, 0, 0, 500, 0, 900], np.int32), -1.0),                # zero width
        (np.array([0, 0, 1 << 22, 0, 0, 100], np.int32), -1.0),            # |x| = 2^22
        (np.array([0, 0, 0, -(1 << 22), 100, 0], np.int32), -1.0),         # |y| = 2^22
        (np.array([-big, 0, big, 0, 0, 300 * 256], np.int32), None),       # |x| = 2^22 - 1
    ]
    for xy, want in cases:
        nv = len(xy) // 2
        inp = synth.AtlasInput(xy, np.array([0, nv], np.int32), 16000, 16000, 1, 2)
        _say("degenerate input", xy.tolist())
        got = _pack(tabi, inp)
        if want is not None:
            assert got[2] == want and np.all(got[0] == -1)
        else:
            assert got[2] > 0
        _same_as_oracle(orc, inp, got)
    big_chart = synth.rect_input(1, 100 * 256, 100 * 256, 1, 1, 0)
    got = _pack(tabi, big_chart)
    assert got[2] == 0.0 and np.all(got[0] == -1)
