"""Pins of the oracle's pre-rotation of UV charts to their tight boxes
(Sec. 5 "Experimental Setup": UV charts are turned so that their tight
bounding boxes line up with the axes before packing; TSS charts are not).

The oracle searches 64 directions m pi / 128, turns the chart about its box
corner and moves the turned box to the origin.  What fixes it independently of its own arithmetic:
  * a rectangle turned by one of the 64 angles comes back to that angle, and
    an axis-aligned rectangle stays at 0;
  * rotating calipers: the least-area box of a convex polygon has a side on
    one of its edges, so a polygon whose edges all lie at searched angles
    finds its exact minimum;
  * the result is a rotation (distances, signed area and handedness kept, to
    the rounding of a Q8 unit) by the angle of the reported direction,
    computed here with floating-point trigonometry;
  * the chosen box is no larger than the box at any other searched angle
    (brute force in floating point, to rounding);
  * the pack of the rotated charts is a valid layout (independent rasteriser).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from cases import small_input
from paper_2602_07782_amd import synth

Q = 256


def _turn(P, th, shift=(100000, 70000)):
    c, s = math.cos(th), math.sin(th)
    R = np.array([[c, -s], [s, c]])
    return np.rint(np.asarray(P, float) @ R.T + np.array(shift)).astype(np.int64)


def _box_area(P):
    e = P.max(0) - P.min(0)
    return float(e[0]) * float(e[1])


@pytest.mark.parametrize("m0", [0, 1, 5, 8, 17, 31, 32, 40, 56, 63])
@pytest.mark.parametrize("wh", [(40, 15), (7, 30), (100, 3)])
def test_turned_rectangle_comes_back(orc, m0, wh):
    w, h = wh[0] * Q, wh[1] * Q
    P = _turn([(0, 0), (w, 0), (w, h), (0, h)], m0 * math.pi / 128)
    r, m = orc.prerotate(P)
    assert m == m0
    assert tuple(r.min(0)) == (0, 0)
    ext = r.max(0)
    assert abs(ext[0] - w) <= 2 and abs(ext[1] - h) <= 2, ext


@pytest.mark.parametrize("seed", range(6))
def test_axis_rectangle_and_square_stay(orc, seed):
    rng = np.random.default_rng(seed)
    w, h = int(rng.integers(1, 5000)), int(rng.integers(1, 5000))
    x0, y0 = int(rng.integers(-10000, 10000)), int(rng.integers(-10000, 10000))
    P = np.array([(x0, y0), (x0 + w, y0), (x0 + w, y0 + h), (x0, y0 + h)], np.int64)
    r, m = orc.prerotate(P)
    assert m == 0
    assert np.array_equal(r, P - np.array([x0, y0]))


@pytest.mark.parametrize("m0", [3, 12, 24, 45])
def test_convex_octagon_on_searched_edges(orc, m0):
    """A convex octagon whose edge directions are all multiples of pi/128
    (the box's side must lie on one of them, by rotating calipers): an
    elongated octagon with sides at th, th + pi/2 and chamfers at th + pi/4
    has its least-area box along th."""
    th = m0 * math.pi / 128
    L, Wd, c = 60 * Q, 20 * Q, 4 * Q
    P = [(c, 0), (L - c, 0), (L, c), (L, Wd - c), (L - c, Wd), (c, Wd), (0, Wd - c), (0, c)]
    r, m = orc.prerotate(_turn(P, th))
    assert m == m0


def _signed2(P):
    x, y = P[:, 0].astype(float), P[:, 1].astype(float)
    return float(np.dot(x, np.roll(y, -1)) - np.dot(np.roll(x, -1), y))


def _rotation_residual(P, r, m):
    """Largest deviation of r from P turned by -m pi/128, both boxes moved to
    the origin."""
    th = m * math.pi / 128
    c, s = math.cos(th), math.sin(th)
    d = P.astype(float) - P.min(0).astype(float)
    exp = np.stack([c * d[:, 0] + s * d[:, 1], -s * d[:, 0] + c * d[:, 1]], 1)
    exp -= exp.min(0)
    return float(np.abs(exp - r).max()), float(np.abs(d).max())


@pytest.mark.parametrize("seed", range(20))
def test_result_is_the_reported_rotation_and_least_box(orc, seed):
    inp = small_input(9100 + seed)
    for ci in range(inp.n):
        P = inp.chart(ci).astype(np.int64)
        r, m = orc.prerotate(P)
        assert 0 <= m < 64
        assert tuple(r.min(0)) == (0, 0)
        dev, R = _rotation_residual(P, r, m)
        # table entries are rounded to 2^-14, each result and the shift to
        # the origin to a Q8 unit
        assert dev <= 1.0 + 4.0 * R * 2.0 ** -14 + 1e-9, (ci, m, dev)
        # signed area kept (no reflection) to the rounding of the vertices
        a0 = synth._shoelace(P.astype(float))
        assert _signed2(P) * _signed2(r) > 0
        per = float(np.sum(np.hypot(*np.diff(np.vstack([P, P[:1]]), axis=0).T)))
        assert abs(synth._shoelace(r.astype(float)) - a0) <= per * 0.75 + 1, ci
        # least box among the searched angles, in floating point
        best = min(_box_area(_turn(P - P.min(0), -j * math.pi / 128, (0, 0)).astype(float))
                   for j in range(64))
        ext = r.max(0) - r.min(0)
        assert float(ext[0]) * float(ext[1]) <= best + 4 * (ext.sum() + 4), (ci, m)


def test_charts_the_pack_rejects_are_copied(orc):
    """Fewer than 3 vertices, or a coordinate outside (-2^22, 2^22): copied
    unchanged with direction 0, so the pack reports them as it would."""
    big = 1 << 22
    for P in ([(0, 0), (500, 900)], [(0, 0), (big, 0), (big, 300), (0, 300)],
              [(-big, 0), (10, 5), (20, 400)], []):
        P = np.array(P, np.int64).reshape(-1, 2)
        r, m = orc.prerotate(P)
        assert m == 0 and np.array_equal(r, P)
    # just inside the range: turned as usual
    P = np.array([(-big + 1, 0), (big - 1, 0), (big - 1, 3000), (-big + 1, 3000)], np.int64)
    r, m = orc.prerotate(P)
    assert m == 0 and tuple(r.min(0)) == (0, 0) and tuple(r.max(0)) == (2 * big - 2, 3000)


@pytest.mark.parametrize("seed", range(6))
def test_pack_after_prerotation(orc, chk, seed):
    """The pre-rotated pack is the plain pack of the rotated charts, and
    its layout is valid."""
    inp = small_input(9200 + seed, n=16)
    polys = [orc.prerotate(inp.chart(c))[0] for c in range(inp.n)]
    xy, off = synth.pack_csr(polys)
    rot = synth.AtlasInput(xy, off, inp.atlas_w, inp.atlas_h, inp.padding, inp.quality)
    got = orc.pack_prerotate(inp)
    ref = orc.pack(rot)
    assert got[2] == ref[2] and got[3] == ref[3]
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    assert list(got[4]) == [orc.prerotate(inp.chart(c))[1] for c in range(inp.n)]
    if got[3] > 0:
        st = chk.check_layout(rot, got[0], got[1], got[3])
        assert st["overlap"] == 0 and st["outside"] == 0


def test_prerotation_does_not_lose_scale_on_average(orc):
    """Reported, with a weak assertion: on randomly turned charts the
    pre-rotated pack reaches a scale at least as high on average as the plain
    one (the paper applies it because it improves packing quality)."""
    ks0, ks1 = [], []
    for s in range(10):
        inp = small_input(9300 + s, n=20, q=2)
        ks0.append(orc.pack(inp)[3])
        ks1.append(orc.pack_prerotate(inp)[3])
    assert np.mean(ks1) >= np.mean(ks0) - 1.0, (ks0, ks1)
