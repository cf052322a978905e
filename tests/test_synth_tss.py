"""The TSS-like workload generator: charts lie on the 1920 x 1080 screen,
border patches are clipped to it (straight edges along the screen edges),
every chart is a simple polygon, and the oracle packs a frame."""
from __future__ import annotations

import numpy as np

from paper_2602_07782_amd import synth

Q8 = 256


def test_tss_frame_is_clipped_to_the_screen_and_simple():
    inp = synth.make_tss(1, n=600)
    SW, SH = synth.TSS["screen"]
    assert inp.n == 600
    on_border = 0
    for c in range(inp.n):
        P = inp.chart(c).astype(np.int64)
        assert P[:, 0].min() >= 0 and P[:, 0].max() <= SW * Q8
        assert P[:, 1].min() >= 0 and P[:, 1].max() <= SH * Q8
        assert synth.polygon_is_simple(P)
        on_border += bool(np.any((P[:, 0] == 0) | (P[:, 0] == SW * Q8) | (P[:, 1] == 0) |
                                 (P[:, 1] == SH * Q8)))
    assert 0.02 * inp.n < on_border < 0.3 * inp.n  # some, not most, are clipped


def test_clip_to_rect_matches_exact_cases():
    sq = np.array([[-1.0, -1.0], [3.0, -1.0], [3.0, 3.0], [-1.0, 3.0]])
    C = synth.clip_to_rect(sq, 0, 0, 2, 2)
    assert abs(synth._shoelace(C) - 4.0) < 1e-12
    tri = np.array([[0.0, 0.0], [4.0, 0.0], [0.0, 4.0]])
    C = synth.clip_to_rect(tri, 0, 0, 2, 2)  # the unit square minus nothing: x+y<=4 covers it
    assert abs(synth._shoelace(C) - 4.0) < 1e-12
    C = synth.clip_to_rect(tri + 10.0, 0, 0, 2, 2)
    assert C.shape[0] == 0


def test_oracle_packs_a_small_tss_frame(orc, chk):
    inp = synth.make_tss(2, n=300, atlas=256)
    xy, ori, sc, k = orc.pack(inp)
    assert k > 0
    st = chk.check_layout(inp, xy, ori, k)
    assert st["overlap"] == 0 and st["outside"] == 0
