"""Seeded test inputs shared by the oracle pins and the GPU parity tests."""
from __future__ import annotations

import numpy as np

from paper_2602_07782_amd import synth

SMALL_MIX = [("star", 0.5, 5, 16, 6.0), ("lu", 0.3, 6, 8, 6.0), ("quad", 0.2, 4, 8, 10.0)]


def small_input(seed, n=None, W=None, p=None, q=None):
    """A few charts of every shape family in a small square atlas."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 24)) if n is None else n
    W = int(rng.choice([32, 64, 96, 128])) if W is None else W
    p = int(rng.integers(0, 4)) if p is None else p
    q = int(rng.integers(0, 3)) if q is None else q
    return synth.make_custom(n, W, W, p, q, float(rng.uniform(0.3, 1.5)),
                             float(rng.uniform(0.2, 1.2)), SMALL_MIX, 90000 + seed)


def with_quality(inp, q):
    return synth.AtlasInput(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h, inp.padding, q)


def many_pairs_input(quality=2, slivers=400):
    """A row with more than 256 pairs of charts that share columns without
    being neighbours: a chart shaped like a T on its side (a full-height bar
    on the left, a bar to the right across the middle, empty above and below
    it on the right) followed by `slivers` one-texel-wide rectangles short
    enough to slide into its empty top-right part.  In a 1024^2 atlas with
    padding 1, at scale 64/64 the first sliver compacts under the T and every
    sliver starting within the T's width shares columns with it."""
    Q = 256
    Wl, Hl, wv, ym, hb = 700, 800, 100, 300, 60  # texels; the empty part above the bar is 300 tall
    hs = 200 if quality == 2 else 150            # below the slice that meets the bar
    tee = np.array([(0, 0), (wv, 0), (wv, ym), (Wl, ym), (Wl, ym + hb), (wv, ym + hb), (wv, Hl),
                    (0, Hl)], np.int64) * Q
    polys = [tee]
    for i in range(slivers):
        x0 = 2000 + 3 * i  # anywhere: positions come from the packer
        polys.append(np.array([(x0, 0), (x0 + 1, 0), (x0 + 1, hs), (x0, hs)], np.int64) * Q)
    xy, off = synth.pack_csr(polys)
    return synth.AtlasInput(xy, off, 1024, 1024, 1, quality)
