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
