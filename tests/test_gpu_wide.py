"""Wider seed sweeps of single-pack parity with the oracle, bit for bit:
100 instances of the 64-chart workload, 10 of the 2,000-chart workload at
the lowest and the highest quality, and 3 of the 20,000-chart workload.
The first mismatch stops the test and names its instance."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2602_07782_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tabi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_07782_amd as t
    t.lib()
    return t


def _check(tabi, orc, inp, label):
    xy, ori, sc = tabi.pack(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h, inp.padding,
                            inp.quality, device="cuda:0")
    oxy, oori, osc, ok = orc.pack(inp)
    assert float(sc.cpu().numpy()[0]) == osc, label
    assert np.array_equal(xy.cpu().numpy(), oxy), label
    assert np.array_equal(ori.cpu().numpy(), oori), label


def test_stars64_hundred_instances(tabi, orc):
    for inst in range(1, 101):
        _check(tabi, orc, synth.make_input("stars64", inst), f"stars64/{inst}")
    print("stars64: 100 instances equal", file=sys.stderr, flush=True)


@pytest.mark.parametrize("q", [0, 2])
def test_mixed2k_ten_instances(tabi, orc, q):
    for inst in range(1, 11):
        print("mixed2k instance", inst, "q", q, file=sys.stderr, flush=True)
        _check(tabi, orc, synth.make_input("mixed2k", inst, quality=q), f"mixed2k/{inst}/q{q}")


def test_lightmap20k_three_instances(tabi, orc):
    for inst in range(1, 4):
        print("lightmap20k instance", inst, file=sys.stderr, flush=True)
        _check(tabi, orc, synth.make_input("lightmap20k", inst), f"lightmap20k/{inst}")
