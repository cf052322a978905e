"""GPU parity of charts with several boundary loops (tabi_pack_loops):
mesh charts with holes and charts of islands, against the oracle bit for
bit; a chart with a short loop is degenerate."""
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


def _check(tabi, orc, L, label):
    print("loops parity:", label, "n =", L.n, file=sys.stderr, flush=True)
    xy, ori, sc = tabi.pack_loops(L.xy, L.loop_offsets, L.chart_loops, L.atlas_w, L.atlas_h,
                                  L.padding, L.quality, device="cuda:0")
    oxy, oor, osc, ok = orc.pack_loops(L)
    assert float(sc.cpu().numpy()[0]) == osc, (label, osc)
    assert np.array_equal(xy.cpu().numpy(), oxy), label
    assert np.array_equal(ori.cpu().numpy(), oor), label


@pytest.mark.parametrize("seed,holes,islands,q", [(0, 0.4, 0.2, 2), (1, 1.0, 0.0, 2),
                                                  (2, 0.0, 1.0, 2), (3, 0.5, 0.3, 0),
                                                  (4, 0.3, 0.3, 1)])
def test_loops_parity_small(tabi, orc, seed, holes, islands, q):
    L, _ = synth.make_loops(120, 384, 384, 2, q, 800 + seed, hole_frac=holes, island_frac=islands)
    _check(tabi, orc, L, f"small {seed}")


def test_loops_parity_large(tabi, orc):
    L, _ = synth.make_loops(1500, 2048, 2048, 2, 2, 900)
    _check(tabi, orc, L, "1,500 charts")


def test_short_loop_is_degenerate(tabi, orc):
    good = np.array([[0, 0], [2560, 0], [2560, 2560], [0, 2560]], np.int64)
    L = synth.loops_csr([[good], [good + 5000, np.array([[1, 1], [5, 5]], np.int64)]],
                        64, 64, 1, 2)
    _check(tabi, orc, L, "short loop")
