"""GPU parity of the method's knobs and ablation variants (Sec. 5
"Ablations"; App. D local-AABB count and t_opt tables): tabi_pack_method and
tabi_pack_many_method against the oracle's pack with the same knobs, bit for
bit (positions, orientation bits, scale)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from cases import small_input
from paper_2602_07782_amd import synth

pytestmark = pytest.mark.gpu

KNOBS = [(1, -1, 0), (2, 0, 0), (5, 1, 0), (10, 2, 0), (10, 5, 0), (2, 5, 0), (10, 100, 0),
         (10, -1, 1), (2, -1, 1), (10, -1, 2), (5, 3, 2)]


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


def _check(tabi, orc, inp, K, topt, v, label):
    _say("method parity:", label, "n =", inp.n, "knobs", (K, topt, v))
    xy, ori, sc = tabi.pack_method(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h, inp.padding,
                                   K, topt, v, device="cuda:0")
    oxy, oor, osc, ok = orc.pack_method(inp, K, topt, v)
    assert float(sc.cpu().numpy()[0]) == osc, (label, K, topt, v)
    assert np.array_equal(xy.cpu().numpy(), oxy), (label, K, topt, v)
    assert np.array_equal(ori.cpu().numpy(), oor), (label, K, topt, v)


@pytest.mark.parametrize("K,topt,v", KNOBS)
def test_method_parity_small(tabi, orc, K, topt, v):
    for seed in range(4):
        _check(tabi, orc, small_input(9100 + seed), K, topt, v, f"small {seed}")


@pytest.mark.parametrize("K,topt,v", [(10, -1, 1), (10, -1, 2), (5, 1, 0), (2, 0, 0)])
def test_method_parity_stars64(tabi, orc, K, topt, v):
    _check(tabi, orc, synth.make_input("stars64", 3), K, topt, v, "stars64")


@pytest.mark.parametrize("K,topt,v", [(10, -1, 1), (10, -1, 2), (10, 1, 0), (2, 2, 0)])
def test_method_parity_mixed2k(tabi, orc, K, topt, v):
    _check(tabi, orc, synth.make_input("mixed2k", 2), K, topt, v, "mixed2k")


def test_invalid_knobs_are_refused(tabi):
    inp = small_input(9200)
    for K, topt, v in [(3, 0, 0), (10, 101, 0), (10, -2, 0), (10, 0, 3), (0, 0, 0)]:
        with pytest.raises(tabi.TabiError):
            tabi.pack_method(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h, inp.padding, K, topt,
                             v, device="cuda:0")


@pytest.mark.parametrize("K,topt,v", [(10, -1, 1), (10, -1, 2), (5, 2, 0)])
def test_batched_method_parity(tabi, orc, K, topt, v):
    rng = np.random.default_rng(9300)
    mix = synth.CONFIGS["mixed2k"]["mix"]
    inputs = [synth.make_custom(int(rng.integers(20, 300)), side, side, 2, 2, 1.2, 1.2, mix,
                                9300 + a)
              for a, side in enumerate([256, 512, 1024, 512, 256, 1024])]
    b = tabi.Batch(inputs, device="cuda:0")
    xy, ori, sc = b.run_method(K, topt, v)
    xy, ori, sc = xy.cpu().numpy(), ori.cpu().numpy(), sc.cpu().numpy()
    c0 = 0
    for a, inp in enumerate(inputs):
        oxy, oor, osc, _ = orc.pack_method(inp, K, topt, v)
        assert float(sc[a]) == osc, (a, K, topt, v)
        assert np.array_equal(xy[c0:c0 + inp.n], oxy), a
        assert np.array_equal(ori[c0:c0 + inp.n], oor), a
        c0 += inp.n
