"""GPU parity of the hybrid tail (Sec. 4.4 "Performance Optimization"):
tabi_pack_hybrid against the oracle's hybrid pack, bit for bit (positions,
orientation bits, each chart's scale, the head scale)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from cases import small_input
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


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _check(tabi, orc, inp, K, topt, label):
    _say("hybrid parity:", label, "n =", inp.n, "K", K, "t_opt", topt)
    xy, ori, ks, sc = tabi.pack_hybrid(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h,
                                       inp.padding, K, topt, device="cuda:0")
    oxy, oori, oks, ok = orc.pack_hybrid(inp, K, topt)
    sc = float(sc.cpu().numpy()[0])
    want = -1.0 if ok < 0 else ok / 64.0
    assert sc == want, (label, sc, ok)
    assert np.array_equal(ks.cpu().numpy(), oks.astype(np.float32) / 64.0), label
    assert np.array_equal(xy.cpu().numpy(), oxy), (label, np.argwhere(xy.cpu().numpy() != oxy)[:4])
    assert np.array_equal(ori.cpu().numpy(), oori), label
    return oks, ok


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("topt", [5, 20, 100])
def test_hybrid_parity_small(tabi, orc, seed, topt):
    _check(tabi, orc, small_input(9600 + seed, n=60, W=128, q=2), 10, topt, f"small {seed}")


@pytest.mark.parametrize("seed", [0, 1, 8, 9])
@pytest.mark.parametrize("topt", [30, 100])
def test_hybrid_parity_where_a_lower_head_scale_wins(tabi, orc, seed, topt):
    _check(tabi, orc, small_input(9650 + seed, n=50, W=128, q=2), 10, topt, f"choice {seed}")


@pytest.mark.parametrize("K", [1, 2, 5])
def test_hybrid_parity_other_slices(tabi, orc, K):
    for seed in range(3):
        _check(tabi, orc, small_input(9700 + seed, n=60, W=128, q=2), K, 20, f"K{K} {seed}")


@pytest.mark.parametrize("a,b,n,Wa,Ha,p", [
    (256 * 3, 256 * 5, 37, 40, 60, 1), (1000, 1900, 50, 64, 90, 2), (700, 3000, 25, 50, 200, 3),
    (256 * 2, 256 * 7, 120, 64, 300, 0), (900, 1300, 80, 100, 100, 2)])
def test_hybrid_parity_identical_rectangles(tabi, orc, a, b, n, Wa, Ha, p):
    _check(tabi, orc, synth.rect_input(n, a, b, Wa, Ha, p, q=2, seed=n), 10, 100, "rectangles")


def test_hybrid_without_tail_is_the_method(tabi, orc):
    inp = small_input(9500, n=30)
    xy, ori, ks, sc = tabi.pack_hybrid(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h,
                                       inp.padding, 10, 0, device="cuda:0")
    pxy, pori, psc = tabi.pack_method(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h,
                                      inp.padding, 10, 0, 0, device="cuda:0")
    assert float(sc.cpu().numpy()[0]) == float(psc.cpu().numpy()[0])
    assert np.array_equal(xy.cpu().numpy(), pxy.cpu().numpy())
    assert np.array_equal(ori.cpu().numpy(), pori.cpu().numpy())


@pytest.mark.parametrize("topt", [1, 2, 5])
def test_hybrid_parity_mixed2k(tabi, orc, topt):
    oks, ok = _check(tabi, orc, synth.make_input("mixed2k", 0), 10, topt, "mixed2k")
    assert ok > 0


def test_hybrid_parity_tss_frame(tabi, orc):
    _check(tabi, orc, synth.make_tss(0), 10, 5, "tss 4000")


def test_hybrid_parity_lightmap20k_paper_setting(tabi, orc):
    """The paper's setting (t_opt 1 % above 10,000 charts) on the 20,000-chart
    workload: most charts land in the tail."""
    oks, ok = _check(tabi, orc, synth.make_input("lightmap20k", 0), 10, -1, "lightmap20k")
    assert ok > 0 and (oks < ok).any()


def test_hybrid_degenerate_and_empty(tabi, orc):
    two = synth.AtlasInput(np.array([0, 0, 100, 100, 0, 0, 500, 0, 500, 500], np.int32),
                           np.array([0, 2, 5], np.int32), 64, 64, 1, 2)
    _check(tabi, orc, two, 10, 5, "degenerate")
    big = synth.rect_input(1, 100 * 256, 100 * 256, 1, 1, 0)
    _check(tabi, orc, big, 10, 5, "no fit")
    xy, ori, ks, sc = tabi.pack_hybrid(np.zeros(0, np.int32), np.zeros(1, np.int32), 64, 64, 1,
                                       10, 5, device="cuda:0")
    assert float(sc.cpu().numpy()[0]) == 1.0


def test_hybrid_refuses_other_variants(tabi):
    import ctypes
    inp = small_input(9500, n=5)
    ch = tabi.Charts(0, 0, 0)
    m = tabi.Method(10, 5, 1)
    rc = tabi.lib().tabi_pack_hybrid(ctypes.byref(ch), 0, 64, 64, 1, ctypes.byref(m), None, None,
                                     None, None, None)
    assert rc == tabi.TABI_EINVAL
    del inp
