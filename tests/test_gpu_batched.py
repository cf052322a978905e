"""Batched path (tabi_pack_many) on the GPU: every atlas of a batch equals the
oracle's pack of that atlas alone, bit for bit; the work-space variant can be
captured in a HIP graph and replayed."""
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


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def small_batch(count, seed, nmin=20, nmax=400, sides=(256, 512, 1024)):
    rng = np.random.default_rng(seed)
    mix = synth.CONFIGS["mixed2k"]["mix"]
    out = []
    for a in range(count):
        side = int(rng.choice(sides))
        n = int(rng.integers(nmin, nmax + 1))
        out.append(synth.make_custom(n, side, side, 2, 2, 1.2, 1.2, mix, seed * 1000 + a))
    return out


def check_batch(tabi, orc, inputs, use_workspace=False):
    xy, ori, sc = tabi.pack_many(inputs, use_workspace=use_workspace)
    xy, ori, sc = xy.cpu().numpy(), ori.cpu().numpy(), sc.cpu().numpy()
    c0 = 0
    for a, inp in enumerate(inputs):
        oxy, oori, osc, ok = orc.pack(inp)
        n = inp.n
        assert float(sc[a]) == osc, (a, sc[a], osc)
        assert np.array_equal(xy[c0:c0 + n], oxy), a
        assert np.array_equal(ori[c0:c0 + n], oori), a
        c0 += n


@pytest.mark.parametrize("seed", range(3))
def test_batch_equals_oracle_per_atlas(tabi, orc, seed):
    inputs = small_batch(12, 700 + seed)
    _say("batch", seed, [i.n for i in inputs])
    check_batch(tabi, orc, inputs)


def test_batch_workspace_variant(tabi, orc):
    check_batch(tabi, orc, small_batch(8, 777), use_workspace=True)


def test_batch_with_degenerate_and_empty_atlas(tabi, orc):
    inputs = small_batch(4, 900)
    bad = synth.AtlasInput(np.array([0, 0, 100, 100, 5, 5, 9, 9, 300, 0, 0, 300], np.int32),
                           np.array([0, 2, 6], np.int32), 64, 64, 2, 2)
    empty = synth.AtlasInput(np.zeros(0, np.int32), np.zeros(1, np.int32), 64, 64, 2, 2)
    inputs = inputs[:2] + [bad] + inputs[2:] + [empty]
    xy, ori, sc = tabi.pack_many(inputs)
    sc = sc.cpu().numpy()
    assert sc[2] == -1.0 and sc[-1] == 1.0
    good = [i for j, i in enumerate(inputs) if j not in (2, len(inputs) - 1)]
    check_batch(tabi, orc, good)


def test_batch_of_mixed2k_atlases(tabi, orc):
    inputs = [synth.make_input("mixed2k", i) for i in range(2)] + small_batch(3, 901)
    check_batch(tabi, orc, inputs)


def test_graph_capture_replay(tabi):
    import torch
    inputs = small_batch(6, 905)
    batch = tabi.Batch(inputs)
    ref = [t.clone() for t in batch.run(use_workspace=True)]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run(stream=s, use_workspace=True)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        batch.run(stream=s, use_workspace=True)
    for rep in range(3):
        batch.out_xy.fill_(-7)
        batch.out_scale.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = (batch.out_xy.sum() + 1).item()  # eager work between replays
        assert torch.equal(batch.out_xy, ref[0]), rep
        assert torch.equal(batch.out_orient, ref[1]), rep
        assert torch.equal(batch.out_scale, ref[2]), rep


def test_every_batched_shape_gives_the_same_results(tabi, orc):
    """Each candidate shape of the batched path (slots per round, workgroup
    size, LDS cap) packs the batch identically, and equals the oracle."""
    inputs = small_batch(8, 930)
    q = inputs[0].quality
    first = None
    try:
        for idx in range(int(tabi.lib().tabi_many_shape_count())):
            tabi.debug_set_many_shape(q, idx)
            _say("shape", idx, tabi.many_shape(q, len(inputs)))
            out = [t.cpu().numpy() for t in tabi.pack_many(inputs)]
            if first is None:
                first = out
                check_batch(tabi, orc, inputs)
            else:
                for x, y in zip(out, first):
                    assert np.array_equal(x, y), idx
    finally:
        tabi.debug_set_many_shape(q, -1)


def test_tuner_keeps_results(tabi):
    """tabi_tune_many times the candidate shapes, keeps the fastest, and
    later batched calls (plain and work-space) still give the same results."""
    inputs = small_batch(6, 931)
    q = inputs[0].quality
    try:
        ref = [t.cpu().numpy() for t in tabi.pack_many(inputs)]
        batch = tabi.Batch(inputs)
        res = batch.tune(reps=1)
        _say("tuned", res)
        assert res["shape"] == tabi.many_shape(q, len(inputs))
        assert min(m for m in res["ms"] if m >= 0) > 0
        for use_ws in (False, True):
            out = [t.cpu().numpy() for t in tabi.Batch(inputs).run(use_workspace=use_ws)]
            for x, y in zip(out, ref):
                assert np.array_equal(x, y), use_ws
    finally:
        tabi.debug_set_many_shape(q, -1)


@pytest.mark.parametrize("q,p", [(0, 0), (1, 5)])
def test_batch_other_quality_and_padding(tabi, orc, q, p):
    """Fewer slices per axis and other gutters through the batched path."""
    rng = np.random.default_rng(940 + q)
    mix = synth.CONFIGS["mixed2k"]["mix"]
    inputs = [synth.make_custom(int(rng.integers(20, 300)), int(s), int(s), p, q, 1.2, 1.2, mix,
                                9400 + 10 * q + a)
              for a, s in enumerate(rng.choice([256, 512, 1024], size=6))]
    _say("batch q", q, "p", p, [i.n for i in inputs])
    check_batch(tabi, orc, inputs)


@pytest.mark.parametrize("shape", [0, 5])
def test_large_batch_equals_single_packs(tabi, shape):
    """A batch of more than 64 atlases (its own shape class) under the
    default shape and under a doubling round schedule equals one tabi_pack
    per atlas."""
    inputs = small_batch(72, 950, nmin=20, nmax=200, sides=(256, 512))
    q = inputs[0].quality
    try:
        tabi.debug_set_many_shape(q, shape)
        _say("large batch shape", tabi.many_shape(q, len(inputs)))
        xy, ori, sc = [t.cpu().numpy() for t in tabi.pack_many(inputs)]
    finally:
        tabi.debug_set_many_shape(q, -1)
    c0 = 0
    for a, inp in enumerate(inputs):
        pxy, por, psc = tabi.pack(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h, inp.padding,
                                  inp.quality)
        n = inp.n
        assert float(sc[a]) == float(psc.cpu().numpy()[0]), a
        assert np.array_equal(xy[c0:c0 + n], pxy.cpu().numpy()), a
        assert np.array_equal(ori[c0:c0 + n], por.cpu().numpy()), a
        c0 += n


@pytest.mark.parametrize("words", [0, 60000])
def test_batch_without_stored_profiles(tabi, orc, words):
    """Profile blocks whose pairs have no stored rows are queued by the lean
    profile kernel and evaluated in full form by the queued-block launch;
    the batch still equals the oracle per atlas (0: no arena, every block
    queued; 60000 words: some segments stored, the others not)."""
    tabi.debug_set_profile_cap(words)
    try:
        inputs = small_batch(6, 960 + words % 7)
        _say("batch arena", words, [i.n for i in inputs])
        check_batch(tabi, orc, inputs)
        check_batch(tabi, orc, small_batch(3, 970), use_workspace=True)
    finally:
        tabi.debug_set_profile_cap(-1)


def test_batch_above_reorder_limit(tabi, orc):
    """More atlases than the packing kernel reorders (4,096): the batch keeps
    its own dispatch order and every sampled atlas still equals the oracle."""
    rng = np.random.default_rng(990)
    mix = synth.CONFIGS["mixed2k"]["mix"]
    count = 4100
    inputs = [synth.make_custom(int(rng.integers(1, 5)), 64, 64, 2, 2, 1.2, 1.2, mix, 99000 + a,
                                fast=True)
              for a in range(count)]
    _say("batch of", count, "atlases,", sum(i.n for i in inputs), "charts")
    xy, ori, sc = [t.cpu().numpy() for t in tabi.pack_many(inputs)]
    starts = np.cumsum([0] + [i.n for i in inputs])
    for a in list(range(0, count, 97)) + [count - 1]:
        inp = inputs[a]
        oxy, oori, osc, ok = orc.pack(inp)
        c0 = starts[a]
        assert float(sc[a]) == osc, (a, sc[a], osc)
        assert np.array_equal(xy[c0:c0 + inp.n], oxy), a
        assert np.array_equal(ori[c0:c0 + inp.n], oori), a


def test_records_entry_points_on_one_stream(tabi, orc):
    """tabi_prep_records, tabi_splice_records and tabi_pack_many_records on
    the current stream: a batch packed from records equals the oracle per
    atlas, and a spliced re-pack equals the oracle on the new chart set."""
    import torch
    inputs = small_batch(3, 41, nmax=250)
    dev = torch.device("cuda:0")
    xy, voff, aoff, wh = [], [0], [0], []
    for inp in inputs:
        xy.append(np.asarray(inp.xy, np.int32).reshape(-1))
        o = np.asarray(inp.offsets, np.int64)
        voff += list((o[1:] + voff[-1]).astype(np.int64))
        aoff.append(aoff[-1] + inp.n)
        wh += [inp.atlas_w, inp.atlas_h]
    rec = tabi.prep_records(np.concatenate(xy), np.array(voff, np.int32),
                            np.array(aoff, np.int32), 2, device=dev)
    N = aoff[-1]
    aoff_t = torch.tensor(aoff, dtype=torch.int32).to(dev)
    wh_t = torch.tensor(wh, dtype=torch.int32).to(dev)
    oxy = torch.empty((N, 2), dtype=torch.int32, device=dev)
    oor = torch.empty(N, dtype=torch.uint8, device=dev)
    osc = torch.empty(len(inputs), dtype=torch.float32, device=dev)
    side = max(max(i.atlas_w, i.atlas_h) for i in inputs)
    tabi.pack_many_records(rec, aoff_t, wh_t, max(i.n for i in inputs), side, 2, 2, oxy, oor, osc)
    gxy, gor, gsc = oxy.cpu().numpy(), oor.cpu().numpy(), osc.cpu().numpy()
    for a, inp in enumerate(inputs):
        _say("records batch atlas", a, "n =", inp.n)
        e_xy, e_or, e_sc, _ = orc.pack(inp)
        assert float(gsc[a]) == e_sc
        assert np.array_equal(gxy[aoff[a]:aoff[a + 1]], e_xy)
        assert np.array_equal(gor[aoff[a]:aoff[a + 1]], e_or)
    # re-pack of the first atlas with three charts replaced by charts of the second
    base, donor = inputs[0], inputs[1]
    idx = np.array([1, 4, 7], np.int32)
    polys = [base.chart(c) for c in range(base.n)]
    for j, c in enumerate(idx):
        polys[c] = donor.chart(j)
    nxy, noff = synth.pack_csr(polys)
    new_inp = synth.AtlasInput(nxy, noff, base.atlas_w, base.atlas_h, base.padding, base.quality)
    sub_xy, sub_off = synth.pack_csr([donor.chart(j) for j in range(len(idx))])
    new = tabi.prep_records(sub_xy, sub_off, np.array([0, len(idx)], np.int32), 2, device=dev)
    rec0 = rec[:base.n].clone()
    tabi.splice_records(rec0, idx, new)
    one = torch.tensor([0, base.n], dtype=torch.int32).to(dev)
    wh1 = torch.tensor([base.atlas_w, base.atlas_h], dtype=torch.int32).to(dev)
    oxy1 = torch.empty((base.n, 2), dtype=torch.int32, device=dev)
    oor1 = torch.empty(base.n, dtype=torch.uint8, device=dev)
    osc1 = torch.empty(1, dtype=torch.float32, device=dev)
    tabi.pack_many_records(rec0, one, wh1, base.n, max(base.atlas_w, base.atlas_h), 2, 2, oxy1,
                           oor1, osc1)
    e_xy, e_or, e_sc, _ = orc.pack(new_inp)
    assert float(osc1.cpu().numpy()[0]) == e_sc
    assert np.array_equal(oxy1.cpu().numpy(), e_xy)
    assert np.array_equal(oor1.cpu().numpy(), e_or)


def test_timed_256_atlas_batch_sample_equals_oracle(tabi, orc):
    """The timed batch itself (256 atlases, sides 512-2048, 50-5,000 charts),
    packed in one tabi_pack_many call; the three largest 2048^2 atlases and
    five others drawn at random are compared with the oracle."""
    batch = synth.make_batch(256, 4000)
    _say("timed batch: generated, charts", sum(i.n for i in batch))
    xy, ori, sc = tabi.pack_many(batch)
    xy, ori, sc = xy.cpu().numpy(), ori.cpu().numpy(), sc.cpu().numpy()
    ns = np.array([i.n for i in batch])
    c0 = np.concatenate([[0], np.cumsum(ns)])
    big = [int(i) for i in np.argsort(-ns, kind="stable") if batch[i].atlas_w == 2048][:3]
    rng = np.random.default_rng(4001)
    rest = [int(i) for i in rng.choice(np.setdiff1d(np.arange(256), big), 5, replace=False)]
    for a in big + rest:
        _say("timed batch atlas", a, "n =", batch[a].n, "side", batch[a].atlas_w)
        oxy, oori, osc, ok = orc.pack(batch[a])
        assert float(sc[a]) == osc, (a, sc[a], osc)
        assert np.array_equal(xy[c0[a]:c0[a + 1]], oxy), a
        assert np.array_equal(ori[c0[a]:c0[a + 1]], oori), a
