"""Serving path on the GPU: the library's serving context (tabi_ctx) on a
Poisson trace of new atlases and re-packs of resident ones, with several
launch slots so that batches overlap.  Every request's result in the mix
equals the same chart set packed alone by tabi_pack (tolerance 0), and the
oracle's on a sample."""
from __future__ import annotations

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _trace():
    from paper_2602_07782_amd import serve
    return serve.make_trace(rate=2000.0, seconds=0.06, seed=77, pool_size=8, nmin=16, nmax=1500,
                            sides=(256, 512, 1024))


def _serve(reqs, **kw):
    from paper_2602_07782_amd import serve
    srv = serve.Server(**kw)
    _say("serving", len(reqs), "requests with", kw)
    srv.run(reqs)
    st = srv.stats()
    srv.close()
    _say("stats", st)
    return st


@pytest.fixture(scope="module")
def served():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    reqs = _trace()
    st = _serve(reqs, streams=3, max_batch=16, hbm_budget=1 << 30, staging_bytes=16 << 20)
    return reqs, st


def _alone(r):
    import torch
    import paper_2602_07782_amd as tabi
    xy, ori, sc = tabi.pack(r.inp.xy, r.inp.offsets, r.inp.atlas_w, r.inp.atlas_h, r.inp.padding,
                            r.inp.quality, device="cuda:0")
    torch.cuda.synchronize()
    return xy.cpu().numpy(), ori.cpu().numpy(), float(sc.cpu().numpy()[0])


def _same(r, ref):
    assert r.result is not None, r.rid
    assert r.result[2] == ref[2], (r.rid, r.result[2], ref[2])
    assert np.array_equal(r.result[0], ref[0]), (r.rid, np.argwhere(r.result[0] != ref[0])[:5])
    assert np.array_equal(r.result[1], ref[1]), r.rid


def test_trace_has_repacks_and_overlap(served):
    reqs, st = served
    assert any(r.replaced is not None for r in reqs)
    assert st["finished"] == len(reqs) and st["failed"] == 0
    assert st["launches"] < len(reqs)          # requests were batched
    assert st["peak_in_flight"] >= 2           # batches overlapped on several slots


def test_served_equals_alone(served):
    reqs, _ = served
    for r in reqs:
        _same(r, _alone(r))


def test_served_sample_equals_oracle(served, orc):
    reqs, _ = served
    sample = [r for r in reqs if r.replaced is not None][:3] + [r for r in reqs if r.inp.n < 400][:3]
    for r in sample:
        oxy, oor, osc, _ = orc.pack(r.inp)
        assert r.result[2] == osc
        assert np.array_equal(r.result[0], oxy) and np.array_equal(r.result[1], oor)


def test_tight_budget_evicts_and_gives_same_results():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    reqs = _trace()
    st = _serve(reqs, streams=2, max_batch=8, hbm_budget=12 << 20, staging_bytes=8 << 20)
    assert st["evicted"] > 0
    assert st["device_bytes_peak"] <= 12 << 20
    for r in reqs:
        _same(r, _alone(r))


def test_single_slot_gives_same_results():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    reqs = _trace()[:40]
    _serve(reqs, streams=1, max_batch=4, hbm_budget=256 << 20, staging_bytes=4 << 20)
    for r in reqs:
        _same(r, _alone(r))


def test_requests_with_their_own_padding_and_quality():
    """tabi_submit_with: requests of mixed padding and quality in one
    context (batched only with same-setting neighbours); each result equals
    tabi_pack of that request alone with its settings, and re-packs keep
    their atlas's settings."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_07782_amd as tabi
    from paper_2602_07782_amd import synth
    rng = np.random.default_rng(515)
    mix = synth.CONFIGS["mixed2k"]["mix"]
    ctx = tabi.ServeContext(quality=2, padding=2, streams=3, max_batch=8, device_bytes=512 << 20,
                            staging_bytes=8 << 20)
    reqs = []
    for i in range(24):
        p, q = int(rng.choice([0, 1, 2, 5])), int(rng.integers(0, 3))
        inp = synth.make_custom(int(rng.integers(20, 300)), 512, 512, p, q, 1.2, 1.2, mix, 5150 + i)
        aid, t = ctx.submit(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h, padding=p, quality=q)
        reqs.append((t, aid, inp))
    got = {}
    while len(got) < len(reqs):
        for ticket, aid, status, batch, lat, out in ctx.poll(wait=True):
            assert status == tabi.TABI_OK
            got[ticket] = out
    # a re-pack of the first atlas keeps its padding and quality
    t0, aid0, inp0 = reqs[0]
    idx = np.array([0, 2], np.int32)
    polys = [inp0.chart(c) for c in range(inp0.n)]
    donor = reqs[1][2]
    for j, c in enumerate(idx):
        polys[c] = donor.chart(j)
    nxy, noff = synth.pack_csr(polys)
    new_inp = synth.AtlasInput(nxy, noff, inp0.atlas_w, inp0.atlas_h, inp0.padding, inp0.quality)
    sxy, soff = synth.pack_csr([donor.chart(j) for j in range(len(idx))])
    tr = ctx.repack(aid0, idx, sxy, soff, inp0.n)
    while tr not in got:
        for ticket, aid, status, batch, lat, out in ctx.poll(wait=True):
            assert status == tabi.TABI_OK
            got[ticket] = out
    st = ctx.stats()
    ctx.close()
    _say("mixed-setting serving stats", st)
    from types import SimpleNamespace
    for t, aid, inp in reqs + [(tr, aid0, new_inp)]:
        xy, ori, sc = got[t]
        r = SimpleNamespace(rid=t, inp=inp, result=(xy, ori, float(sc[0])))
        _same(r, _alone(r))
