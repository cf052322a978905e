"""Serving path on the GPU: continuous batching over several streams with
resident proxy records.  Every request's result in the mix equals the same
request packed alone (tolerance 0), and the oracle for a sample."""
from __future__ import annotations

import numpy as np
import pytest

# Skipped: two full-trace runs of this serving path (four streams, thousands
# of batches) faulted the GPU and no cause has been found in the kernels or
# in the server; these smaller runs stay off the GPU until one is.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="multi-stream serving faulted the GPU on full traces; "
                                      "cause not yet found")]


@pytest.fixture(scope="module")
def served():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_07782_amd import serve
    reqs = serve.make_trace(rate=2000.0, seconds=0.06, seed=77, pool_size=8, nmin=16, nmax=1500,
                            sides=(256, 512, 1024))
    srv = serve.Server(streams=3, max_batch=16)
    srv.run(reqs)
    return reqs


def test_trace_has_repacks(served):
    assert any(r.replaced is not None for r in served)
    assert all(r.done >= r.arrival for r in served)


def test_served_equals_alone(served):
    import paper_2602_07782_amd as tabi
    for r in served:
        xy, ori, sc = tabi.pack(r.inp.xy, r.inp.offsets, r.inp.atlas_w, r.inp.atlas_h,
                                r.inp.padding, r.inp.quality)
        assert float(sc.cpu().numpy()[0]) == r.result[2], r.rid
        assert np.array_equal(xy.cpu().numpy(), r.result[0]), r.rid
        assert np.array_equal(ori.cpu().numpy(), r.result[1]), r.rid


def test_served_sample_equals_oracle(served, orc):
    picks = [r for r in served if r.replaced is not None][:3] + served[:3]
    for r in picks:
        oxy, oori, osc, ok = orc.pack(r.inp)
        assert r.result[2] == osc
        assert np.array_equal(r.result[0], oxy)
        assert np.array_equal(r.result[1], oori)


def test_tight_budget_gives_same_results(served):
    """A budget that admits one request at a time changes batching, not results."""
    from paper_2602_07782_amd import serve
    import copy
    reqs = [copy.copy(r) for r in served[:20]]
    for r in reqs:
        r.done, r.result = -1.0, None
    srv = serve.Server(streams=2, max_batch=4, hbm_budget=1)
    srv.run(reqs)
    for a, b in zip(reqs, served[:20]):
        assert a.result[2] == b.result[2]
        assert np.array_equal(a.result[0], b.result[0])
        assert np.array_equal(a.result[1], b.result[1])
