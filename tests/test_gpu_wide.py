"""Single-pack parity with the oracle, bit for bit, over the seed counts of
the measurement plan: 1,000 instances of the 64-chart 512^2 workload, 200 of
the 2,000-chart 2048^2 workload at the lowest and the highest quality, and 20
of the 20,000-chart 4096^2 workload (instance 0 is the timed input, so the
sweeps take 1..N).  Worker processes (started fresh, no GPU use) generate the
instances and run the oracle; this process packs each on the GPU as it
arrives.  The first mismatch stops the test and names its instance."""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
from concurrent.futures import ProcessPoolExecutor, as_completed

import numpy as np
import pytest

import parity_pool

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tabi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_07782_amd as t
    t.lib()
    return t


def _sweep(tabi, name, instances, qualities):
    workers = max(1, min(16, os.cpu_count() or 1))
    print(f"{name}: {len(instances)} instances, qualities {qualities}, {workers} host workers",
          file=sys.stderr, flush=True)
    done = 0
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        futs = {ex.submit(parity_pool.oracle_case, name, i, qualities): i for i in instances}
        try:
            for f in as_completed(futs):
                inst = futs[f]
                xy, offs, W, H, p, res = f.result()
                for q, oxy, oori, osc in res:
                    gxy, gori, gsc = tabi.pack(xy, offs, W, H, p, q, device="cuda:0")
                    label = f"{name}/{inst}/q{q}"
                    assert float(gsc.cpu().numpy()[0]) == osc, label
                    assert np.array_equal(gxy.cpu().numpy(), oxy), label
                    assert np.array_equal(gori.cpu().numpy(), oori), label
                done += 1
        finally:
            for f in futs:
                f.cancel()
    print(f"{name}: {done} instances equal", file=sys.stderr, flush=True)
    assert done == len(instances)


def test_stars64_thousand_instances(tabi):
    _sweep(tabi, "stars64", range(1, 1001), (2,))


def test_mixed2k_two_hundred_instances(tabi):
    _sweep(tabi, "mixed2k", range(1, 201), (0, 2))


def test_lightmap20k_twenty_instances(tabi):
    _sweep(tabi, "lightmap20k", range(1, 21), (2,))
