"""Serving workload and driver over the library's serving context.

Requests (new atlases, or re-packs of a resident atlas with some charts
replaced) arrive over time as a Poisson trace.  The library's serving
context (tabi_ctx, C ABI) admits them while their device footprint fits its
memory budget and a launch slot (stream) is free, merges every admitted
request into one batched launch on that slot, and keeps going: batches on
different slots overlap on the GPU, and requests that arrive meanwhile join
the next batch.  Per-chart proxy records stay resident on the device per
atlas, so a re-pack recomputes only the replaced charts' records.

Latency = completion of the request's batch on the GPU (HIP event) - arrival.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque

import numpy as np

from . import synth


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float              # seconds since trace start
    atlas_id: int               # resident atlas this request creates or updates
    inp: synth.AtlasInput       # the full chart set to pack
    replaced: np.ndarray | None = None   # for re-packs: replaced chart indices
    done: float = -1.0
    result: tuple | None = None  # (xy[n,2], orient[n], scale) on the host
    t_sub: float = -1.0          # when it was (last) submitted, since trace start


def make_trace(rate=2000.0, seconds=1.0, seed=5000, pool_size=24, repack_frac=0.2,
               replace_frac=0.05, nmin=32, nmax=20000, sides=(1024, 2048, 4096), quality=2,
               padding=2):
    """Poisson arrivals; new atlases drawn from a pool of pre-generated chart
    sets (chart counts log-uniform in [nmin, nmax], the 2,000-chart recipe);
    repack_frac of the requests re-pack a resident atlas with replace_frac of
    its charts replaced by fresh charts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mix = synth.CONFIGS["mixed2k"]["mix"]
    pool = []
    for i in range(pool_size):
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        side = int(rng.choice(sides))
        pool.append(synth.make_custom(n, side, side, padding, quality, 1.2, 1.2, mix,
                                      seed * 100 + i, fast=True))
    spare = synth.generate_charts_fast(2000, 1024, 1024, 1.2, 1.2 * 2000 / 3000, mix,
                                       seed * 100 + 99)
    reqs, t, rid, resident = [], 0.0, 0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > seconds:
            break
        if resident and rng.uniform() < repack_frac:
            aid = int(rng.choice(resident))
            base = _latest(reqs, aid)
            m = max(1, int(round(replace_frac * base.n)))
            idx = np.sort(rng.choice(base.n, size=min(m, base.n), replace=False)).astype(np.int32)
            polys = [base.chart(c) for c in range(base.n)]
            for c in idx:
                polys[c] = spare[int(rng.integers(0, len(spare)))]
            xy, off = synth.pack_csr(polys)
            inp = synth.AtlasInput(xy, off, base.atlas_w, base.atlas_h, padding, quality)
            reqs.append(Request(rid, t, aid, inp, idx))
        else:
            inp = pool[int(rng.integers(0, pool_size))]
            reqs.append(Request(rid, t, rid, inp))
            resident.append(rid)
        rid += 1
    return reqs


def _latest(reqs, aid):
    for r in reversed(reqs):
        if r.atlas_id == aid:
            return r.inp
    raise KeyError(aid)


class Server:
    """Serving loop over the library's serving context (tabi_ctx): each
    request is submitted at its arrival time (tabi_submit for a new atlas,
    tabi_repack with the replaced charts for a re-pack of a resident one) and
    completions are polled.  The context batches what is queued into free
    launch slots, admits by device-memory footprint and keeps every atlas's
    proxy records resident; a re-pack whose atlas was evicted under the budget
    is submitted again as a new atlas with its whole chart set."""

    def __init__(self, quality=2, padding=2, hbm_budget=16 << 30, streams=4, max_batch=256,
                 staging_bytes=64 << 20, device="cuda"):
        import paper_2602_07782_amd as tabi
        self.tabi = tabi
        self.ctx = tabi.ServeContext(quality, padding, streams, max_batch, hbm_budget,
                                     staging_bytes)
        self.ids = {}        # trace atlas id -> context atlas id
        self.by_ticket = {}  # ticket -> request
        self.resubmitted = 0

    def _submit(self, r, now):
        r.t_sub = now
        if r.replaced is not None and r.atlas_id in self.ids:
            sub = [r.inp.chart(int(c)) for c in r.replaced]
            sxy, soff = synth.pack_csr(sub)
            aid = self.ids[r.atlas_id]
            t = self.ctx.repack(aid, r.replaced, sxy, soff, r.inp.n)
        else:
            aid, t = self.ctx.submit(r.inp.xy, r.inp.offsets, r.inp.atlas_w, r.inp.atlas_h)
        self.ids[r.atlas_id] = aid
        self.by_ticket[t] = r

    def _collect(self, wait, now):
        got = self.ctx.poll(wait)
        for ticket, _aid, status, _batch, lat_ms, out in got:
            r = self.by_ticket.pop(ticket)
            if status == self.tabi.TABI_ENOTRESIDENT:
                self.ids.pop(r.atlas_id, None)
                self.resubmitted += 1
                self._submit(r, now)
                continue
            if status != self.tabi.TABI_OK:
                raise self.tabi.TabiError(status, f"request {r.rid}")
            r.result = (out[0], out[1], float(out[2][0]))
            r.done = r.t_sub + lat_ms / 1000.0
        return bool(got)

    def run(self, requests, realtime=True):
        """Serve a trace; returns seconds from the trace start to the last
        completion (arrival times are relative to the start)."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        start = time.perf_counter()
        while pending or self.by_ticket:
            now = time.perf_counter() - start
            while pending and (pending[0].arrival <= now or not realtime):
                self._submit(pending.popleft(), time.perf_counter() - start)
            if self._collect(False, time.perf_counter() - start):
                continue
            if pending and realtime:
                time.sleep(max(0.0, min(0.0005, pending[0].arrival - now)))
            elif self.by_ticket:
                self._collect(True, time.perf_counter() - start)
        return max(r.done for r in requests)

    def stats(self):
        d = self.ctx.stats()
        d["resubmitted"] = self.resubmitted
        return d

    def close(self):
        self.ctx.close()


def serve_plain(requests, quality=2, padding=2, device="cuda", realtime=True):
    """The same trace through single tabi_pack calls, one at a time."""
    import torch
    import paper_2602_07782_amd as tabi
    reqs = sorted(requests, key=lambda r: r.arrival)
    torch.cuda.synchronize()
    start = time.perf_counter()
    for r in reqs:
        if realtime:
            now = time.perf_counter() - start
            if r.arrival > now:
                time.sleep(r.arrival - now)
        xy, ori, sc = tabi.pack(r.inp.xy, r.inp.offsets, r.inp.atlas_w, r.inp.atlas_h, padding,
                                quality, device=device)
        torch.cuda.synchronize()
        r.done = time.perf_counter() - start
        r.result = (xy.cpu().numpy(), ori.cpu().numpy(), float(sc.cpu().numpy()[0]))
    return max(r.done for r in reqs)


def latency_stats(requests):
    lat = np.array([r.done - r.arrival for r in requests]) * 1000.0
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean())}
