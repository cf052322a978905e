"""Continuous-batching pack server over the C ABI.

Requests (new atlases, or re-packs of a resident atlas with some charts
replaced) arrive over time.  The server admits them while their device
footprint fits an HBM budget and a launch slot (stream) is free, merges every
admitted request into one batched launch (tabi_pack_many_records) on that
stream, and keeps going: batches on different streams overlap on the GPU,
and requests that arrive meanwhile join the next batch.  Per-chart proxy
records stay resident on the device per atlas, so a re-pack recomputes only
the replaced charts' records (tabi_prep_records + tabi_splice_records).

Completion times come from HIP events, latency = completion - arrival.
All packing work runs in the library's kernels; PyTorch supplies device
memory, streams and events.
"""
from __future__ import annotations

import dataclasses
import time
from collections import OrderedDict, deque

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
    def __init__(self, quality=2, padding=2, hbm_budget=16 << 30, streams=4, max_batch=256,
                 device="cuda"):
        import torch
        import paper_2602_07782_amd as tabi
        self.torch, self.tabi = torch, tabi
        self.dev = torch.device(device)
        self.q, self.p = quality, padding
        self.budget = int(hbm_budget)
        self.max_batch = max_batch
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        self.free_streams = deque(range(streams))
        self.inflight = []          # (stream idx, event, requests, outputs, bytes)
        self.used = 0
        self.resident = OrderedDict()  # atlas_id -> device records (LRU order)
        self.resident_event = {}       # atlas_id -> event of the batch that wrote them
        self.resident_bytes = 0
        self.rb = tabi.record_bytes()
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_wall = 0.0

    # -- footprint ---------------------------------------------------------
    def footprint(self, r):
        n = r.inp.n
        side = max(r.inp.atlas_w, r.inp.atlas_h)
        ws = self.tabi.lib().tabi_pack_many_workspace_bytes(1, n, n, side, self.p, self.q)
        return int(ws) + 2 * n * self.rb + 16 * n

    def _evict_for(self, need):
        while self.resident and self.used + self.resident_bytes + need > self.budget:
            aid, rec = self.resident.popitem(last=False)
            self.resident_event.pop(aid, None)
            self.resident_bytes -= rec.numel()

    # -- one batched launch --------------------------------------------------
    def _launch(self, batch):
        torch, tabi = self.torch, self.tabi
        si = self.free_streams.popleft()
        s = self.streams[si]
        nbytes = sum(self.footprint(r) for r in batch)
        with torch.cuda.stream(s):
            recs, wh, aoff = [], [], [0]
            for r in batch:
                inp = r.inp
                base = self.resident.get(r.atlas_id) if r.replaced is not None else None
                if base is not None:
                    ev0 = self.resident_event.get(r.atlas_id)
                    if ev0 is not None:
                        s.wait_event(ev0)  # records written by a batch on another stream
                    base.record_stream(s)
                    rec = base.clone()
                    sub = [inp.chart(int(c)) for c in r.replaced]
                    sxy, soff = synth.pack_csr(sub)
                    new = tabi.prep_records(sxy, soff, np.array([0, len(sub)], np.int32), self.q,
                                            stream=s, device=self.dev)
                    tabi.splice_records(rec, r.replaced, new, stream=s)
                else:
                    rec = tabi.prep_records(inp.xy, inp.offsets, np.array([0, inp.n], np.int32),
                                            self.q, stream=s, device=self.dev)
                self._keep(r.atlas_id, rec)
                recs.append(rec)
                wh += [inp.atlas_w, inp.atlas_h]
                aoff.append(aoff[-1] + inp.n)
            allrec = torch.cat(recs) if len(recs) > 1 else recs[0]
            N = aoff[-1]
            aoff_t = torch.tensor(aoff, dtype=torch.int32).to(self.dev, non_blocking=True)
            wh_t = torch.tensor(wh, dtype=torch.int32).to(self.dev, non_blocking=True)
            out_xy = torch.empty((N, 2), dtype=torch.int32, device=self.dev)
            out_or = torch.empty(N, dtype=torch.uint8, device=self.dev)
            out_sc = torch.empty(len(batch), dtype=torch.float32, device=self.dev)
            tabi.pack_many_records(allrec, aoff_t, wh_t, max(r.inp.n for r in batch),
                                   max(max(r.inp.atlas_w, r.inp.atlas_h) for r in batch), self.p,
                                   self.q, out_xy, out_or, out_sc, stream=s)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        for r in batch:
            self.resident_event[r.atlas_id] = ev
        self.used += nbytes
        self.inflight.append((si, ev, batch, (out_xy, out_or, out_sc, aoff, allrec), nbytes))

    def _keep(self, aid, rec):
        old = self.resident.pop(aid, None)
        if old is not None:
            self.resident_bytes -= old.numel()
        self.resident[aid] = rec
        self.resident_bytes += rec.numel()

    def _poll(self, block=False):
        done_any = False
        keep = []
        for item in self.inflight:
            si, ev, batch, outs, nbytes = item
            if block or ev.query():
                ev.synchronize()
                t_done = self.t0_wall + self.t0_event.elapsed_time(ev) / 1000.0
                out_xy, out_or, out_sc, aoff, _ = outs
                xy, ori, sc = out_xy.cpu().numpy(), out_or.cpu().numpy(), out_sc.cpu().numpy()
                for j, r in enumerate(batch):
                    a, b = aoff[j], aoff[j + 1]
                    r.result = (xy[a:b], ori[a:b], float(sc[j]))
                    r.done = t_done
                self.used -= nbytes
                self.free_streams.append(si)
                done_any = True
                block = False
            else:
                keep.append(item)
        self.inflight = keep
        return done_any

    def run(self, requests, realtime=True):
        """Serve a trace; returns wall seconds from the first arrival to the
        last completion."""
        torch = self.torch
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue = deque()
        torch.cuda.synchronize()
        self.t0_event.record(torch.cuda.current_stream())
        self.t0_wall = time.perf_counter()
        start = self.t0_wall
        while pending or queue or self.inflight:
            now = time.perf_counter() - start
            while pending and (pending[0].arrival <= now or not realtime):
                queue.append(pending.popleft())
            progressed = self._poll()
            launched = False
            while queue and self.free_streams:
                # admit in arrival order while the footprint fits the budget;
                # a request larger than the budget runs alone on an idle GPU
                batch, need = [], 0
                while queue and len(batch) < self.max_batch:
                    f = self.footprint(queue[0])
                    alone = not batch and not self.inflight
                    if self.used + need + f > self.budget and not alone:
                        break
                    self._evict_for(need + f)
                    need += f
                    batch.append(queue.popleft())
                if not batch:
                    break
                self._launch(batch)
                launched = True
            if not launched and not progressed:
                if self.inflight and not pending and not queue:
                    self._poll(block=True)       # nothing else to do: wait for the GPU
                elif self.inflight:
                    time.sleep(0.0002)
                elif pending and realtime:
                    time.sleep(max(0.0, min(0.001, pending[0].arrival - now)))
        # arrivals are relative to start; completions are wall times
        for r in requests:
            r.done -= start
        return max(r.done for r in requests)


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
