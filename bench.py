#!/usr/bin/env python3
"""Benchmark of the MI355X TABI packer.

One step = one tabi_pack call over the 2,000-chart workload (70% star
polygons with 8-64 vertices, 30% concave L/U shapes, log-normal areas with
sigma 1.2 summing to 120% of the atlas) into a 2048x2048 atlas with padding 2,
at the high quality preset (10 local AABBs).  Inputs are resident in HBM
before the timed region; every step runs the whole hot path (proxies, sort,
scale bound, per-scale set-up, neighbour pairs, fold-and-push for every
candidate scale, selection).

Prints one JSON line (rank 0, one GPU).
"""
from __future__ import annotations

import argparse
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per atlas pack (p50/p99) and atlases/sec batched vs plain, bit-exact vs oracle"
PEAK_HBM_GBS = 8000.0


def percentile(v, q):
    v = sorted(v)
    if not v:
        return float("nan")
    i = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[i]


def cpu_baseline(inp, seconds):
    """The oracle, as it stands, on one host core over a bounded sample."""
    import oracle
    t0 = time.perf_counter()
    reps, out = 0, None
    while True:
        out = oracle.pack(inp)
        reps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return dt * 1000.0 / reps, reps, out


def batched_leg(tabi, torch, count=256, reps=3, cpu_seconds=15.0):
    """The batch workload: `count` atlases (sides 512/1024/2048, 50-5,000
    charts each, 2,000-chart recipe) in one tabi_pack_many, captured in a HIP
    graph and replayed, against the same atlases through tabi_pack back to
    back on one stream."""
    import numpy as np
    from paper_2602_07782_amd import synth
    inputs = synth.make_batch(count)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    plain_in = [(torch.from_numpy(np.ascontiguousarray(i.xy, np.int32)).to(dev),
                 torch.from_numpy(np.ascontiguousarray(i.offsets, np.int32)).to(dev)) for i in inputs]
    plain_out = [(torch.empty((i.n, 2), dtype=torch.int32, device=dev),
                  torch.empty(i.n, dtype=torch.uint8, device=dev),
                  torch.empty(1, dtype=torch.float32, device=dev)) for i in inputs]

    def plain_pass():
        for inp, (xy, off), (oxy, oor, osc) in zip(inputs, plain_in, plain_out):
            tabi.pack_into(xy, off, inp.n, inp.atlas_w, inp.atlas_h, inp.padding, inp.quality,
                           oxy, oor, osc, stream=stream)
    plain_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_pass()
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0

    batch = tabi.Batch(inputs)
    s = torch.cuda.Stream()
    s.wait_stream(stream)
    # autotune the batched shape on this batch (outside the timed region)
    tuned = batch.tune(stream=s, reps=1)
    with torch.cuda.stream(s):
        batch.run(stream=s, use_workspace=True)
    stream.wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        batch.run(stream=s, use_workspace=True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        g.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    batched_s = ev0.elapsed_time(ev1) / 1000.0 / reps
    # per-stage split of one more (eager) batch, outside the timed region
    tabi.timing_reset()
    tabi.timing_enable(True)
    with torch.cuda.stream(s):
        batch.run(stream=s, use_workspace=True)
    torch.cuda.synchronize()
    tabi.timing_enable(False)
    stages = {k: round(v[0], 3) for k, v in tabi.timing_read().items()}
    same, c0 = True, 0
    bsc = batch.out_scale.cpu().numpy()
    for ai, (inp, (oxy, oor, osc)) in enumerate(zip(inputs, plain_out)):
        n = inp.n
        same &= bool(torch.equal(batch.out_xy[c0:c0 + n], oxy)) and \
            bool(torch.equal(batch.out_orient[c0:c0 + n], oor)) and \
            float(bsc[ai]) == float(osc.cpu().numpy()[0])
        c0 += n
    alg = sum(atlas_algorithmic_bytes(inp, int(round(float(bsc[a]) * 64)))
              for a, inp in enumerate(inputs))
    gbs = alg / batched_s / 1e9
    out = {"atlases": count, "charts": int(sum(i.n for i in inputs)),
            "atlases_per_s_batched": round(count / batched_s, 2),
            "atlases_per_s_plain": round(count / plain_s, 2),
            "speedup_vs_plain": round(plain_s / batched_s, 2),
            "ms_per_batch": round(batched_s * 1000.0, 3), "hip_graph": True,
            "stage_ms_per_batch": stages,
            "autotuned_shape": {"first_round_slots": tuned["shape"][0],
                                "rounds_at_first": tuned["shape"][1],
                                "max_round_slots": tuned["shape"][2],
                                "pack_threads": tuned["shape"][3],
                                "pack_lds_cap": tuned["shape"][4],
                                "candidate_ms": tuned["ms"]},
            "hbm": {"algorithmic_bytes_per_batch": alg, "achieved_GBps": round(gbs, 2),
                    "peak_GBps": PEAK_HBM_GBS, "frac": round(gbs / PEAK_HBM_GBS, 6)},
            "bitexact_vs_plain": bool(same)}
    if cpu_seconds > 0:
        out["cpu_baseline"] = batched_cpu_baseline(inputs, cpu_seconds)
    return out


def host_cores():
    """Host cores this process may run on, capped at the 16 a one-GPU share
    of the box holds."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def batched_cpu_baseline(inputs, seconds):
    """The oracle over the batch's atlases on all host cores (one atlas per
    task, a thread per core; the oracle's C code runs outside the Python
    lock), for about `seconds` of wall time: atlases per second."""
    import concurrent.futures as cf
    import oracle
    oracle.build()
    cores = host_cores()
    t0 = time.perf_counter()
    done = 0
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        it = iter(inputs)
        running = set()
        for _ in range(cores):
            inp = next(it, None)
            if inp is not None:
                running.add(ex.submit(oracle.pack, inp))
        while running:
            fin, running = cf.wait(running, return_when=cf.FIRST_COMPLETED)
            done += len(fin)
            if time.perf_counter() - t0 < seconds:
                for _ in fin:
                    inp = next(it, None)
                    if inp is not None:
                        running.add(ex.submit(oracle.pack, inp))
    wall = time.perf_counter() - t0
    return {"value": round(done / wall, 3), "unit": "atlases/s", "cores": cores,
            "kind": "oracle", "sample": f"the first {done} atlases of the same batch, "
                                        f"one per thread, {wall:.1f} s wall"}


def ablation_leg(tabi, torch, reps=10):
    """The paper's ablations on synthetic sets (Sec. 5 ablation table; App. D
    local-AABB count and t_opt tables): per setting, the mean over inputs of
    the p50 time of tabi_pack_method and of the L2 stretch 64/k."""
    import numpy as np
    from paper_2602_07782_amd import synth
    inputs = [synth.make_input("mixed2k", i) for i in range(4)]
    inputs += [synth.make_input("lightmap20k", i) for i in range(2)]
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    dev_in = [(torch.from_numpy(np.ascontiguousarray(i.xy, np.int32)).to(dev),
               torch.from_numpy(np.ascontiguousarray(i.offsets, np.int32)).to(dev))
              for i in inputs]
    settings = {"full": (10, -1, 0), "tight_only": (10, -1, 1), "balanced_only": (10, -1, 2),
                "K2": (2, -1, 0), "K5": (5, -1, 0), "topt5": (10, 5, 0), "topt2": (10, 2, 0),
                "topt1": (10, 1, 0), "topt0": (10, 0, 0)}
    out = {"inputs": "mixed2k instances 0-3 (2,000 charts, 2048^2) and lightmap20k "
                     "instances 0-1 (20,000 charts, 4096^2)"}
    for name, (K, t, v) in settings.items():
        ms, stretch = [], []
        for inp, (xy, off) in zip(inputs, dev_in):
            res = None
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps)]
            tabi.pack_method(xy, off, inp.atlas_w, inp.atlas_h, inp.padding, K, t, v, stream=st)
            for a, b in ev:
                a.record(st)
                res = tabi.pack_method(xy, off, inp.atlas_w, inp.atlas_h, inp.padding, K, t, v,
                                       stream=st)
                b.record(st)
            torch.cuda.synchronize()
            ms.append(percentile([a.elapsed_time(b) for a, b in ev], 50))
            k = int(round(float(res[2].cpu().numpy()[0]) * 64))
            stretch.append(64.0 / k if k > 0 else float("inf"))
        out[name] = {"mean_ms": round(float(np.mean(ms)), 4),
                     "mean_stretch": round(float(np.mean(stretch)), 4)}
    return out


def config_legs(tabi, torch, cpu):
    """The other single-pack configurations: the 64-chart 512^2 workload,
    the 2,000-chart 2048^2 workload at low quality, the 20,000-chart 4096^2
    workload and a TSS-like frame (4,000 clipped screen-space patches into
    1024^2); p50 / p99 of tabi_pack (HIP events per call) and the oracle on
    one host core (one pack each)."""
    import numpy as np
    from paper_2602_07782_amd import synth
    import oracle
    legs = {}
    for name, q, steps in (("stars64", 2, 100), ("mixed2k", 0, 100), ("lightmap20k", 2, 30),
                           ("tss4k", 2, 100)):
        base = synth.make_tss(0) if name == "tss4k" else synth.make_input(name, 0)
        inp = synth.AtlasInput(base.xy, base.offsets, base.atlas_w, base.atlas_h, base.padding, q)
        dev = torch.device("cuda:0")
        xy = torch.from_numpy(np.ascontiguousarray(inp.xy, np.int32)).to(dev)
        off = torch.from_numpy(np.ascontiguousarray(inp.offsets, np.int32)).to(dev)
        oxy = torch.empty((inp.n, 2), dtype=torch.int32, device=dev)
        oor = torch.empty(inp.n, dtype=torch.uint8, device=dev)
        osc = torch.empty(1, dtype=torch.float32, device=dev)
        st = torch.cuda.current_stream()
        for _ in range(5):
            tabi.pack_into(xy, off, inp.n, inp.atlas_w, inp.atlas_h, inp.padding, q, oxy, oor,
                           osc, stream=st)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(st)
            tabi.pack_into(xy, off, inp.n, inp.atlas_w, inp.atlas_h, inp.padding, q, oxy, oor,
                           osc, stream=st)
            b.record(st)
        torch.cuda.synchronize()
        per = [a.elapsed_time(b) for a, b in ev]
        gsc = float(osc.cpu().numpy()[0])
        leg = {"charts": inp.n, "atlas": [inp.atlas_w, inp.atlas_h], "padding": inp.padding,
               "quality": q, "p50_ms": round(percentile(per, 50), 4),
               "p99_ms": round(percentile(per, 99), 4), "scale": gsc}
        if cpu:
            t0 = time.perf_counter()
            e_xy, e_or, e_sc, _ = oracle.pack(inp)
            leg["cpu_baseline"] = {"value": round((time.perf_counter() - t0) * 1000.0, 2),
                                   "unit": "ms per atlas pack", "cores": 1, "kind": "oracle",
                                   "sample": "one pack of the same input"}
            leg["bitexact_vs_oracle"] = bool(e_sc == gsc and
                                             np.array_equal(e_xy, oxy.cpu().numpy()) and
                                             np.array_equal(e_or, oor.cpu().numpy()))
        legs[f"{name}_q{q}"] = leg
    return legs


def variants_leg(tabi, torch, reps=20):
    """Input-side and tail variants, p50 of HIP-event times per call: the
    2,000-chart workload pre-rotated to tight boxes (tabi_pack_prerotate,
    against tabi_pack on the same charts as given); the hybrid tail
    (tabi_pack_hybrid) on the 20,000-chart workload at the paper's t_opt and
    on the 2,000-chart workload at t_opt 5 %, against tabi_pack_method with the
    same knobs (exact greedy tail), with the area-weighted mean L2 stretch
    (64 / k per chart); and 2,000 mesh charts of several boundary loops
    (tabi_pack_loops)."""
    import numpy as np
    from paper_2602_07782_amd import synth
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()

    def timed(fn):
        out = fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(st)
            out = fn()
            b.record(st)
        torch.cuda.synchronize()
        return round(percentile([a.elapsed_time(b) for a, b in ev], 50), 4), out

    def area2(inp):
        out = []
        for c in range(inp.n):
            P = inp.chart(c).astype(np.int64)
            x, y = P[:, 0], P[:, 1]
            out.append(abs(int(np.dot(x, np.roll(y, -1)) - np.dot(np.roll(x, -1), y))))
        return np.array(out, np.float64)

    res = {}
    inp = synth.make_input("mixed2k", 0)
    xy = torch.from_numpy(np.ascontiguousarray(inp.xy, np.int32)).to(dev)
    off = torch.from_numpy(np.ascontiguousarray(inp.offsets, np.int32)).to(dev)
    ms, out = timed(lambda: tabi.pack_prerotate(xy, off, inp.atlas_w, inp.atlas_h, inp.padding, 2,
                                                stream=st))
    ms0, out0 = timed(lambda: tabi.pack(xy, off, inp.atlas_w, inp.atlas_h, inp.padding, 2,
                                        stream=st))
    res["prerotate_mixed2k_q2"] = {"p50_ms": ms, "scale": float(out[4].cpu()[0]),
                                   "plain_p50_ms": ms0, "plain_scale": float(out0[2].cpu()[0])}
    for name, topt in (("lightmap20k", -1), ("mixed2k", 5)):
        inp = synth.make_input(name, 0)
        xy = torch.from_numpy(np.ascontiguousarray(inp.xy, np.int32)).to(dev)
        off = torch.from_numpy(np.ascontiguousarray(inp.offsets, np.int32)).to(dev)
        ms, out = timed(lambda: tabi.pack_hybrid(xy, off, inp.atlas_w, inp.atlas_h, inp.padding,
                                                 10, topt, stream=st))
        ms0, out0 = timed(lambda: tabi.pack_method(xy, off, inp.atlas_w, inp.atlas_h,
                                                   inp.padding, 10, topt, 0, stream=st))
        w = area2(inp)
        ks = out[2].cpu().numpy().astype(np.float64)
        k0 = float(out0[2].cpu()[0])
        res[f"hybrid_{name}_topt{topt}"] = {
            "p50_ms": ms, "head_scale": float(out[3].cpu()[0]),
            "tail_charts": int((ks < float(out[3].cpu()[0])).sum()),
            "area_weighted_stretch": round(float((w / ks).sum() / w.sum()), 4) if ks.min() > 0
            else None,
            "greedy_tail_p50_ms": ms0,
            "greedy_tail_stretch": round(1.0 / k0, 4) if k0 > 0 else None}
    L, _ = synth.make_loops(2000, 2048, 2048, 2, 2, 7100)
    lxy = torch.from_numpy(np.ascontiguousarray(L.xy, np.int32)).to(dev)
    llo = torch.from_numpy(np.ascontiguousarray(L.loop_offsets, np.int32)).to(dev)
    lcl = torch.from_numpy(np.ascontiguousarray(L.chart_loops, np.int32)).to(dev)
    ms, out = timed(lambda: tabi.pack_loops(lxy, llo, lcl, L.atlas_w, L.atlas_h, L.padding,
                                            L.quality, stream=st))
    res["loops_2000"] = {"p50_ms": ms, "scale": float(out[2].cpu()[0]),
                         "loops": int(len(L.loop_offsets) - 1)}
    return res


def atlas_algorithmic_bytes(inp, kstar):
    """Bytes the method must move for one atlas pack: vertices and offsets
    read (8 V + 4 (n + 1)), per-chart proxies written and read
    (n (16 K + 80)), for every evaluated scale the grown profiles written
    once and read once (8 per grown column and row: two int16 bounds each
    way), and the outputs (9 n + 4).  The evaluated scales are those from
    the largest candidate down to the chosen one (all candidates when none
    fits).  Chart extents come from the input polygons (host numpy)."""
    import numpy as np
    n = inp.n
    if n == 0:
        return 4
    K = {0: 2, 1: 5, 2: 10}[inp.quality]
    xy = np.asarray(inp.xy, np.int64).reshape(-1)
    xs, ys = xy[0::2], xy[1::2]
    off = np.asarray(inp.offsets, np.int64)
    starts = off[:-1]
    ex = np.maximum.reduceat(xs, starts) - np.minimum.reduceat(xs, starts)
    ey = np.maximum.reduceat(ys, starts) - np.minimum.reduceat(ys, starts)
    W, H = np.minimum(ex, ey), np.maximum(ex, ey)
    x1 = np.roll(xs, -1)
    y1 = np.roll(ys, -1)
    last = off[1:] - 1
    x1[last], y1[last] = xs[starts], ys[starts]
    cross = xs * y1 - x1 * ys
    area2 = np.abs(np.add.reduceat(cross, starts)).astype(object).sum()
    ktop = 0
    for k in range(1, 65):  # area bound and the tallest / widest chart
        if (area2 * k * k <= (1 << 29) * inp.atlas_w * inp.atlas_h and
                -(-k * int(W.max()) // 16384) <= inp.atlas_w and
                -(-k * int(H.max()) // 16384) <= inp.atlas_h):
            ktop = k
    klo = kstar if kstar > 0 else 1
    prof = 0
    for k in range(klo, ktop + 1):
        wk, hk = -(-k * W // 16384) + inp.padding, -(-k * H // 16384) + inp.padding
        prof += 8 * int((wk + hk).sum())
    V = int(off[-1])
    return 8 * V + 4 * (n + 1) + n * (16 * K + 80) + prof + 9 * n + 4


def served_leg(seconds=1.0, rate=2000.0):
    """Poisson trace served by the library's serving context (continuous
    batching, resident proxies) vs one tabi_pack at a time."""
    import copy
    import numpy as np
    from paper_2602_07782_amd import serve
    reqs = serve.make_trace(rate=rate, seconds=seconds)
    plain = [copy.copy(r) for r in reqs]
    srv = serve.Server()
    wall = srv.run(reqs)
    stats = srv.stats()
    srv.close()
    st = serve.latency_stats(reqs)
    pwall = serve.serve_plain(plain)
    pst = serve.latency_stats(plain)
    same = all(a.result[2] == b.result[2] and np.array_equal(a.result[0], b.result[0]) and
               np.array_equal(a.result[1], b.result[1]) for a, b in zip(reqs, plain))
    alg = sum(atlas_algorithmic_bytes(r.inp, int(round(r.result[2] * 64))) for r in reqs)
    # capacity: the same requests all waiting at once (no arrival pacing), so
    # the rate is what each path can sustain rather than the trace's 2,000/s
    sat = [copy.copy(r) for r in reqs]
    splain = [copy.copy(r) for r in reqs]
    for r in sat + splain:
        r.done, r.result = -1.0, None
    srv = serve.Server()
    swall = srv.run(sat, realtime=False)
    srv.close()
    spwall = serve.serve_plain(splain, realtime=False)
    same &= all(a.result[2] == b.result[2] and np.array_equal(a.result[0], b.result[0])
                for a, b in zip(sat, plain))
    gbs = alg / swall / 1e9
    return {"requests": len(reqs), "rate_per_s": rate,
            "repacks": int(sum(r.replaced is not None for r in reqs)),
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
            "atlases_per_s": round(len(reqs) / wall, 2),
            "plain_p50_ms": round(pst["p50_ms"], 3), "plain_p99_ms": round(pst["p99_ms"], 3),
            "plain_atlases_per_s": round(len(plain) / pwall, 2),
            "speedup_vs_plain": round(pwall / wall, 2),
            "capacity_atlases_per_s": round(len(sat) / swall, 2),
            "plain_capacity_atlases_per_s": round(len(splain) / spwall, 2),
            "capacity_speedup_vs_plain": round(spwall / swall, 2),
            "capacity_hbm": {"algorithmic_bytes": alg, "achieved_GBps": round(gbs, 2),
                             "peak_GBps": PEAK_HBM_GBS, "frac": round(gbs / PEAK_HBM_GBS, 6)},
            "context": {k: stats[k] for k in ("launches", "evicted", "resubmitted",
                                               "device_bytes_peak", "peak_in_flight",
                                               "cross_slot_waits")},
            "bitexact_vs_alone": bool(same)}


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "k_pack_mixed2k_traffic.md")


def kernel_sources_sha256():
    """Digest of the HIP sources, and of the build script that holds their
    compiler flags, that the counters were taken from."""
    import hashlib
    pkg = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2602_07782_amd")
    d = os.path.join(pkg, "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    with open(os.path.join(pkg, "build.py"), "rb") as fh:
        h.update(b"build.py")
        h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per fold-and-push launch from the committed FETCH_SIZE /
    WRITE_SIZE summary, or None when the kernels changed since it was taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = dict(re.findall(r"^(sources_sha256|traffic_bytes_per_launch):\s*(\S+)\s*$", text, re.M))
    if vals.get("sources_sha256") != kernel_sources_sha256():
        return None
    try:
        return int(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def pack_algorithmic_bytes(inp, k_top):
    """Algorithmic bytes of one fold-and-push launch over the scales 1..k_top:
    per (chart, scale) the chart's grown column profile, 4 (w_k + p) bytes,
    where w_k = ceil(k W / 16384) is its texel width at scale k/64 and W the
    smaller side of its Q8 bounding box (charts are turned so that H >= W),
    plus 22 bytes of per-chart fields and placement."""
    import numpy as np
    xs, ys = inp.xy[0::2].astype(np.int64), inp.xy[1::2].astype(np.int64)
    starts = inp.offsets[:-1]
    ex = np.maximum.reduceat(xs, starts) - np.minimum.reduceat(xs, starts)
    ey = np.maximum.reduceat(ys, starts) - np.minimum.reduceat(ys, starts)
    wq = np.minimum(ex, ey)
    ks = np.arange(1, k_top + 1, dtype=np.int64)[:, None]
    wk = -(-(ks * wq[None, :]) // 16384)
    units = int(wk.size)
    return int((4 * (wk + inp.padding) + 22).sum()), units


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--quality", type=int, default=2)
    ap.add_argument("--workload", default="mixed2k",
                    choices=["mixed2k", "stars64", "lightmap20k", "tss4k"],
                    help="the single-pack workload of the main leg (the default is the "
                         "headline configuration; the others are for per-workload profiles)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other single-pack configurations")
    ap.add_argument("--phase-clock", action="store_true",
                    help="with the diagnostic library (python -m paper_2602_07782_amd.build "
                         "--phase-clock): the fold-and-push kernel's per-row phase split of the "
                         "main leg's workload, per scale slot, then exit")
    ap.add_argument("--traffic-pass", action="store_true",
                    help="for hardware-counter runs: a few packs, then one plain 256 MiB device "
                         "copy whose byte count calibrates FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path here "
              "(atlases and scales would shard across GPUs without communication)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2602_07782_amd as tabi
    from paper_2602_07782_amd import synth

    if args.phase_clock:
        from paper_2602_07782_amd import build as tabi_build
        if not os.path.exists(tabi_build.OUT_PHASE):
            print(f"{tabi_build.OUT_PHASE} is missing: build it with "
                  "`python -m paper_2602_07782_amd.build --phase-clock`", file=sys.stderr)
            sys.exit(2)
        tabi.LIB_PATH = tabi_build.OUT_PHASE
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    base = synth.make_tss(0) if args.workload == "tss4k" else synth.make_input(args.workload, 0)
    inp = synth.AtlasInput(base.xy, base.offsets, base.atlas_w, base.atlas_h, base.padding,
                           args.quality)
    n = inp.n
    xy = torch.from_numpy(np.ascontiguousarray(inp.xy, np.int32)).to(dev)
    off = torch.from_numpy(np.ascontiguousarray(inp.offsets, np.int32)).to(dev)
    out_xy = torch.empty((n, 2), dtype=torch.int32, device=dev)
    out_or = torch.empty(n, dtype=torch.uint8, device=dev)
    out_sc = torch.empty(1, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        tabi.pack_into(xy, off, n, inp.atlas_w, inp.atlas_h, inp.padding, inp.quality, out_xy,
                       out_or, out_sc, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.phase_clock:
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ph = tabi.debug_phase_clock(64)
        names = ["commit_and_loop_head", "knee_update", "fold", "configs_and_staging", "push",
                 "correction_and_score", "selection_and_knee_detection"]
        slots = {}
        for r in ph:
            if r[8] <= 0:
                continue
            slots[int(r[9])] = {"rows": int(r[8]), "feasible": int(r[10]),
                                "rows_pairs_overflow": int(r[7]) >> 32,
                                "pairs_listed": int(r[7]) & 0xffffffff,
                                "us": {nm: round(int(r[q]) / 100.0, 1) for q, nm in enumerate(names)},
                                "us_total": round(int(r[:7].sum()) / 100.0, 1)}
        print(json.dumps({"phase_clock": True, "workload": args.workload, "packs": args.steps,
                          "clock": "constant 100 MHz device clock, sums over the last pack's rows",
                          "slots": slots}))
        return
    if args.traffic_pass:
        for _ in range(args.steps):
            step()
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)  # reads and writes exactly 256 MiB
        torch.cuda.synchronize()
        print(json.dumps({"traffic_pass": True, "packs": args.steps, "copy_bytes": 256 << 20}))
        return
    _, khi_t = tabi.debug_order(xy, off, inp.atlas_w, inp.atlas_h, inp.padding, inp.quality)
    k_top = int(khi_t.cpu()[0])

    # the timed region brackets only the fold-and-push launch with the
    # library's HIP events (its duration feeds the roofline): every bracketed
    # stage adds a pair of event records to each pack, so the full stage split
    # comes from a separate loop after the timed region
    tabi.timing_reset()
    tabi.timing_stages(["pack"])
    tabi.timing_enable(True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tabi.timing_enable(False)
    pack_timed = tabi.timing_read()["pack"]
    tabi.timing_reset()
    tabi.timing_stages(None)
    tabi.timing_enable(True)
    for _ in range(min(args.steps, 50)):
        step()
    torch.cuda.synchronize()
    tabi.timing_enable(False)
    stages = tabi.timing_read()
    tabi.timing_reset()
    per = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    p50, p99 = percentile(per, 50), percentile(per, 99)
    ms_per_step = wall * 1000.0 / args.steps

    gxy = out_xy.cpu().numpy()
    gor = out_or.cpu().numpy()
    gsc = float(out_sc.cpu().numpy()[0])
    kstar = int(round(gsc * 64))

    # roofline of the dominant kernel (fold-and-push over every candidate
    # scale 1..k_top): algorithmic bytes per (chart, scale) unit = the chart's
    # stored grown column profile (one 4-byte word per grown texel column,
    # w_k + p of them) + grown width, compacting distance, interlock flags and
    # height read by the fold (13 B) + placement written (9 B)
    pack_bytes, units = pack_algorithmic_bytes(inp, k_top)
    unit_bytes = pack_bytes / max(units, 1)
    dom = max(stages, key=lambda s: stages[s][0])
    dom_ms, dom_launches = stages[dom]
    pack_ms, pack_launches = pack_timed
    avg_pack_ms = pack_ms / max(pack_launches, 1)
    achieved = pack_bytes / (avg_pack_ms * 1e-3) / 1e9 if avg_pack_ms > 0 else 0.0

    mix = " (70% stars 8-64 verts, 30% L/U)" if args.workload == "mixed2k" else ""
    result = {
        "metric": METRIC,
        "value": round(p50, 4),
        "unit": "ms per atlas pack (p50)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n} charts{mix} into "
                               f"{inp.atlas_w}x{inp.atlas_h}, padding {inp.padding}, quality "
                               f"{inp.quality}, plain single pack",
                   "charts": n, "atlas": [inp.atlas_w, inp.atlas_h], "padding": inp.padding,
                   "quality": inp.quality},
        "p50_ms": round(p50, 4),
        "p99_ms": round(p99, 4),
        "atlases_per_s_plain": round(1000.0 / ms_per_step, 2),
        "scale": gsc,
        "k_top": k_top,
        "stage_ms_per_pack": {s: round(v[0] / max(v[1], 1), 4) for s, v in stages.items()},
        "roofline": {"bound": "hbm", "kernel": "k_pack (fold-and-push, all candidate scales)",
                     "achieved": round(achieved, 3), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 6), "traffic": recorded_traffic() if args.workload == "mixed2k" else None,
                     "bytes_per_unit": round(unit_bytes, 2), "units_per_launch": units,
                     "bytes_per_launch": pack_bytes,
                     "avg_launch_ms": round(avg_pack_ms, 4), "dominant_stage": dom},
    }
    if not args.no_cpu:
        ms, reps, (oxy, oori, osc, ok) = cpu_baseline(inp, args.cpu_seconds)
        result["cpu_baseline"] = {"value": round(ms, 2), "unit": "ms per atlas pack",
                                  "cores": 1, "kind": "oracle",
                                  "sample": f"{reps} full packs of the same {n}-chart input"}
        result["bitexact_vs_oracle"] = bool(osc == gsc and np.array_equal(oxy, gxy) and
                                            np.array_equal(oori, gor))
    result["host_cores"] = host_cores()
    if not args.no_configs:
        try:
            result["configs"] = config_legs(tabi, torch, not args.no_cpu)
        except Exception as e:  # report, do not lose the main line
            result["configs"] = {"error": repr(e)}
    if not args.no_configs:
        try:
            result["ablations"] = ablation_leg(tabi, torch)
        except Exception as e:
            result["ablations"] = {"error": repr(e)}
    if not args.no_configs:
        try:
            result["variants"] = variants_leg(tabi, torch)
        except Exception as e:
            result["variants"] = {"error": repr(e)}
    if not args.no_batched:
        try:
            result["batched"] = batched_leg(tabi, torch,
                                            cpu_seconds=0.0 if args.no_cpu else args.cpu_seconds)
        except Exception as e:
            result["batched"] = {"error": repr(e)}
    if not args.no_served:
        try:
            result["served"] = served_leg()
        except Exception as e:
            result["served"] = {"error": repr(e)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
