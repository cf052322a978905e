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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--quality", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(atlases and scales shard across GPUs without communication; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2602_07782_amd as tabi
    from paper_2602_07782_amd import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    base = synth.make_input("mixed2k", 0)
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
    _, khi_t = tabi.debug_order(xy, off, inp.atlas_w, inp.atlas_h, inp.padding, inp.quality)
    k_top = int(khi_t.cpu()[0])

    tabi.timing_reset()
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
    stages = tabi.timing_read()
    per = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    p50, p99 = percentile(per, 50), percentile(per, 99)
    ms_per_step = wall * 1000.0 / args.steps

    gxy = out_xy.cpu().numpy()
    gor = out_or.cpu().numpy()
    gsc = float(out_sc.cpu().numpy()[0])
    kstar = int(round(gsc * 64))

    # roofline of the dominant kernel (fold-and-push): algorithmic bytes per
    # (chart, scale) unit = per-scale chart record + neighbour pair data +
    # chart fields read for OBB evaluation + placement written
    K = {0: 2, 1: 5, 2: 10}[inp.quality]
    rec = 16 + 4 * 16 + 2 * K * 8
    unit_bytes = rec + 4 + 1 + 40 + 9
    dom = max(stages, key=lambda s: stages[s][0])
    dom_ms, dom_launches = stages[dom]
    pack_ms, pack_launches = stages["pack"]
    avg_pack_ms = pack_ms / max(pack_launches, 1)
    units = n * k_top
    achieved = unit_bytes * units / (avg_pack_ms * 1e-3) / 1e9 if avg_pack_ms > 0 else 0.0

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
        "config": {"workload": f"mixed2k: {n} charts (70% stars 8-64 verts, 30% L/U) into "
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
                     "frac": round(achieved / PEAK_HBM_GBS, 6), "traffic": None,
                     "bytes_per_unit": unit_bytes, "units_per_launch": units,
                     "avg_launch_ms": round(avg_pack_ms, 4), "dominant_stage": dom},
    }
    if not args.no_cpu:
        ms, reps, (oxy, oori, osc, ok) = cpu_baseline(inp, args.cpu_seconds)
        result["cpu_baseline"] = {"value": round(ms, 2), "unit": "ms per atlas pack",
                                  "cores": 1, "kind": "oracle",
                                  "sample": f"{reps} full packs of the same 2,000-chart input"}
        result["bitexact_vs_oracle"] = bool(osc == gsc and np.array_equal(oxy, gxy) and
                                            np.array_equal(oori, gor))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
