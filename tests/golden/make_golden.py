"""Writes tests/golden/oracle_packs.json: seeded inputs and the oracle's pack
of each (placements, orientations, scale).  Only the oracle computes the
expected values; the inputs come from the seeded generators.  The paper
prints no worked example, so these fixtures pin the oracle against
unintended change and give the GPU tests stored expectations; they are not
independent evidence of correctness (the pins in test_oracle_pins.py are).

    python tests/golden/make_golden.py
"""
from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from paper_2602_07782_amd import synth  # noqa: E402
from cases import small_input, with_quality  # noqa: E402


def cases():
    s64 = synth.make_input("stars64", 0)
    out = [("stars64 instance 0, quality 2", s64),
           ("stars64 instance 0, quality 1", with_quality(s64, 1)),
           ("stars64 instance 0, quality 0", with_quality(s64, 0))]
    for seed in range(6):
        out.append((f"small_input({seed})", small_input(seed)))
    return out


def main():
    oracle.build()
    recs = []
    for name, inp in cases():
        xy, ori, sc, k = oracle.pack(inp)
        recs.append({
            "name": name,
            "atlas_w": int(inp.atlas_w), "atlas_h": int(inp.atlas_h),
            "padding": int(inp.padding), "quality": int(inp.quality),
            "xy": [int(v) for v in inp.xy], "offsets": [int(v) for v in inp.offsets],
            "scale": sc, "k": k,
            "out_xy": [int(v) for v in xy.reshape(-1)], "out_orient": [int(v) for v in ori],
        })
    path = os.path.join(HERE, "oracle_packs.json")
    with open(path, "w") as f:
        json.dump({"written_by": "tests/golden/make_golden.py (oracle only)", "cases": recs}, f,
                  separators=(",", ":"))
        f.write("\n")
    print(path, len(recs), "cases")


if __name__ == "__main__":
    main()
