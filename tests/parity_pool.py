"""Host-side work of the wide parity sweeps, run in worker processes that
never touch the GPU: generate one seeded instance of a named workload and
pack it with the oracle at each requested quality."""
from __future__ import annotations

import numpy as np


def oracle_case(name: str, instance: int, qualities: tuple[int, ...]):
    """Returns (xy, offsets, atlas_w, atlas_h, padding, [(q, out_xy, out_orient, scale)])."""
    import oracle
    from paper_2602_07782_amd import synth
    base = synth.make_input(name, instance)
    res = []
    for q in qualities:
        inp = synth.AtlasInput(base.xy, base.offsets, base.atlas_w, base.atlas_h, base.padding, q)
        oxy, oori, osc, _ = oracle.pack(inp)
        res.append((q, np.asarray(oxy), np.asarray(oori), float(osc)))
    return (np.asarray(base.xy), np.asarray(base.offsets), base.atlas_w, base.atlas_h,
            base.padding, res)
