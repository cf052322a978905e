"""Stage timing brackets exactly the selected stages, and timing a call
changes none of its outputs."""
from __future__ import annotations

import sys

import pytest

from cases import small_input

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tabi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_07782_amd as t
    t.lib()
    return t


def test_stage_mask_brackets_only_the_selected_stages(tabi):
    import torch
    inp = small_input(41, n=300, W=512)
    print("timing: 300 charts, 512x512, seeds 41", file=sys.stderr, flush=True)
    ref = tabi.pack(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h, inp.padding, inp.quality,
                    device="cuda:0")
    torch.cuda.synchronize()
    try:
        for stages in (["pack"], ["prep", "profile"], None):
            tabi.timing_reset()
            tabi.timing_stages(stages)
            tabi.timing_enable(True)
            out = tabi.pack(inp.xy, inp.offsets, inp.atlas_w, inp.atlas_h, inp.padding,
                            inp.quality, device="cuda:0")
            torch.cuda.synchronize()
            tabi.timing_enable(False)
            got = tabi.timing_read()
            want = set(tabi.STAGES if stages is None else stages)
            for s, (ms, launches) in got.items():
                if s in want and s != "select":  # a single pack selects inside k_pack
                    assert launches == 1 and ms > 0.0, (stages, s, ms, launches)
                elif s not in want:
                    assert launches == 0 and ms == 0.0, (stages, s, ms, launches)
            for a, b in zip(ref, out):
                assert torch.equal(a, b)
    finally:
        tabi.timing_enable(False)
        tabi.timing_stages(None)
        tabi.timing_reset()
