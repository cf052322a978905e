"""Stored oracle packs (tests/golden/oracle_packs.json, written by
tests/golden/make_golden.py from the oracle alone): the oracle still gives
them bit for bit, they are valid layouts (no overlap, nothing outside the
atlas, no chart lost), and their inputs are the seeded generators' current
output."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from paper_2602_07782_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "oracle_packs.json")


def golden_cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def as_input(c):
    return synth.AtlasInput(np.array(c["xy"], np.int32), np.array(c["offsets"], np.int32),
                            c["atlas_w"], c["atlas_h"], c["padding"], c["quality"])


CASES = golden_cases()


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_oracle_reproduces_stored_pack(orc, c):
    xy, ori, sc, k = orc.pack(as_input(c))
    assert sc == c["scale"] and k == c["k"]
    assert np.array_equal(xy.reshape(-1), np.array(c["out_xy"], np.int32))
    assert np.array_equal(ori, np.array(c["out_orient"], np.uint8))


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_stored_pack_is_a_valid_layout(chk, c):
    st = chk.check_layout(as_input(c), np.array(c["out_xy"], np.int32),
                          np.array(c["out_orient"], np.uint8), c["k"])
    assert st["overlap"] == 0 and st["outside"] == 0 and st["empty"] == 0, st


def test_stored_inputs_match_the_generators():
    from cases import small_input, with_quality
    s64 = synth.make_input("stars64", 0)
    expect = {"stars64 instance 0, quality 2": s64,
              "stars64 instance 0, quality 1": with_quality(s64, 1),
              "stars64 instance 0, quality 0": with_quality(s64, 0)}
    for seed in range(6):
        expect[f"small_input({seed})"] = small_input(seed)
    assert set(expect) == {c["name"] for c in CASES}
    for c in CASES:
        e = expect[c["name"]]
        assert np.array_equal(e.xy, np.array(c["xy"], np.int32)), c["name"]
        assert np.array_equal(e.offsets, np.array(c["offsets"], np.int32)), c["name"]
        assert (e.atlas_w, e.atlas_h, e.padding, e.quality) == (
            c["atlas_w"], c["atlas_h"], c["padding"], c["quality"]), c["name"]
