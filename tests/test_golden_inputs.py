"""CPU: every stored whole-grid oracle file still belongs to the seeded inputs
the GPU tests generate (a changed generator would otherwise compare the GPU
against values of other inputs)."""
import json
import os

import pytest

import mala_synth
from tests.golden.make_golden import CASES, fingerprint

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("case", sorted(CASES))
def test_golden_fingerprint_matches_inputs(case):
    g = json.load(open(os.path.join(GOLD, "full_%s.json" % case)))
    snap, net = CASES[case][0](), CASES[case][1]()
    assert g["fingerprint"] == fingerprint(snap, net)
    assert g["n_points"] == snap.n_points and g["n_atoms"] == snap.n_atoms


def test_slab_sample_definition():
    g = json.load(open(os.path.join(GOLD, "full_slab_sample.json")))
    snap = mala_synth.slab()
    pts = mala_synth.strided_points(snap.n_points, g["stride"], g["offset"])
    assert (g["stride"], g["offset"]) == mala_synth.SLAB_SAMPLE
    assert len(pts) == g["n_sample"] and len(g["sample"]["dos"]) == mala_synth.EGRID[2]
    assert pts[0] == g["offset"] and pts[-1] < snap.n_points
