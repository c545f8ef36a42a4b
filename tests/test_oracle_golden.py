"""The oracle's tiny renders match the committed digests (regression guard)."""
import json
import os

from tests.golden.make_golden import digests


def test_oracle_tiny_digests(orc):
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_tiny.json")) as f:
        ref = json.load(f)["cases"]
    got = digests()
    for a, b in zip(ref, got):
        assert a["case"] == b["case"]
        assert a["rays_per_bounce"] == b["rays_per_bounce"]
        assert a["sha256"] == b["sha256"], a["case"]
