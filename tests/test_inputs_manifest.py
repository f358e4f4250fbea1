"""The seeded workload inputs are the ones recorded in tests/golden/inputs_sha256.json (written
by tests/golden/make_inputs_manifest.py): a generator change shows up here first."""
import json
import os

from graphgen.manifest import manifest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "inputs_sha256.json")


def test_inputs_match_the_manifest():
    want = json.load(open(GOLDEN))
    got = manifest()
    assert got == want
