"""Write tests/golden/inputs_sha256.json: SHA-256 fingerprints of the seeded workload inputs
(graphgen only; no expected result is involved)."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from graphgen.manifest import manifest  # noqa: E402

if __name__ == "__main__":
    m = manifest()
    with open(os.path.join(HERE, "inputs_sha256.json"), "w") as f:
        json.dump(m, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(m, indent=1))
