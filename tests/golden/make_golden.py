"""Writes the stored determinism hashes of the seeded input generator
(tests/golden/inputs_hashes.json).  Calls only the input generator; no value
stored here comes from the GPU path.

    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import inputs  # noqa: E402


def graph_hash(g):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(g.row_ptr).tobytes())
    h.update(np.ascontiguousarray(g.col_idx).tobytes())
    return h.hexdigest()


def main():
    out = {"graphs": {}}
    for kind, name in ((inputs.RMAT, "rmat"), (inputs.UNIFORM, "uniform")):
        for scale, seed in ((10, 1), (16, 1)):
            g = inputs.Graph(kind, scale, 16, seed)
            out["graphs"]["%s-%d-%d" % (name, scale, seed)] = graph_hash(g)
    g = inputs.graph(inputs.RMAT, 16, 16, 1)
    out["roots_s16_seed1"] = [int(x) for x in inputs.roots(g, 8, 1)]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "inputs_hashes.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
