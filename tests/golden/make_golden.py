"""Writes the stored expected values under tests/golden/ from the oracle only.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as w  # noqa: E402
from oracle import ground  # noqa: E402


def sk20():
    out = []
    for index in range(16):
        J, h = w.sk1(20, seed=1, index=index)
        e, _, count = ground.brute_force(J, h)
        out.append({"seed": 1, "index": index, "e_gs": e, "count": count})
    return out


if __name__ == "__main__":
    rows = sk20()
    json.dump(rows[0], open(os.path.join(HERE, "sk20_ground.json"), "w"), indent=1)
    json.dump(rows, open(os.path.join(HERE, "sk20_ground_all.json"), "w"), indent=1)
    print(rows)
