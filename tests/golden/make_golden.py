"""Writes the stored expected values under tests/golden/ that are not taken
from the paper.  It calls only the CPU oracle (oracle/), never the GPU path.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle  # noqa: E402


def sampler_vectors():
    cases = []
    for T, seed, epoch in [(1, 0, 0), (2, 1, 0), (10, 1, 0), (1000, 3000, 0), (1000, 3000, 9),
                           (90_001, 3001, 2), (1 << 20, 7, 1), ((1 << 20) + 1, 7, 1)]:
        p = oracle.perm(T, seed, epoch)
        cases.append({"T": T, "seed": seed, "epoch": epoch, "head": p[:32].tolist()})
    return {"_source": "oracle.perm (Feistel cycle-walk sampler), see oracle/stdecomp_oracle.c",
            "cases": cases}


if __name__ == "__main__":
    with open(os.path.join(HERE, "sampler_vectors.json"), "w") as f:
        json.dump(sampler_vectors(), f, indent=1)
    print("wrote", os.path.join(HERE, "sampler_vectors.json"))
