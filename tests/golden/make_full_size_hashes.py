#!/usr/bin/env python3
"""Write full_size_sha256.txt: the CPU oracle's output digest for every
full-size case of full_size_cases.py.  Calls only the oracle and the seeded
generators."""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
import full_size_cases as fc  # noqa: E402


def main():
    oracle.build(force=False)
    lines = ["# name sha256(int32 LE [N(N+1)/2][2] of the oracle's output) N T",
             "# written by make_full_size_hashes.py (CPU oracle only)"]
    t0 = time.time()
    for name, x in fc.cases():
        v = oracle.correlate(x)
        lines.append(f"{name} {fc.vis_sha256(v)} {x.shape[1]} {x.shape[0]}")
        print(f"{time.time() - t0:7.1f} s  {lines[-1]}", flush=True)
    with open(fc.DIGESTS, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
