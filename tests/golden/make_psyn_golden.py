"""Writes psyn_full.json: count and checksum of the paper's synthetic R join S join T
(Section 3.1.1) at the sizes the paper uses for its comparison (M = 10^7, r = 10^4,
d = 10; about 2e8 input rows, 10^7 result tuples), computed by the oracle's join-tree
DP (oracle.join_tree_dp, pinned against brute force and the binary hash join in
tests/test_oracle_join.py). The count must also equal the closed form r * d^3.
Run: python tests/golden/make_psyn_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

PATH = os.path.join(HERE, "psyn_full.json")
M, R, D, SEED = 10_000_000, 10_000, 10, 0x5EED0006


def main():
    t = time.perf_counter()
    q = W.psyn(M, R, D, seed=SEED)
    cnt, chk = oracle.join_tree_dp(q)
    assert cnt == R * D ** 3, (cnt, R * D ** 3)
    doc = {"about": "oracle.join_tree_dp on workloads.psyn(M, r, d, seed), written by make_psyn_golden.py",
           "M": M, "r": R, "d": D, "seed": SEED, "rows": [r.nrows for r in q.rels], "count": cnt, "checksum": chk}
    with open(PATH, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(doc, "%.1f s" % (time.perf_counter() - t))


if __name__ == "__main__":
    main()
