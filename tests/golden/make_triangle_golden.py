"""Writes triangle_cycles.json: count and checksum of the directed 3-cycle query on
the power-law edge workload (50M directed edges over 2^22 vertices, gamma 2.1, scaled
down by the factor given) computed by the oracle's adjacency-intersection count
(oracle.triangle_cycles, pinned against the binary hash-join plan and brute force in
tests/test_oracle_join.py). Run: python tests/golden/make_triangle_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

SCALES = [1 / 16]


def main():
    out = []
    for sc in SCALES:
        q = W.config4(scale=sc)
        cnt, chk = oracle.triangle_cycles(*q.rels[0].cols)
        out.append({"workload": "config4 (E join E join E, power-law edges)", "scale": sc,
                    "seed": q.meta.get("seed"), "edges": q.rels[0].nrows, "count": cnt, "checksum": chk})
        print(out[-1], flush=True)
    with open(os.path.join(HERE, "triangle_cycles.json"), "w") as fh:
        json.dump({"about": "oracle.triangle_cycles on workloads.config4(scale=...), written by "
                            "make_triangle_golden.py", "cases": out}, fh, indent=1)


if __name__ == "__main__":
    main()
