"""Writes triangle_cycles.json: count and checksum of the directed 3-cycle query on
the power-law edge workload (50M directed edges over 2^22 vertices, gamma 2.1, scaled
down by the factor given) computed by the oracle's adjacency-intersection count
(oracle.triangle_cycles, pinned against the binary hash-join plan and brute force in
tests/test_oracle_join.py). Run: python tests/golden/make_triangle_golden.py [scale ...]
"""
import json
from fractions import Fraction
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

SCALES = [1 / 16]
PATH = os.path.join(HERE, "triangle_cycles.json")


def main(argv):
    """Scales to compute (fractions such as 1/4 or 1.0; default 1/16). Each case
    replaces the stored case of the same scale; the others are kept."""
    scales = [float(Fraction(a)) for a in argv] or SCALES
    for sc in scales:
        q = W.config4(scale=sc)
        cnt, chk = oracle.triangle_cycles(*q.rels[0].cols)
        case = {"workload": "config4 (E join E join E, power-law edges)", "scale": sc,
                "seed": q.meta.get("seed"), "edges": q.rels[0].nrows, "count": cnt, "checksum": chk}
        print(case, flush=True)
        doc = {"about": "oracle.triangle_cycles on workloads.config4(scale=...), written by "
                        "make_triangle_golden.py", "cases": []}
        if os.path.exists(PATH):
            with open(PATH) as fh:
                doc = json.load(fh)
        doc["cases"] = sorted([c for c in doc["cases"] if abs(c["scale"] - sc) > 1e-12] + [case],
                              key=lambda c: c["scale"])
        with open(PATH + ".tmp%d" % os.getpid(), "w") as fh:
            json.dump(doc, fh, indent=1)
        os.replace(PATH + ".tmp%d" % os.getpid(), PATH)


if __name__ == "__main__":
    main(sys.argv[1:])
