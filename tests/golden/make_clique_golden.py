"""Writes clique_wiki.json: count and checksum of the 4-clique query (oracle.clique4)
and of the 3-clique query (oracle.hash_join) over the vote-network-sized power-law
edge list (workloads.config6: 103,663 edges on 7,066 vertices, gamma 2.5).
Run: python tests/golden/make_clique_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))


def main():
    import oracle
    import workloads as W
    t = time.perf_counter()
    q4 = W.config6(k=4)
    c4, k4 = oracle.clique4(q4)
    q3 = W.config6(k=3)
    _, c3, k3 = oracle.hash_join(q3)
    doc = {"about": "oracle.clique4 (4-clique) and oracle.hash_join (3-clique) on workloads.config6, written by "
                    "make_clique_golden.py", "seed": q4.meta["seed"], "edges": q4.rels[0].nrows,
           "nverts": q4.meta["nverts"], "gamma": q4.meta["gamma"],
           "clique4": {"count": c4, "checksum": k4}, "clique3": {"count": c3, "checksum": k3}}
    with open(os.path.join(HERE, "clique_wiki.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
    print(doc, "%.1f s" % (time.perf_counter() - t))


if __name__ == "__main__":
    main()
