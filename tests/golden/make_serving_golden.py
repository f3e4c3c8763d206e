"""Writes serving_mix.json: for every query of the batched / served mix (256 chain and
star joins, workloads.serving with seed 0x5EED0005 and rows in [10^4, 2*10^7]) the draw
that the redraw rule keeps (the first whose exact count is at most 2^26) and its exact
count and checksum, computed by the oracle's join-tree DP (oracle.join_tree_dp, pinned
against brute force and the binary hash join in tests/test_oracle_join.py) on the
numpy columns (workloads.serving.query_cpu). Queries are spread over worker processes.
Run: python tests/golden/make_serving_golden.py [workers]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

PATH = os.path.join(HERE, "serving_mix.json")
SEED, N, MIN_ROWS, MAX_ROWS, CAP = 0x5EED0005, 256, 10_000, 20_000_000, 1 << 26


def one(index):
    import oracle
    from workloads import serving as S
    sp = S.draw_spec(SEED, index, 0, min_rows=MIN_ROWS, max_rows=MAX_ROWS)
    while True:
        cnt, chk = oracle.join_tree_dp(S.query_cpu(sp))
        if cnt <= CAP:
            break
        sp = S.redraw(SEED, sp, min_rows=MIN_ROWS, max_rows=MAX_ROWS)
    return {"index": index, "draw": sp.draw, "kind": sp.kind, "rows": sp.rows, "s": sp.s, "count": cnt,
            "checksum": chk}


def main(argv):
    workers = int(argv[0]) if argv else 6
    t = time.perf_counter()
    with mp.Pool(workers) as pool:
        out = []
        for i, r in enumerate(pool.imap(one, range(N))):
            out.append(r)
            if i % 16 == 15:
                print("%d queries, %.0f s" % (i + 1, time.perf_counter() - t), flush=True)
    doc = {"about": "oracle.join_tree_dp of every query of workloads.serving's mix, written by "
                    "make_serving_golden.py", "seed": SEED, "n": N, "min_rows": MIN_ROWS, "max_rows": MAX_ROWS,
           "count_cap": CAP, "queries": out}
    with open(PATH, "w") as fh:
        json.dump(doc, fh, indent=0)
    print("done in %.0f s" % (time.perf_counter() - t))


if __name__ == "__main__":
    main(sys.argv[1:])
