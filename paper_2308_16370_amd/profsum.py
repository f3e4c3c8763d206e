"""Summaries of rocprofv3 output databases (rocpd SQLite) for the profiles folder.

    python -m paper_2308_16370_amd.profsum stats RUN.db [--cmd TEXT]
        Markdown: the per-kernel totals rocprofv3 --stats reports, then each kernel's
        launches by their position inside a step (a step ends with the launch of the
        kernel named by --step-end), averaged over the steady steps.

    python -m paper_2308_16370_amd.profsum traffic FETCH.db WRITE.db
            --pick LABEL=KERNEL@I [--pick ...] --copy-kernel NAME --copy-bytes N [--cmd TEXT]
        JSON: for each pick, HBM bytes per launch of occurrence I (in a step) of the
        kernel whose name contains KERNEL, from FETCH_SIZE and WRITE_SIZE (KiB per
        dispatch), each scaled by bytes / counter of a plain copy kernel of N bytes read
        and N bytes written in the same run; with a hash of the kernel sources.

    python -m paper_2308_16370_amd.profsum counters PASS1.db [PASS2.db ...] [--kernel SUBSTR]
        Markdown: the mean of every PMC counter per (kernel, launch position in a step).

    python -m paper_2308_16370_amd.profsum timeline RUN.db [--cmd TEXT]
        Markdown: per steady step, the span from its first launch's start to its last
        launch's end, the time some kernel runs (union of the launches' intervals) and
        the sum of launch durations; then the launches of the median step in start
        order, each with its start offset, duration and the idle time before it.
"""
from __future__ import annotations

import argparse
import json
import sqlite3
import statistics
import sys


def _short(name: str) -> str:
    n = name.replace("void ", "").replace("sj::", "").replace("(anonymous namespace)::", "")
    return n.split("(")[0]


def _dispatches(db):
    return db.execute("select name, start, end, grid_x, workgroup_x from kernels order by start").fetchall()


def _steps(rows, step_end: str):
    """Split the dispatch list into steps, each ending with a `step_end` launch."""
    steps, cur = [], []
    for r in rows:
        cur.append(r)
        if step_end in r[0]:
            steps.append(cur)
            cur = []
    return steps


def occurrence_table(rows, step_end: str, skip: int = 1):
    """{(kernel, i): [durations in us]} for the i-th launch of each kernel per step."""
    steps = _steps(rows, step_end)[skip:]
    table = {}
    for st in steps:
        seen = {}
        for name, s, e, _, _ in st:
            k = _short(name)
            i = seen.get(k, 0)
            seen[k] = i + 1
            table.setdefault((k, i), []).append((e - s) / 1e3)
    return table, len(steps)


def cmd_stats(args):
    db = sqlite3.connect(args.db)
    out = []
    if args.cmd:
        out.append("Command: `%s`\n" % args.cmd)
    out.append("| kernel | calls | total us | average us | % |")
    out.append("|---|---:|---:|---:|---:|")
    for name, calls, tot, avg, pct in db.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels "
            "order by total_duration desc limit %d" % args.top):
        out.append("| %s | %d | %.1f | %.2f | %.2f |" % (_short(name), calls, tot, avg, pct))
    rows = _dispatches(db)
    table, nsteps = occurrence_table(rows, args.step_end)
    if nsteps:
        out.append("")
        out.append("Launches by position in a step (%d steady steps, each ending with %s):\n"
                   % (nsteps, args.step_end))
        out.append("| kernel | occurrence | launches | mean us | median us |")
        out.append("|---|---:|---:|---:|---:|")
        for (k, i), d in sorted(table.items(), key=lambda kv: -statistics.mean(kv[1])):
            if statistics.mean(d) < args.min_us:
                continue
            out.append("| %s | %d | %d | %.2f | %.2f |" % (k, i, len(d), statistics.mean(d), statistics.median(d)))
    print("\n".join(out))


def _counter_per_dispatch(db, counter: str):
    """[(kernel name, dispatch start, value)] of one PMC counter, in dispatch order."""
    return db.execute("select name, start, counter_value from pmc_events where counter_name = ? order by start",
                      (counter,)).fetchall()


def _pick(vals, kernel: str, occurrence: int, step_end: str):
    """Mean counter value of the occurrence-th launch of `kernel` per step."""
    steps, cur = [], []
    for name, _, v in vals:
        cur.append((name, v))
        if step_end in name:
            steps.append(cur)
            cur = []
    picked = []
    for st in steps:
        n = [v for name, v in st if kernel in name]
        if len(n) > occurrence:
            picked.append(n[occurrence])
    return statistics.mean(picked) if picked else None, len(picked)


def source_hash() -> str:
    """Hash of the kernel sources (the same one bench.py compares)."""
    import hashlib
    import os
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def cmd_traffic(args):
    dbs = {}
    for counter, path in (("FETCH_SIZE", args.fetch_db), ("WRITE_SIZE", args.write_db)):
        db = sqlite3.connect(path)
        vals = _counter_per_dispatch(db, counter)
        copies = [v for name, _, v in vals if args.copy_kernel in name]
        cv = max(copies) if copies else None
        dbs[counter] = (vals, cv, args.copy_bytes / (cv * 1024.0) if cv else None)
    entries = []
    for pick in args.pick:
        label, rest = pick.split("=", 1)
        kernel, occ = rest.rsplit("@", 1)
        e = {"label": label, "kernel": kernel, "occurrence": int(occ)}
        for counter, (vals, cv, scale) in dbs.items():
            kv, n = _pick(vals, kernel, int(occ), args.step_end)
            e[counter] = {"kib_per_launch": kv, "launches": n, "copy_kib": cv, "scale": scale,
                          "bytes_per_launch": kv * 1024.0 * scale if (kv and scale) else None}
        f, w = e["FETCH_SIZE"]["bytes_per_launch"], e["WRITE_SIZE"]["bytes_per_launch"]
        e["bytes_per_launch"] = f + w if (f is not None and w is not None) else None
        entries.append(e)
    print(json.dumps({"command": args.cmd, "source_hash": source_hash(), "entries": entries}, indent=1))


def cmd_counters(args):
    """Markdown: per (kernel, occurrence in a step), the mean value of every PMC counter
    found in the given databases (one rocprofv3 --pmc pass each)."""
    cols = []
    data = {}
    for path in args.dbs:
        db = sqlite3.connect(path)
        names = [r[0] for r in db.execute("select distinct counter_name from pmc_events")]
        for cn in names:
            cols.append(cn)
            steps, cur = [], []
            for name, _, v in _counter_per_dispatch(db, cn):
                cur.append((_short(name), v))
                if args.step_end in name:
                    steps.append(cur)
                    cur = []
            for st in steps[1:]:
                seen = {}
                for k, v in st:
                    i = seen.get(k, 0)
                    seen[k] = i + 1
                    data.setdefault((k, i), {}).setdefault(cn, []).append(v)
    out = []
    if args.cmd:
        out.append("Commands:\n\n" + "\n".join("    " + c for c in args.cmd) + "\n")
    out.append("| kernel | occ | " + " | ".join(cols) + " |")
    out.append("|---|---:|" + "---:|" * len(cols))
    keys = sorted(data, key=lambda kv: (kv[0], kv[1]))
    for k in keys:
        if args.kernel and not any(x in k[0] for x in args.kernel):
            continue
        row = ["%.4g" % statistics.mean(data[k][c]) if c in data[k] else "" for c in cols]
        out.append("| %s | %d | %s |" % (k[0], k[1], " | ".join(row)))
    print("\n".join(out))


def _union(iv):
    """Total length covered by a list of (start, end) intervals."""
    tot, cur_s, cur_e = 0, None, None
    for a, b in sorted(iv):
        if cur_e is None or a > cur_e:
            if cur_e is not None:
                tot += cur_e - cur_s
            cur_s, cur_e = a, b
        else:
            cur_e = max(cur_e, b)
    if cur_e is not None:
        tot += cur_e - cur_s
    return tot


def cmd_timeline(args):
    db = sqlite3.connect(args.db)
    steps = _steps(_dispatches(db), args.step_end)[args.skip:]
    if args.max_launches:
        steps = [st for st in steps if len(st) <= args.max_launches]
    out = []
    if args.cmd:
        out.append("Command: `%s`\n" % args.cmd)
    if not steps:
        print("no steady steps")
        return
    rows = []
    for st in steps:
        t0 = min(r[1] for r in st)
        t1 = max(r[2] for r in st)
        busy = _union([(r[1], r[2]) for r in st])
        tot = sum(r[2] - r[1] for r in st)
        rows.append((t1 - t0, busy, tot, len(st), st))
    out.append("| step | launches | span us | busy us | idle us | sum of durations us |")
    out.append("|---:|---:|---:|---:|---:|---:|")
    for i, (span, busy, tot, n, _) in enumerate(rows):
        out.append("| %d | %d | %.1f | %.1f | %.1f | %.1f |" % (i, n, span / 1e3, busy / 1e3, (span - busy) / 1e3,
                                                                tot / 1e3))
    med = sorted(rows, key=lambda r: r[0])[len(rows) // 2]
    st = sorted(med[4], key=lambda r: r[1])
    t0 = st[0][1]
    out.append("")
    out.append("Median step (span %.1f us), launches in start order:\n" % (med[0] / 1e3))
    out.append("| # | kernel | grid | start us | duration us | idle before us |")
    out.append("|---:|---|---:|---:|---:|---:|")
    reach = t0
    for i, (name, s, e, gx, wx) in enumerate(st):
        idle = max(0, s - reach)
        reach = max(reach, e)
        out.append("| %d | %s | %d | %.1f | %.1f | %.1f |" % (i, _short(name), gx // max(wx, 1), (s - t0) / 1e3,
                                                               (e - s) / 1e3, idle / 1e3))
    print("\n".join(out))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--cmd", default="")
    s.add_argument("--top", type=int, default=30)
    s.add_argument("--step-end", default="k_materialize")
    s.add_argument("--min-us", type=float, default=5.0)
    s.set_defaults(fn=cmd_stats)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("--pick", action="append", required=True, help="LABEL=KERNEL@OCCURRENCE")
    t.add_argument("--copy-kernel", default="copyBuffer")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--step-end", default="k_materialize")
    t.add_argument("--cmd", default="")
    t.set_defaults(fn=cmd_traffic)
    c = sub.add_parser("counters")
    c.add_argument("dbs", nargs="+")
    c.add_argument("--step-end", default="k_materialize")
    c.add_argument("--kernel", action="append", default=[])
    c.add_argument("--cmd", action="append", default=[])
    c.set_defaults(fn=cmd_counters)
    tl = sub.add_parser("timeline")
    tl.add_argument("db")
    tl.add_argument("--cmd", default="")
    tl.add_argument("--step-end", default="k_materialize")
    tl.add_argument("--skip", type=int, default=1)
    tl.add_argument("--max-launches", type=int, default=0)
    tl.set_defaults(fn=cmd_timeline)
    args = ap.parse_args(argv)
    args.fn(args)


if __name__ == "__main__":
    sys.exit(main())
