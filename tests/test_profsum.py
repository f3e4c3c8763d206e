"""The rocprofv3 summaries (paper_2308_16370_amd.profsum) on small synthetic databases:
steps split at the step-end kernel, per-occurrence durations, the timeline's span, busy
and idle times, and the counter traffic of picked launches scaled by a copy kernel."""
import json
import sqlite3
import subprocess
import sys

import pytest

from paper_2308_16370_amd import profsum


def _db(path, rows, pmc=()):
    db = sqlite3.connect(path)
    db.execute("create table kernels(name, start, end, grid_x, workgroup_x)")
    db.executemany("insert into kernels values(?,?,?,?,?)", rows)
    db.execute("create table pmc_events(name, start, counter_name, counter_value)")
    db.executemany("insert into pmc_events values(?,?,?,?)", pmc)
    db.commit()
    db.close()


def _run(*argv):
    r = subprocess.run([sys.executable, "-m", "paper_2308_16370_amd.profsum", *argv], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return r.stdout


def test_occurrences_and_timeline(tmp_path):
    # three steps of: a (5 us), b (5 us) overlapping a by 1 us, then k_materialize (2 us)
    rows, t = [], 0
    for _ in range(3):
        rows.append(("void sj::k_a(x)", t, t + 5000, 256, 256))
        rows.append(("void sj::k_b(y)", t + 4000, t + 9000, 512, 256))
        rows.append(("void sj::k_materialize<4, false>(z)", t + 12000, t + 14000, 1024, 256))
        t += 20000
    _db(tmp_path / "k.db", rows)
    table, n = profsum.occurrence_table(profsum._dispatches(sqlite3.connect(tmp_path / "k.db")), "k_materialize",
                                        skip=0)
    assert n == 3 and table[("k_b", 0)] == [5.0, 5.0, 5.0]
    out = _run("timeline", str(tmp_path / "k.db"), "--skip", "0")
    # span 14 us, busy 9 + 2 = 11 us, idle 3 us, sum of durations 12 us
    assert "| 0 | 3 | 14.0 | 11.0 | 3.0 | 12.0 |" in out
    assert "| 2 | k_materialize<4, false> | 4 | 12.0 | 2.0 | 3.0 |" in out


def test_traffic_picks_scale_by_the_copy_kernel(tmp_path):
    pmc_f, pmc_w, t = [], [], 0
    for _ in range(2):
        for name, f, w in (("k_probe<2>", 100.0, 10.0), ("k_probe<2>", 300.0, 30.0), ("k_materialize<4>", 50.0, 400.0)):
            pmc_f.append((name, t, "FETCH_SIZE", f))
            pmc_w.append((name, t, "WRITE_SIZE", w))
            t += 1
    pmc_f.append(("copyBuffer", t, "FETCH_SIZE", 512.0))   # a 1 KiB copy reads as 512 KiB... scale 2
    pmc_w.append(("copyBuffer", t, "WRITE_SIZE", 1.0))
    _db(tmp_path / "f.db", [], pmc_f)
    _db(tmp_path / "w.db", [], pmc_w)
    out = json.loads(_run("traffic", str(tmp_path / "f.db"), str(tmp_path / "w.db"), "--copy-bytes", "1024",
                          "--pick", "second=k_probe<2>@1", "--pick", "mat=k_materialize@0"))
    e = {x["label"]: x for x in out["entries"]}
    assert e["second"]["FETCH_SIZE"]["kib_per_launch"] == 300.0
    assert e["second"]["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(300.0 * 1024 * (1024 / (512.0 * 1024)))
    assert e["second"]["WRITE_SIZE"]["bytes_per_launch"] == pytest.approx(30.0 * 1024)
    assert e["mat"]["WRITE_SIZE"]["launches"] == 2
    assert out["source_hash"] == profsum.source_hash()
