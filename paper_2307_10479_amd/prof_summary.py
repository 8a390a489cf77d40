"""Summaries of rocprofv3 result databases (kernel trace and counters) as text.

    python -m paper_2307_10479_amd.prof_summary trace <kt_results.db> [name filter]
    python -m paper_2307_10479_amd.prof_summary pmc <pmc_results.db> [name filter]

`trace` prints, per kernel name, the dispatch count, the total, average, minimum
and maximum duration (ms) and the VGPR / SGPR / LDS figures of its launches; `pmc`
prints every dispatch's counter values. Reads the SQLite views rocprofv3 writes.
"""
from __future__ import annotations

import sqlite3
import sys


def trace(db: str, filt: str = "") -> str:
    cur = sqlite3.connect(db).cursor()
    rows = cur.execute("select name, duration, vgpr_count, accum_vgpr_count, sgpr_count, lds_size, "
                       "scratch_size, grid_x, workgroup_x from kernels").fetchall()
    agg = {}
    for name, dur, vg, ag, sg, lds, scr, gx, wx in rows:
        if filt and filt not in name:
            continue
        a = agg.setdefault(name, dict(n=0, tot=0, mn=None, mx=0, vg=vg, ag=ag, sg=sg, lds=lds,
                                      scr=scr, waves=gx // max(1, wx)))
        a["n"] += 1
        a["tot"] += dur
        a["mn"] = dur if a["mn"] is None else min(a["mn"], dur)
        a["mx"] = max(a["mx"], dur)
    out = ["| kernel | calls | total ms | avg ms | min ms | max ms | VGPR | AGPR | SGPR | LDS B | "
           "scratch B | waves |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for name, a in sorted(agg.items(), key=lambda kv: -kv[1]["tot"]):
        out.append("| `%s` | %d | %.3f | %.3f | %.3f | %.3f | %d | %d | %d | %d | %d | %d |" % (
            name[:90], a["n"], a["tot"] / 1e6, a["tot"] / a["n"] / 1e6, a["mn"] / 1e6,
            a["mx"] / 1e6, a["vg"], a["ag"], a["sg"], a["lds"], a["scr"], a["waves"]))
    return "\n".join(out)


def pmc(db: str, filt: str = "") -> str:
    cur = sqlite3.connect(db).cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(counters_collection)")]
    res = {}
    for r in cur.execute("select * from counters_collection").fetchall():
        d = dict(zip(cols, r))
        name = d.get("kernel_name", "")
        if filt and filt not in name:
            continue
        res.setdefault((d.get("dispatch_id"), name), {})[d.get("counter_name")] = d.get("value")
    out = []
    for (disp, name), v in sorted(res.items()):
        out.append("dispatch %s `%s`: %s" % (disp, name[:90], ", ".join(
            "%s = %.1f" % (k, x) for k, x in sorted(v.items()))))
    return "\n".join(out)


if __name__ == "__main__":
    mode, db = sys.argv[1], sys.argv[2]
    filt = sys.argv[3] if len(sys.argv) > 3 else ""
    print(trace(db, filt) if mode == "trace" else pmc(db, filt))
