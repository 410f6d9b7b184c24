"""Text summary of a rocprofv3 results database (the `*_results.db` that
`rocprofv3 -d DIR -o run ...` writes): per kernel the dispatch count, total
and average duration, and, for a `--pmc` run, each counter's average, minimum
and maximum per dispatch (summed over the counter's hardware instances).

    python -m paper_2507_11542_amd.rocprof_summary RESULTS.db [KERNEL_SUBSTRING]

Measurement only; nothing here is part of the solver.
"""
from __future__ import annotations

import collections
import sqlite3
import sys


def kernel_times(db: str):
    con = sqlite3.connect(db)
    rows = con.execute(
        "select s.display_name, d.start, d.end, d.grid_size_x from rocpd_kernel_dispatch d "
        "join rocpd_info_kernel_symbol s on d.kernel_id = s.id order by d.start").fetchall()
    out = collections.OrderedDict()
    for name, start, end, grid in rows:
        e = out.setdefault((name, grid), [0, 0.0])
        e[0] += 1
        e[1] += (end - start) / 1e3
    return out


def counters(db: str, key: str = ""):
    con = sqlite3.connect(db)
    q = ("select s.display_name, d.id, p.name, e.value, d.grid_size_x from rocpd_pmc_event e "
         "join rocpd_info_pmc p on e.pmc_id = p.id "
         "join rocpd_kernel_dispatch d on e.event_id = d.event_id "
         "join rocpd_info_kernel_symbol s on d.kernel_id = s.id")
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    grids = {}
    for name, did, cname, val, grid in con.execute(q):
        if key and key not in name:
            continue
        per[(name, did)][cname] += val
        grids[(name, did)] = grid
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for (name, did), cs in per.items():
        for c, v in cs.items():
            agg[(name, grids[(name, did)])][c].append(v)
    return agg


def main(argv) -> int:
    if len(argv) < 2:
        print(__doc__)
        return 2
    db = argv[1]
    key = argv[2] if len(argv) > 2 else ""
    times = kernel_times(db)
    total = sum(t for _, t in times.values()) or 1.0
    print("| kernel | grid (threads) | dispatches | total us | avg us | % |")
    print("|---|---|---|---|---|---|")
    for (name, grid), (n, t) in sorted(times.items(), key=lambda kv: -kv[1][1]):
        if key and key not in name:
            continue
        print("| %s | %d | %d | %.1f | %.3f | %.2f |" % (name, grid, n, t, t / n, 100 * t / total))
    agg = counters(db, key)
    if agg:
        print()
        print("| kernel | grid | dispatches | counter | avg | min | max |")
        print("|---|---|---|---|---|---|---|")
        for (name, grid), cs in sorted(agg.items()):
            for c, vs in sorted(cs.items()):
                print("| %s | %d | %d | %s | %.1f | %.1f | %.1f |"
                      % (name, grid, len(vs), c, sum(vs) / len(vs), min(vs), max(vs)))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
