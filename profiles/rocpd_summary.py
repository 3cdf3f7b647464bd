"""Summarize a rocprofv3 rocpd database (kernel trace) as a per-kernel table.

Usage: python profiles/rocpd_summary.py <run_results.db>
Prints name, calls, total ms, average us, min/max us, VGPR/AGPR/SGPR, LDS.
"""
import sqlite3
import sys


def main(path):
    db = sqlite3.connect(path)
    cur = db.cursor()
    rows = cur.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration), "
        "max(vgpr_count), max(accum_vgpr_count), max(sgpr_count), max(lds_size), max(grid_x), max(workgroup_x) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    print("%-60s %6s %12s %12s %12s %12s %5s %5s %5s %7s %8s %5s %6s" % (
        "kernel", "calls", "total_ms", "avg_us", "min_us", "max_us", "vgpr", "agpr", "sgpr", "lds", "grid", "wg", "pct"))
    for r in rows:
        name = r[0] if len(r[0]) <= 60 else r[0][:57] + "..."
        print("%-60s %6d %12.3f %12.2f %12.2f %12.2f %5d %5d %5d %7d %8d %5d %6.2f" % (
            name, r[1], r[2] / 1e6, r[3] / 1e3, r[4] / 1e3, r[5] / 1e3, r[6] or 0, r[7] or 0, r[8] or 0,
            r[9] or 0, r[10] or 0, r[11] or 0, 100.0 * r[2] / total))


if __name__ == "__main__":
    main(sys.argv[1])
