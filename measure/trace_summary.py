"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite, written by
`rocprofv3 --kernel-trace --stats -d DIR -o NAME -- ...`): per-kernel totals
and, for one kernel, the durations of its first N dispatches (or of N
dispatches from index FIRST on, with the wall time they span).

    python measure/trace_summary.py DB [KERNEL_SUBSTRING N [FIRST]]
"""
import sqlite3
import sys


def main():
    db = sys.argv[1]
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, count(*), sum(duration), avg(duration) from kernels "
                          "group by name order by sum(duration) desc"))
    total = sum(r[2] for r in rows)
    print("| kernel | dispatches | total ms | average ms | % |")
    print("|---|---|---|---|---|")
    for name, n, tot, avg in rows[:12]:
        print(f"| `{name[:80]}` | {n} | {tot / 1e6:.3f} | {avg / 1e6:.3f} | {100 * tot / total:.2f} |")
    if len(sys.argv) > 3:
        key, n = sys.argv[2], int(sys.argv[3])
        first = int(sys.argv[4]) if len(sys.argv) > 4 else 0
        rows = list(c.execute("select duration, start, end from kernels where name like ? order by start",
                              (f"%{key}%",)))[first:first + n]
        d = [r[0] for r in rows]
        what = f"first {len(d)}" if first == 0 else f"{len(d)} (from index {first})"
        print(f"\n{what} dispatches of *{key}*: " + ", ".join(f"{v / 1e6:.3f}" if first else f"{v / 1e6:.2f}" for v in d)
              + f" ms; average {sum(d) / len(d) / 1e6:.2f} ms")
        if first:
            print(f"sum {sum(d) / 1e6:.1f} ms of kernel time; {(rows[-1][2] - rows[0][1]) / 1e6:.1f} ms from the first "
                  f"one's start to the last one's end")


if __name__ == "__main__":
    main()
