"""Summarise rocprofv3 counter collections written as CSV
(`rocprofv3 --pmc C1 C2 ... -f csv -d DIR -o NAME -- ...`): for every kernel
whose name contains one of the given substrings, the number of dispatches
and, per counter, the sum over dispatches and the mean per dispatch.

    python measure/pmc_summary.py CSV [KERNEL_SUBSTRING ...]

With no substrings every kernel is listed.
"""
import csv
import sys
from collections import defaultdict


def summarise(path, keys=()):
    per = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = row.get("Kernel_Name", "")
            if keys and not any(k in name for k in keys):
                continue
            disp[name].add(row.get("Dispatch_Id", row.get("Correlation_Id", "")))
            per[name][row["Counter_Name"]] += float(row["Counter_Value"])
    return per, disp


def main():
    path, keys = sys.argv[1], tuple(sys.argv[2:])
    per, disp = summarise(path, keys)
    counters = sorted({c for v in per.values() for c in v})
    print("| kernel | dispatches | " + " | ".join(f"{c} (sum) | {c} (per dispatch)" for c in counters) + " |")
    print("|---|---|" + "---|---|" * len(counters))
    for name in sorted(per, key=lambda n: -max(per[n].values())):
        n = len(disp[name])
        cells = " | ".join(f"{per[name].get(c, 0.0):.6g} | {per[name].get(c, 0.0) / n:.6g}" for c in counters)
        print(f"| `{name[:80]}` | {n} | {cells} |")


if __name__ == "__main__":
    main()
