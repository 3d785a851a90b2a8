"""Formats rocprofv3 CSV output (kernel stats, FETCH_SIZE / WRITE_SIZE) as text.

usage: python profiles/summarize.py <trace_dir> <fetch_dir> <write_dir> "<command>" > out.txt
"""
import collections
import csv
import os
import sys


def main():
    trace, fetch, write, command = sys.argv[1:5]
    print(f"# command: {command}")
    print("# kernel trace (rocprofv3 --kernel-trace --stats)")
    rows = list(csv.DictReader(open(os.path.join(trace, "run_kernel_stats.csv"))))
    print(f"{'kernel':80s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'pct':>6s}")
    for r in rows:
        print(f"{r['Name'][:80]:80s} {r['Calls']:>6s} {float(r['AverageNs'])/1e3:9.2f} "
              f"{float(r['MinNs'])/1e3:9.2f} {float(r['MaxNs'])/1e3:9.2f} {float(r['Percentage']):6.1f}")
    for label, d in (("FETCH_SIZE", fetch), ("WRITE_SIZE", write)):
        print(f"# {label} per dispatch (KiB, rocprofv3 --pmc {label})")
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            agg[r["Kernel_Name"][:80]].append(float(r["Counter_Value"]))
        for k, v in agg.items():
            print(f"{k:80s} n={len(v):3d} mean={sum(v)/len(v):12.1f} KiB")


if __name__ == "__main__":
    main()
