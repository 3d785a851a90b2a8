"""Formats rocprofv3 CSV output (kernel stats, FETCH_SIZE / WRITE_SIZE) as a
short text summary, and reads the HBM traffic of a kernel back from one.

usage: python -m paper_2001_08289_amd.profile_summary <trace_dir> <fetch_dir> <write_dir> "<command>" > out.txt

The byte counters are scaled by what they read for two calibration kernels
of known size that ``bench.py --profile-only`` runs first: a 256 MiB fill
(writes only) and a 256 MiB sum (reads only).  The summary records a digest
of the kernel sources, so a reader can tell whether the kernels have changed
since the counters were taken.
"""
import collections
import csv
import hashlib
import os
import sys

CAL_BYTES = 256 * 1024 * 1024
CAL_WRITE = "FillFunctor"     # torch fill_ kernel (writes CAL_BYTES)
CAL_READ = "reduce_kernel"    # torch sum kernel (reads CAL_BYTES)
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def sources_digest() -> str:
    """sha256 over the device-code sources (file names and contents, sorted):
    the headers that define the kernels and the units that instantiate them;
    the host driver scfft.hip defines no kernel and is left out."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp")) and name != "scfft.hip":
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def _counter(d):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
        agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def _cal(agg, key):
    v = [x for k, xs in agg.items() if key in k for x in xs]
    return max(v) if v else None


def main():
    trace, fetch, write, command = sys.argv[1:5]
    print(f"# command: {command}")
    print(f"# kernel sources digest: {sources_digest()}")
    print("# kernel trace (rocprofv3 --kernel-trace --stats)")
    rows = list(csv.DictReader(open(os.path.join(trace, "run_kernel_stats.csv"))))
    print(f"{'kernel':80s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'pct':>6s}")
    for r in rows:
        print(f"{r['Name'][:80]:80s} {r['Calls']:>6s} {float(r['AverageNs'])/1e3:9.2f} "
              f"{float(r['MinNs'])/1e3:9.2f} {float(r['MaxNs'])/1e3:9.2f} {float(r['Percentage']):6.1f}")
    fa, wa = _counter(fetch), _counter(write)
    cf, cw = _cal(fa, CAL_READ), _cal(wa, CAL_WRITE)
    ff = CAL_BYTES / 1024 / cf if cf else None
    wf = CAL_BYTES / 1024 / cw if cw else None
    print(f"# calibration: 256 MiB sum -> FETCH_SIZE {cf} KiB (factor {ff}); "
          f"256 MiB fill -> WRITE_SIZE {cw} KiB (factor {wf})")
    for label, agg in (("FETCH_SIZE", fa), ("WRITE_SIZE", wa)):
        print(f"# {label} per dispatch (KiB, rocprofv3 --pmc {label})")
        for k, v in agg.items():
            print(f"{k[:80]:80s} n={len(v):3d} mean={sum(v)/len(v):12.1f} KiB")
    print("# HBM traffic per dispatch (bytes, calibrated FETCH + WRITE)")
    for k in fa:
        if k in wa and ff and wf:
            b = (sum(fa[k]) / len(fa[k]) * ff + sum(wa[k]) / len(wa[k]) * wf) * 1024
            print(f"traffic {k[:80]:80s} {b:14.0f}")


def read_traffic(path: str, kernel_prefix: str):
    """Calibrated bytes per dispatch of the first kernel whose name starts
    with ``kernel_prefix``, or None if the summary is missing or was taken
    from different kernel sources."""
    if not os.path.exists(path):
        return None
    digest = None
    for line in open(path):
        if line.startswith("# kernel sources digest:"):
            digest = line.split(":", 1)[1].strip()
        if line.startswith("traffic ") and line[8:].startswith(kernel_prefix):
            return float(line.split()[-1]) if digest == sources_digest() else None
    return None


if __name__ == "__main__":
    main()
