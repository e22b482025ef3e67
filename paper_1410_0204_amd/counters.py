"""Bytes a kernel moves past the L2, from rocprofv3 counter runs.

Two counter passes of the same command (``--pmc FETCH_SIZE``, then
``--pmc WRITE_SIZE``; one pass each, since the counters share hardware) give
kibibytes per dispatch as the counters report them.  The same two passes over
a plain device copy of a known size (``bench.py --mode copy``: 512 MiB read
and written) calibrate each counter: scale = bytes / reported.  This writes
the summary that ``bench.py`` reads (``traffic``), keyed by the hash of the
kernel sources it was taken with.

Usage (after the four rocprofv3 runs, each with ``-d DIR --output-format csv``):
  python -m paper_1410_0204_amd.counters KERNEL WORKLOAD FETCH_DIR WRITE_DIR \\
      COPY_FETCH_DIR COPY_WRITE_DIR OUT_JSON [--per-launch-units N]
and, for the idle time between the launches of a graph-replayed kernel in a
kernel trace:
  python -m paper_1410_0204_amd.counters gaps TRACE_DIR KERNEL
"""

import argparse
import csv
import glob
import json
import os
import sys

from .build import source_hash


def dispatch_values(directory, counter, kernel=None):
    """{dispatch id: summed counter value} for dispatches whose kernel name
    contains ``kernel`` (all dispatches if None), from a rocprofv3 CSV run."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {directory}")
    out = {}
    names = {}
    for path in files:
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                name = row.get("Kernel_Name", "")
                if kernel is not None and kernel not in name:
                    continue
                key = (path, row.get("Dispatch_Id") or row.get("Correlation_Id"))
                out[key] = out.get(key, 0.0) + float(row["Counter_Value"])
                names[key] = name
    return out, names


def mean_per_dispatch(directory, counter, kernel):
    vals, _ = dispatch_values(directory, counter, kernel)
    if not vals:
        raise ValueError(f"no {counter} values for kernel {kernel!r} under {directory}")
    return sum(vals.values()) / len(vals), len(vals)


def largest_dispatch(directory, counter, kernel=None):
    vals, names = dispatch_values(directory, counter, kernel)
    key = max(vals, key=vals.get)
    return vals[key], names[key]


def launch_gaps(directory, kernel):
    """Idle time between consecutive dispatches of ``kernel`` in a rocprofv3
    kernel trace (``--kernel-trace --output-format csv``): the dispatches are
    grouped into runs separated by gaps of more than 1 ms (host work between
    model years); within the runs, the sum of the gaps against the sum of the
    kernel durations."""
    files = glob.glob(os.path.join(directory, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no kernel_trace.csv under {directory}")
    spans = []
    for path in files:
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                if kernel in row.get("Kernel_Name", ""):
                    spans.append((int(row["Start_Timestamp"]), int(row["End_Timestamp"])))
    spans.sort()
    busy = gap = 0
    runs = 1
    for (s0, e0), (s1, _) in zip(spans, spans[1:]):
        d = s1 - e0
        if d > 1_000_000:
            runs += 1
        else:
            gap += max(d, 0)
    busy = sum(e - s for s, e in spans)
    return {"kernel": kernel, "dispatches": len(spans), "runs": runs, "busy_ns": busy, "gap_ns": gap,
            "gap_fraction": gap / (busy + gap) if busy + gap else 0.0,
            "mean_gap_us": gap / max(len(spans) - runs, 1) / 1000.0}


def main(argv):
    if argv and argv[0] == "gaps":
        print(json.dumps(launch_gaps(argv[1], argv[2])))
        return
    ap = argparse.ArgumentParser()
    for a in ("kernel", "workload", "fetch_dir", "write_dir", "copy_fetch_dir", "copy_write_dir", "out"):
        ap.add_argument(a)
    ap.add_argument("--copy-bytes", type=int, default=512 * 1024 * 1024)
    ap.add_argument("--copy-kernel", default="copyBuffer", help="name of the copy kernel in the calibration runs")
    ap.add_argument("--commands", nargs="*", default=[])
    ap.add_argument("--per-launch-units", type=int, default=1,
                    help="units (time steps) of one launch, for the per-unit figure")
    args = ap.parse_args(argv)
    fetch, nf = mean_per_dispatch(args.fetch_dir, "FETCH_SIZE", args.kernel)
    write, nw = mean_per_dispatch(args.write_dir, "WRITE_SIZE", args.kernel)
    cf, cf_name = largest_dispatch(args.copy_fetch_dir, "FETCH_SIZE", args.copy_kernel)
    cw, cw_name = largest_dispatch(args.copy_write_dir, "WRITE_SIZE", args.copy_kernel)
    fscale = args.copy_bytes / (cf * 1024.0)
    wscale = args.copy_bytes / (cw * 1024.0)
    total = fetch * 1024.0 * fscale + write * 1024.0 * wscale
    rec = {"kernel": args.kernel, "workload": args.workload, "source_hash": source_hash(),
           "bytes_per_launch": total, "bytes_per_unit": total / args.per_launch_units,
           "fetch_bytes_per_launch": fetch * 1024.0 * fscale, "write_bytes_per_launch": write * 1024.0 * wscale,
           "fetch_kib_per_launch": fetch, "write_kib_per_launch": write,
           "launches_sampled": [nf, nw],
           "copy_calibration": {"bytes": args.copy_bytes, "fetch_kib": cf, "write_kib": cw,
                                "fetch_scale": fscale, "write_scale": wscale, "kernels": [cf_name, cw_name]},
           "commands": args.commands}
    tmp = args.out + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(rec, fh, indent=1)
    os.replace(tmp, args.out)
    print(json.dumps(rec))


if __name__ == "__main__":
    main(sys.argv[1:])
