"""rocprofv3 summaries for the profiles/ directory and the HBM traffic record
bench.py reports beside its roofline.

Usage (from the repository root, on CSV output written by rocprofv3):

    python -m paper_1602_02618_amd.profiling trace <kernel_stats.csv> <out.md> "<command>"
    python -m paper_1602_02618_amd.profiling pmc <fetch_counter_collection.csv> <write_counter_collection.csv> \
        <out.md> "<fetch command>" "<write command>"

The counter summary keeps, per kernel, FETCH_SIZE and WRITE_SIZE averaged per
dispatch.  Both counters are scaled by what they read for the plain device copy
that the profiled command runs after its timed steps (bench.py
--pmc-calibration: COPY_BYTES read and COPY_BYTES written), so the scaled
figures are HBM bytes.  The record for the dominant kernel carries a digest of
the kernel sources; bench.py reports the traffic only while the sources still
match it.
"""
import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/rdft.hip", "csrc/fft_lds.h", "csrc/cjt_internal.h")
COPY_BYTES = 256 << 20
RECORD_TAG = "traffic-record:"
# the kernel the roofline is quoted on: the inverse Hahn-block column pass
DOMINANT = "k_pass1_terms<double,(Src)1>"


def source_digest():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(k):
    """Kernel name without its return type, namespace and parameter list."""
    k = k.replace("void ", "").replace("cjt::", "")
    depth = 0
    for i, ch in enumerate(k):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            k = k[:i]
            break
    return re.sub(r"\s+", "", k)


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def _per_dispatch(path, counter):
    """{kernel: (dispatches, mean counter value per dispatch)} for one counter."""
    tot = defaultdict(float)
    disp = defaultdict(set)
    for r in _rows(path):
        if r.get("Counter_Name") != counter:
            continue
        k = short_name(r["Kernel_Name"])
        tot[k] += float(r["Counter_Value"])
        disp[k].add(r["Dispatch_Id"])
    return {k: (len(disp[k]), tot[k] / max(len(disp[k]), 1)) for k in tot}


def _largest_copy(path, counter):
    """(kernel, value) of the copy dispatch with the largest counter value:
    the calibration copy of COPY_BYTES."""
    best = None
    for r in _rows(path):
        if r.get("Counter_Name") != counter:
            continue
        k = short_name(r["Kernel_Name"])
        if "copy" not in k.lower():
            continue
        v = float(r["Counter_Value"])
        if best is None or v > best[1]:
            best = (k, v)
    return best


def summarize_pmc(fetch_csv, write_csv, out_md, fetch_cmd, write_cmd):
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")
    cf, cw = _largest_copy(fetch_csv, "FETCH_SIZE"), _largest_copy(write_csv, "WRITE_SIZE")
    if cf is None or cw is None:
        raise SystemExit("no copy kernel in the counter output: run bench.py with --pmc-calibration")
    fscale = COPY_BYTES / (cf[1] * 1024.0)
    wscale = COPY_BYTES / (cw[1] * 1024.0)
    lines = ["# HBM traffic per dispatch (rocprofv3 FETCH_SIZE / WRITE_SIZE)", "",
             "Commands (from the repository root, one counter per run):", "",
             "```", fetch_cmd, write_cmd, "```", "",
             f"Calibration: the {COPY_BYTES >> 20} MiB device copy `{cf[0]}` reads as "
             f"{cf[1] / 1024:.1f} MiB FETCH_SIZE and writes as {cw[1] / 1024:.1f} MiB WRITE_SIZE, "
             f"so FETCH_SIZE is scaled by {fscale:.3f} and WRITE_SIZE by {wscale:.3f}.", "",
             "Per dispatch (mean over the dispatches of each kernel); HBM MB are the scaled figures.", "",
             "| kernel | dispatches | FETCH KiB/dispatch | WRITE KiB/dispatch | HBM read MB | HBM write MB |",
             "|---|---|---|---|---|---|"]
    for k in sorted(fetch, key=lambda k: -fetch[k][1] * fetch[k][0])[:14]:
        n, f = fetch[k]
        w = write.get(k, (0, 0.0))[1]
        lines.append(f"| `{k[:90]}` | {n} | {f:.0f} | {w:.0f} | {f * 1024 * fscale / 1e6:.1f} | "
                     f"{w * 1024 * wscale / 1e6:.1f} |")
    dom = [k for k in fetch if k.startswith(DOMINANT)]
    if dom:
        k = max(dom, key=lambda k: fetch[k][0])
        rec = {"kernel": k, "source_digest": source_digest(),
               "read_bytes_per_launch": fetch[k][1] * 1024 * fscale,
               "write_bytes_per_launch": write.get(k, (0, 0.0))[1] * 1024 * wscale,
               "fetch_scale": fscale, "write_scale": wscale}
        lines += ["", f"{RECORD_TAG} {json.dumps(rec)}"]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize_trace(stats_csv, out_md, command):
    rows = _rows(stats_csv)
    lines = ["# Kernel trace (rocprofv3 --kernel-trace --stats)", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for r in rows[:24]:
        name = short_name(r["Name"])
        lines.append(f"| `{name[:90]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.0f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_traffic(md_path):
    """The traffic record of a counter summary, or None when absent or when the
    kernel sources have changed since the counters were taken."""
    try:
        with open(md_path) as f:
            for line in f:
                if line.startswith(RECORD_TAG):
                    rec = json.loads(line[len(RECORD_TAG):])
                    return rec if rec.get("source_digest") == source_digest() else None
    except OSError:
        return None
    return None


if __name__ == "__main__":
    if len(sys.argv) >= 5 and sys.argv[1] == "trace":
        summarize_trace(sys.argv[2], sys.argv[3], sys.argv[4])
    elif len(sys.argv) >= 7 and sys.argv[1] == "pmc":
        summarize_pmc(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6])
    else:
        print(__doc__)
        sys.exit(2)
