"""Summaries of rocprofv3 output for roofline reporting.

    python -m paper_2407_20469_amd.pmc_summary stats <kernel_stats.csv> [top]
    python -m paper_2407_20469_amd.pmc_summary traffic <fetch_dir> <write_dir> \
        <copy_fetch_dir> <copy_write_dir> <min_grid> [out.json]

`traffic` reads the counter-collection CSVs of four `rocprofv3 --pmc` runs
(FETCH_SIZE and WRITE_SIZE of the darkfield gram kernel, and the same two
counters of the library's 4 GiB copy probe), scales each counter by the bytes
the copy is known to move, averages over the gram dispatches whose grid has at
least `min_grid` work-items, and records the hash of the gram's sources so a
later change of the kernel invalidates the figure.
"""

import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
GRAM_SOURCES = ["csrc/kernels_df.hpp", "csrc/common.hpp", "csrc/plan.hpp", "csrc/plan.cpp"]
COPY_BYTES = 4 << 30


def gram_source_hash():
    h = hashlib.sha256()
    for rel in GRAM_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_rows(d):
    path = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
    return list(csv.DictReader(open(path)))


def traffic(fetch_dir, write_dir, cf_dir, cw_dir, min_grid):
    cf = [float(r["Counter_Value"]) for r in _counter_rows(cf_dir)]
    cw = [float(r["Counter_Value"]) for r in _counter_rows(cw_dir)]
    sf = COPY_BYTES / 1024.0 / (sum(cf) / len(cf))
    sw = COPY_BYTES / 1024.0 / (sum(cw) / len(cw))
    f = [float(r["Counter_Value"]) for r in _counter_rows(fetch_dir) if int(r["Grid_Size"]) >= min_grid]
    w = [float(r["Counter_Value"]) for r in _counter_rows(write_dir) if int(r["Grid_Size"]) >= min_grid]
    fb = sum(f) / len(f) * 1024.0 * sf
    wb = sum(w) / len(w) * 1024.0 * sw
    return {"kernel": "k_df_gram", "fetch_scale": sf, "write_scale": sw, "dispatches": len(f),
            "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
            "bytes_per_launch": fb + wb, "source_sha256": gram_source_hash()}


def stats(path, top=16):
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["| total ms | calls | avg us | % | kernel |", "|---:|---:|---:|---:|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        out.append(f"| {float(r['TotalDurationNs']) / 1e6:.2f} | {int(r['Calls'])} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {100 * float(r['TotalDurationNs']) / tot:.1f} | "
                   f"`{r['Name'][:90]}` |")
    return "\n".join(out)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 16))
    elif sys.argv[1] == "traffic":
        res = traffic(*sys.argv[2:6], int(sys.argv[6]))
        text = json.dumps(res, indent=2)
        if len(sys.argv) > 7:
            with open(sys.argv[7], "w") as fh:
                fh.write(text + "\n")
        print(text)
    elif sys.argv[1] == "hash":
        print(gram_source_hash())
