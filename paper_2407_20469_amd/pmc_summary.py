"""Summaries of rocprofv3 output for roofline reporting.

    python -m paper_2407_20469_amd.pmc_summary stats <kernel_stats.csv> [top]
    python -m paper_2407_20469_amd.pmc_summary dispatches <kernel_trace.csv> <regex> <min_grid>
    python -m paper_2407_20469_amd.pmc_summary hbm <fetch_dir> <write_dir> \
        <copy_fetch_dir> <copy_write_dir> <min_grid>
    python -m paper_2407_20469_amd.pmc_summary traffic <fetch_dir> <write_dir> \
        <copy_fetch_dir> <copy_write_dir> <min_grid> [out.json]
    python -m paper_2407_20469_amd.pmc_summary busy <kernel_trace.csv> <regex> [gap_ms]

`traffic` reads the counter-collection CSVs of four `rocprofv3 --pmc` runs
(FETCH_SIZE and WRITE_SIZE of the darkfield gram kernels, and the same two
counters of the library's 4 GiB copy probe), scales each counter by the bytes
the copy is known to move, and sums the gram dispatches whose grid has at least
`min_grid` work-items.  One gram launch is one darkfield image step of a
batch (one `k_df_gram` dispatch).  The hash of the gram's sources is recorded
so a later change of the kernel invalidates the figure.
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
    def gram(d):
        rows = [r for r in _counter_rows(d)
                if int(r["Grid_Size"]) >= min_grid and "k_df_gram" in r["Kernel_Name"]]
        return sum(float(r["Counter_Value"]) for r in rows), len(rows)

    f, steps = gram(fetch_dir)
    w, steps_w = gram(write_dir)
    if steps == 0 or steps != steps_w:
        raise ValueError("the two counter runs must cover the same gram dispatches")
    fb = f / steps * 1024.0 * sf
    wb = w / steps * 1024.0 * sw
    return {"kernel": "k_df_gram", "fetch_scale": sf,
            "write_scale": sw, "image_steps": steps, "fetch_bytes_per_launch": fb,
            "write_bytes_per_launch": wb, "bytes_per_launch": fb + wb,
            "source_sha256": gram_source_hash()}


def dispatches(path, pattern, min_grid):
    """Per-kernel count, mean and spread of the dispatch durations of the kernels
    matching `pattern` whose grid has at least `min_grid` work-items (the batched
    calls, not the single-tile ones)."""
    import re
    rx = re.compile(pattern)
    by = {}
    for r in csv.DictReader(open(path)):
        if "Grid_Size" in r:
            grid = int(r["Grid_Size"])
        else:
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        if not rx.search(r["Kernel_Name"]) or grid < min_grid:
            continue
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        by.setdefault(r["Kernel_Name"][:90], []).append(d)
    out = ["| kernel | dispatches | mean us | min us | max us |", "|---|---:|---:|---:|---:|"]
    for k, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| `{k}` | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} |")
    return "\n".join(out)


def hbm(fetch_dir, write_dir, cf_dir, cw_dir, min_grid):
    """Per-kernel HBM bytes (scaled FETCH_SIZE + WRITE_SIZE) and the rate they
    imply over each dispatch's own duration, for the dispatches with at least
    `min_grid` work-items; also the total over all of them."""
    cf = [float(r["Counter_Value"]) for r in _counter_rows(cf_dir)]
    cw = [float(r["Counter_Value"]) for r in _counter_rows(cw_dir)]
    sf = COPY_BYTES / 1024.0 / (sum(cf) / len(cf))
    sw = COPY_BYTES / 1024.0 / (sum(cw) / len(cw))
    acc = {}
    for d, scale, key in ((fetch_dir, sf, "fetch"), (write_dir, sw, "write")):
        for r in _counter_rows(d):
            if int(r["Grid_Size"]) < min_grid:
                continue
            e = acc.setdefault(r["Kernel_Name"][:90], {"fetch": 0.0, "write": 0.0, "ns": 0.0,
                                                       "n": 0})
            e[key] += float(r["Counter_Value"]) * 1024.0 * scale
            if key == "fetch":
                e["ns"] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                e["n"] += 1
    out = ["| kernel | dispatches | GB per dispatch (read + write) | mean us | GB/s | of 8 TB/s |",
           "|---|---:|---:|---:|---:|---:|"]
    tb = tns = 0.0
    for k, e in sorted(acc.items(), key=lambda kv: -kv[1]["ns"]):
        b = e["fetch"] + e["write"]
        tb += b
        tns += e["ns"]
        out.append(f"| `{k}` | {e['n']} | {b / e['n'] / 1e9:.3f} ({e['fetch'] / e['n'] / 1e9:.3f} + "
                   f"{e['write'] / e['n'] / 1e9:.3f}) | {e['ns'] / e['n'] / 1e3:.1f} | "
                   f"{b / e['ns']:.0f} | {b / e['ns'] / 8000:.2f} |")
    out.append(f"| all of the above | | {tb / 1e9:.2f} GB in total | {tns / 1e6:.2f} ms in total | "
               f"{tb / tns:.0f} | {tb / tns / 8000:.2f} |")
    return "\n".join(out)


def busy(path, pattern, gap_ms=5.0):
    """GPU busy fraction of the longest passes of the kernels matching
    `pattern`: their dispatches are cut into passes at idle gaps longer than
    `gap_ms` (no kernel of the pattern running), and for the two longest
    passes the union of the dispatch intervals is compared with the pass's
    span.  Concurrent dispatches on several streams count once."""
    import re
    rx = re.compile(pattern)
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                for r in csv.DictReader(open(path)) if rx.search(r["Kernel_Name"]))
    passes, cur, end = [], [], None
    for a, b in iv:
        if end is not None and a - end > gap_ms * 1e6:
            passes.append(cur)
            cur = []
            end = None
        cur.append((a, b))
        end = b if end is None else max(end, b)
    if cur:
        passes.append(cur)
    out = ["| pass | dispatches | span s | busy s | busy fraction | idle s |",
           "|---|---:|---:|---:|---:|---:|"]
    ranked = sorted(range(len(passes)),
                    key=lambda i: -(max(b for _, b in passes[i]) - passes[i][0][0]))[:2]
    for i in sorted(ranked):
        p = passes[i]
        span = max(b for _, b in p) - p[0][0]
        tot, ca, cb = 0, None, None
        for a, b in p:
            if cb is None or a > cb:
                if cb is not None:
                    tot += cb - ca
                ca, cb = a, b
            else:
                cb = max(cb, b)
        tot += cb - ca
        out.append(f"| {i} | {len(p)} | {span / 1e9:.3f} | {tot / 1e9:.3f} | {tot / span:.4f} | "
                   f"{(span - tot) / 1e9:.3f} |")
    return "\n".join(out)


def counters(d, pattern, min_grid):
    """Per-dispatch mean of every counter of one --pmc run, over the dispatches
    of the kernels matching `pattern` with at least `min_grid` work-items."""
    import re
    rx = re.compile(pattern)
    tot, cnt = {}, {}
    for r in _counter_rows(d):
        if int(r["Grid_Size"]) < min_grid or not rx.search(r["Kernel_Name"]):
            continue
        k = r["Counter_Name"]
        tot[k] = tot.get(k, 0.0) + float(r["Counter_Value"])
        cnt[k] = cnt.get(k, 0) + 1
    out = ["| counter | dispatches | per dispatch |", "|---|---:|---:|"]
    for k in sorted(tot):
        out.append(f"| {k} | {cnt[k]} | {tot[k] / cnt[k]:.4g} |")
    return "\n".join(out)


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
    elif sys.argv[1] == "dispatches":
        print(dispatches(sys.argv[2], sys.argv[3], int(sys.argv[4])))
    elif sys.argv[1] == "counters":
        print(counters(sys.argv[2], sys.argv[3], int(sys.argv[4])))
    elif sys.argv[1] == "hbm":
        print(hbm(*sys.argv[2:6], int(sys.argv[6])))
    elif sys.argv[1] == "busy":
        print(busy(sys.argv[2], sys.argv[3], float(sys.argv[4]) if len(sys.argv) > 4 else 5.0))
    elif sys.argv[1] == "hash":
        print(gram_source_hash())
