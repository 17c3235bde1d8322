"""Benchmark of the per-tile APIC reconstruction on one MI355X.

Workload (one step = the whole method over one batch): 1024 tiles of
256 x 256 on a 32 x 32 field grid, 16 NA-matched images (ring at NA 0.25) and
32 darkfield images (rings at NA 0.30 and 0.38), Poisson noise at 1e4
photons, float32 inputs resident in HBM, complex64 output on the 2x grid
(512 x 512 per tile).  Metric: output Mpx/s of the batched path; the plain
path (one tile per call, same kernels) is reported beside it.

    python bench.py [--steps K] [--warmup W] [--tiles T] [--no-cpu-baseline]

Prints one JSON line.  Only one GPU is supported.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "APIC output Mpx/s, 1 GPU, batched vs plain, field rel-err ≤1e-4 vs FP64"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FLOP_GROUPS = ("gram", "chol")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per gram launch from the committed counter summary, or None when
    the gram's sources changed since the counters were taken."""
    from paper_2407_20469_amd import pmc_summary
    path = os.path.join(ROOT, "profiles", "gram_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_sha256") != pmc_summary.gram_source_hash():
        return None
    return rec["bytes_per_launch"]


def cpu_baseline(images_host, w):
    """The FP64 oracle on one tile of the same workload, on the host cores."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    geom = oracle.Geometry(**w.geometry_kwargs())
    t0 = time.perf_counter()
    oracle.reconstruct(images_host.astype(np.float64), geom)
    dt = time.perf_counter() - t0
    mpx = (w.n * w.upsample) ** 2 / 1e6
    return {"value": mpx / dt, "unit": "Mpx/s", "cores": int(threads), "kind": "oracle",
            "sample": f"1 tile of the workload (tile 0), full-Q FP64 oracle, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tiles", type=int, default=1024)
    ap.add_argument("--plain-tiles", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the per-tile reconstruction has no "
              "cross-GPU step in this build (tiles shard across GPUs without communication)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import apic_synth as S
    from apic_synth.batch import synth_batch
    from paper_2407_20469_amd import apic

    dev = torch.device("cuda:0")
    w = S.config1(n_tiles=args.tiles)
    log(f"synthesising {w.n_tiles} tiles of {w.n}^2 x {w.n_img} images")
    t0 = time.time()
    images = synth_batch(w, dev, log=log)
    torch.cuda.synchronize()
    log(f"synth done in {time.time() - t0:.1f} s")

    plan = apic.Plan(w.geometry_kwargs())
    plan.upload()
    ws = apic.Workspace()
    nf = w.n * w.upsample
    mpx_step = w.n_tiles * nf * nf / 1e6

    for i in range(args.warmup):
        field, zern, status = apic.reconstruct(plan, images, workspace=ws)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    stream = torch.cuda.current_stream()
    apic.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for i in range(args.steps):
        field, zern, status = apic.reconstruct(plan, images, workspace=ws)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    prof = apic.profile_read()
    apic.profile(False)
    log(f"timed {args.steps} steps: {ms:.1f} ms/step")
    st = status.cpu().numpy()
    bad = int(((st & (apic.TILE_NONFINITE_INPUT | apic.TILE_NONFINITE_OUT)) != 0).sum())

    # plain path: the same kernels, one tile per call
    P = min(args.plain_tiles, w.n_tiles)
    ws1 = apic.Workspace()
    apic.reconstruct(plan, images[:1], workspace=ws1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(P):
        apic.reconstruct(plan, images[t:t + 1], workspace=ws1)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / P
    log(f"plain: {plain_s * 1e3:.1f} ms/tile")

    # executed gram work: live (block pair, E chunk) triples x 16 x 64 x 64 complex MACs
    steps_tab = plan.query(6).reshape(-1, 4)
    gram_exec = w.n_tiles * float(steps_tab[:, 3].sum()) * 16 * 64 * 64 * 8.0
    groups = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps,
                  "work_per_step": v[2] / args.steps} for k, v in prof.items()}
    dom = max(prof, key=lambda k: prof[k][0])
    tot_ms, launches, work = prof[dom]
    if dom in FLOP_GROUPS:
        achieved = work / (tot_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None}
        if dom == "gram":
            roof["executed_tflops"] = gram_exec / (tot_ms / args.steps * 1e-3) / 1e12
            if w.n_tiles == 1024:
                roof["traffic"] = measured_traffic()
    else:
        achieved = work / (tot_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None}

    out = {
        "metric": METRIC, "value": mpx_step / (ms * 1e-3), "unit": "Mpx/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{w.n_tiles} tiles {w.n}x{w.n}, 16 NA-matched + 32 darkfield "
                               f"(NA 0.25 / 0.30 / 0.38), Poisson 1e4, 2x complex64 output",
                   "tiles": w.n_tiles, "n": w.n, "n_bf": w.n_bf, "n_df": w.n_df,
                   "upsample": w.upsample, "mode": "batched (one call per step)"},
        "plain": {"value": (nf * nf / 1e6) / plain_s, "unit": "Mpx/s", "tiles_timed": P,
                  "ms_per_tile": plain_s * 1e3},
        "nonfinite_tiles": bad,
        "roofline": roof,
        "kernel_groups": groups,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on tile 0")
        out["cpu_baseline"] = cpu_baseline(images[0].cpu().numpy(), w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
