"""Benchmark of the per-tile APIC reconstruction on one MI355X.

Default workload (one step = the whole method over one batch): 1024 tiles of
256 x 256 on a 32 x 32 field grid, 16 NA-matched images (ring at NA 0.25) and
32 darkfield images (rings at NA 0.30 and 0.38), Poisson noise at 1e4
photons, float32 inputs resident in HBM, complex64 output on the 2x grid
(512 x 512 per tile).  Metric: output Mpx/s of the batched path (a prepared
tile batch, chunk sizes picked by the autotuner, the pupil of every tile
chosen between the learned surrogate and the closed-form solve by the
fallback rule).  Reported beside it: the same batch with the surrogate off
(the closed-form batched method, ``closed_form_batch``), a graph replay of
that closed-form step, and the plain path (one tile per call, closed form,
same kernels).  The surrogate is trained on the GPU before the timed region on
the closed-form estimates of 8192 training tiles disjoint from the timed ones;
in the timed step the closed form (coarse-to-fine continuation) runs on
every tile and judges the surrogate's prediction, which is kept where the
fallback rule allows.  The line reports the pupil RMSE against the truth of
the chosen coefficients, the closed form, the single pass of Eq. 10, the
surrogate alone and the closed form seeded by the surrogate (its other mode).
``--no-surrogate`` times the closed-form batch as the main value.

The gram's roofline figure counts the nonzero products of its E-sum (the
algorithmic work, from the plan's sets), with the dense E-sum and the
products the kernels issue beside it.  The default line also carries, each
with its own warmup and step count, the uneven batch (one full pass of the
4096 tiles) and the slide stream over its first 128 scanned tiles, while the
whole run stays within its time budget (``--no-extra`` skips them), and the
FP64 oracle timed over 16 tiles in a pool of one process per host core
(run before the GPU is touched; ``--no-cpu-baseline`` skips it).

``--workload uneven`` runs the uneven batch instead: 4096 tiles, 128/256/512 px
in the ratio 4:3:1, 8/12/16 NA-matched LEDs with twice as many darkfield, 40%
background tiles, nine geometry classes run concurrently in chunks that fit
``--ws-gb`` of workspace.

``--workload rgb`` runs a stained slide in three colour channels (0.63, 0.52
and 0.47 um; 256 px tiles, 8 NA-matched + 16 darkfield LEDs per channel) as
one batch of three geometry classes, then the colour combination.

``--workload surrogate`` runs the learned surrogate's own workload: the
surrogate is trained on the closed-form estimates (coarse-to-fine
continuation) of 16384 content tiles of the uneven recipe (nine classes,
NA-matched images only, uniform random field positions; labels whose
linearised residual exceeds 1 rad^2 are left out), then the 4096-tile
uneven batch with 70% background tiles and all darkfield images runs twice:
closed form only, and with the surrogate and its fallback rule (the closed
form replaces the surrogate where the surrogate's residual exceeds the closed
form's by more than 0.05 rad and the closed form is trustworthy).  The line's
value is the pupil RMSE against the truth of the chosen coefficients; beside
it the closed form's, the surrogate's alone, each split into background and
content tiles, and both passes' output rates.

``--workload slide`` streams a slide: 512 px tiles (16 + 32 images) whose image
stacks sit in pinned host memory, reconstructed in chunks through device
staging buffers on several streams, background tiles skipped by their
intensity variance, the pupil chosen by the surrogate with the closed-form
fallback.  The rate is host wall-clock including the host-device copies; the
sample is the first ``--tiles`` scanned tiles of the raster order (default
256).

    python bench.py [--steps K] [--warmup W] [--workload grid|uneven|slide|rgb|surrogate] [--tiles T]
                    [--no-autotune] [--no-surrogate] [--no-cpu-baseline] [--no-extra]

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


def run_env():
    """Software and hardware the line was measured on."""
    import torch
    from paper_2407_20469_amd import apic
    return {"device": torch.cuda.get_device_name(0), "hip": torch.version.hip,
            "torch": torch.__version__, "library": apic.load_library().apic_version().decode(),
            "host_cores": len(os.sched_getaffinity(0))}


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


def _oracle_tile(job):
    """One tile of the FP64 oracle in a worker process (BLAS threads = 1):
    its own forward model and Poisson draw, then the whole reconstruction."""
    import numpy as np
    import oracle
    w, t, photons = job
    k_all = list(w.k_bf) + list(w.k_df)
    img = oracle.forward_images(w.object(t), k_all, w.coeffs[t], w.r)
    img = np.random.default_rng([w.seed_id, 1, t]).poisson(img * photons) / photons
    img = img.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    oracle.reconstruct(img, oracle.Geometry(**w.geometry_kwargs()))
    return time.perf_counter() - t0


def cpu_baseline_pool(w, n_sample=None):
    """The FP64 oracle (full-Q gram, as it stands) over a seeded subset of the
    workload's tiles (tiles 0 .. n_sample-1, images from the oracle's own
    forward model with Poisson noise at the workload's photon level), one tile
    per worker process with one BLAS thread each, a pool over every host core.
    Runs before the GPU is touched: the workers are spawned processes."""
    import multiprocessing as mp
    cores = len(os.sched_getaffinity(0))
    n_sample = n_sample or max(8, min(16, cores))
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(min(cores, n_sample)) as pool:
        per = pool.map(_oracle_tile, [(w, t, w.photons) for t in range(n_sample)])
    wall = time.perf_counter() - t0
    mpx = n_sample * (w.n * w.upsample) ** 2 / 1e6
    return {"value": mpx / wall, "unit": "Mpx/s", "cores": min(cores, n_sample), "kind": "oracle",
            "sample": f"tiles 0..{n_sample - 1} of the workload (oracle forward model, Poisson "
                      f"1e4), full-Q FP64 oracle, one tile per process with BLAS threads = 1, "
                      f"pool of {min(cores, n_sample)} processes on {cores} host cores: "
                      f"{wall:.1f} s wall",
            "per_tile_s_in_pool": {"mean": sum(per) / len(per), "max": max(per)},
            "extrapolated_s_for_workload": wall * w.n_tiles / n_sample,
            "extrapolation": f"linear in tiles: {w.n_tiles} / {n_sample} x the pool's wall time"}


def gram_nonzero_flops(plan, geom):
    """FP64 flops per tile of the nonzero products of the T-E gram's E-sum:
    for each darkfield step and each excluded k, the n_k unknowns u with u + k
    in P give n_k (n_k + 1) / 2 complex MACs of the Hermitian lower triangle,
    8 flops each (counted from the plan's U, P and E tables)."""
    import numpy as np
    n = plan.geoms[geom]["n"]
    h = n // 2
    total = 0.0
    for j in range(plan.geoms[geom]["n_df"]):
        u = plan.query(0, geom, j).reshape(-1, 2).astype(np.int64)
        if len(u) == 0:
            continue
        p = plan.query(1, geom, j).reshape(-1, 2).astype(np.int64)
        e = plan.query(3, geom, j).reshape(-1, 2).astype(np.int64)
        pm = np.zeros((n, n), bool)
        pm[p[:, 0] % n, p[:, 1] % n] = True
        for s in range(0, len(e), 256):
            ky = u[None, :, 0] + e[s:s + 256, None, 0]
            kx = u[None, :, 1] + e[s:s + 256, None, 1]
            ok = (ky >= -h) & (ky < h) & (kx >= -h) & (kx < h)
            nk = (ok & pm[ky % n, kx % n]).sum(axis=1).astype(np.float64)
            total += float((nk * (nk + 1) / 2).sum()) * 8.0
    return total


def pixel_pupil_timing(plan, images, w, chunk=512):
    """The pixel-domain pupil solve (Eq. 10, one unknown per pupil pixel) and
    the Zernike-basis solve over every tile of a single-class workload whose
    image stacks are contiguous in ``images``, in calls of ``chunk`` tiles;
    HIP events on the launch stream.  KK is included in both."""
    import numpy as np
    import torch
    from paper_2407_20469_amd import apic
    per = w.n_img * w.n * w.n
    T = w.n_tiles
    views = [images[c0 * per:(c0 + min(chunk, T - c0)) * per].view(-1, w.n_img, w.n, w.n)
             for c0 in range(0, T, chunk)]
    ws = apic.Workspace()
    apic.estimate_pupil_pixel(plan, views[0], workspace=ws)
    apic.estimate_pupil(plan, views[0], workspace=ws)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    out = [apic.estimate_pupil_pixel(plan, v, workspace=ws) for v in views]
    ev[1].record()
    for v in views:
        apic.estimate_pupil(plan, v, workspace=ws)
    ev[2].record()
    torch.cuda.synchronize()
    its = np.concatenate([o[2].cpu().numpy() for o in out])
    st = np.concatenate([o[3].cpu().numpy() for o in out])
    return {"tiles": T, "chunk": chunk, "ms": ev[0].elapsed_time(ev[1]),
            "ms_zernike_basis": ev[1].elapsed_time(ev[2]),
            "mean_iterations": float(its.mean()), "max_iterations": int(its.max()),
            "not_converged": int(((st & apic.TILE_PIXEL_NOT_CONVERGED) != 0).sum()),
            "pixels": int(plan.sizes()["n_pix"]), "rows": int(plan.sizes()["n_rows"])}


def assembly_timing(field, w, overlap=64, ramp=32.0):
    """Phase alignment and blend of the workload's output fields placed on its
    field grid as a field of view with ``overlap`` output pixels shared by
    neighbours (the fields are independent tiles, so this times the data
    movement, not the seams).  Blend: HIP events on the launch stream;
    algorithmic bytes = every tile read once + the canvas written once."""
    import numpy as np
    import torch
    from paper_2407_20469_amd import apic
    nf = w.n * w.upsample
    T = w.n_tiles
    side = int(round(np.sqrt(T)))
    stride = nf - overlap
    pos = np.array([((t // side) * stride, (t % side) * stride) for t in range(T)], np.int32)
    H = W = (side - 1) * stride + nf
    f = field.view(T, nf, nf)
    t0 = time.perf_counter()
    asm = apic.Assembly(nf, pos, (H, W))
    prep_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    theta = torch.tensor(asm.phases(f), device=f.device)
    phase_ms = (time.perf_counter() - t0) * 1e3
    canvas = asm.blend(f, theta, ramp)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(5):
        asm.blend(f, theta, ramp, out=canvas)
    ev[1].record()
    torch.cuda.synchronize()
    blend_ms = ev[0].elapsed_time(ev[1]) / 5
    asm.close()
    nbytes = T * nf * nf * 8 + H * W * 8
    return {"tiles": T, "canvas": [H, W], "overlap_px": overlap, "ramp": ramp,
            "blend_ms": blend_ms, "blend_GBps": nbytes / (blend_ms * 1e-3) / 1e9,
            "blend_frac_of_8TBps": nbytes / (blend_ms * 1e-3) / 8e12,
            "prepare_ms_host": prep_ms, "phases_ms_host": phase_ms}


def fit_surrogate(x, y, seed, epochs=200):
    """Train the surrogate on inputs x (T, 34) and Noll 4..15 labels y (T, 12),
    both device tensors: standardised inputs and labels, with the labels'
    de-standardisation folded exactly into the last layer afterwards.
    Returns (surrogate, first loss, mean of the last 8 losses)."""
    import numpy as np
    import torch
    from paper_2407_20469_amd import apic
    rng = np.random.default_rng(seed)
    n = x.shape[0]
    y_mean, y_std = y.mean(0), y.std(0) + 1e-6
    mean = x.mean(0).cpu().numpy()
    std = x.std(0).cpu().numpy() + 1e-6
    sur = apic.Surrogate(apic.init_mlp_params(seed), mean, std, device=x.device)
    order = np.concatenate([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)
    loss = sur.train(x, ((y - y_mean) / y_std).contiguous(), order, batch=128,
                     lr=1e-3).cpu().numpy()
    th = sur.theta.cpu().numpy().astype(np.float64)
    o3 = 128 * 64 + 128 + 128 * 128 + 128
    w3 = th[o3:o3 + 16 * 128].reshape(16, 128)
    b3 = th[o3 + 16 * 128:o3 + 16 * 128 + 16]
    ym, ys = y_mean.cpu().numpy(), y_std.cpu().numpy()
    w3[:12] *= ys[:, None]
    b3[:12] = b3[:12] * ys + ym
    sur = apic.Surrogate(th.astype(np.float32), mean, std, device=x.device)
    return sur, float(loss[0]), float(loss[-8:].mean())


def train_slide_surrogate(dev, n_train=512, seed=41):
    """Surrogate for the 512 px slide geometry, trained on the GPU on the
    closed-form pupil estimates of brightfield-only content tiles at random
    field positions (the surrogate's inputs come from the NA-matched images
    only)."""
    import numpy as np
    import torch
    import apic_synth.surrogate_set as SS
    from paper_2407_20469_amd import apic
    rng = np.random.default_rng(seed)
    uv = rng.uniform(-1, 1, (n_train, 2))
    imgs, _ = SS.make_tiles(uv, np.zeros(n_train, bool), seed, dev, max_abs=1.5, chunk=32, n=512)
    plan = apic.Plan(SS.geometry(512))
    z, diag, feat, st = apic.estimate_pupil(plan, imgs)
    del imgs
    x = torch.cat([torch.tensor(uv, dtype=torch.float32, device=dev), feat], dim=1)
    plan.close()
    return fit_surrogate(x, z[:, 3:15].contiguous(), seed)


def grid_training_workload(w, n_train=8192, seed=43):
    """Training tiles for the grid workload's surrogate, disjoint from the
    timed ones: the same geometry without darkfield images (the surrogate's
    inputs and the closed-form labels come from the NA-matched images only),
    objects drawn with their own seed, positions uniform over the field, true
    pupils from the same field model (its quadratic coefficients fitted on the
    workload's 32 x 32 grid)."""
    import numpy as np
    import apic_synth as S
    g = np.arange(1024)
    _, a = S.field_model_quadratic((g % 32 - 15.5) / 15.5, (g // 32 - 15.5) / 15.5)
    uv = np.random.default_rng([seed, 2, 0]).uniform(-1.0, 1.0, (n_train, 2))
    u, v = uv[:, 0], uv[:, 1]
    c = np.zeros((n_train, 15))
    c[:, 3:] = np.stack([np.ones_like(u), u, v, u * u, u * v, v * v], axis=1) @ a.T
    return S.Workload("grid256-train", w.n, w.k_bf, [], upsample=w.upsample, n_tiles=n_train,
                      photons=w.photons, seed_id=seed, coeffs=c, positions=uv)


def train_grid_surrogate(w, dev, seed=43, trust_quantile=0.4):
    """Surrogate for the grid workload, trained on the GPU on the closed-form
    pupil estimates (coarse-to-fine continuation) of 8192 training tiles
    disjoint from the timed ones, at their field positions, keeping the tiles
    whose solve is best supported (weight sum above the given quantile).
    Returns (surrogate, summary)."""
    import torch
    from apic_synth.batch import synth_batch
    from paper_2407_20469_amd import apic
    wt = grid_training_workload(w, seed=seed)
    imgs = synth_batch(wt, dev)
    plan = apic.Plan(wt.geometry_kwargs())
    z, diag, feat, st = apic.estimate_pupil(plan, imgs)
    del imgs
    x = torch.cat([torch.tensor(wt.positions, dtype=torch.float32, device=dev), feat], dim=1)
    sw = diag[:, 2]
    keep = sw >= torch.quantile(sw, trust_quantile)
    sur, l0, l1 = fit_surrogate(x[keep].contiguous(), z[keep, 3:15].contiguous(), seed,
                                epochs=150)
    import numpy as np
    err = z.cpu().numpy()[:, 3:] - wt.coeffs[:, 3:]
    note = {"trained_on": f"closed-form estimates of {int(keep.sum())} best-supported of "
                          f"{wt.n_tiles} training tiles disjoint from the timed ones "
                          f"(own objects and noise, uniform random field positions)",
            "label_rmse_vs_truth": float(np.sqrt(np.mean(np.sum(err * err, axis=1)))),
            "loss_first": l0, "loss_last": l1, "seeds_solve": False}
    plan.close()
    return sur, note


def pupil_accuracy(plan_geom, images, w, z_chosen, sur, pos, dev):
    """Pupil RMSE against the truth (sqrt of the mean over tiles of
    sum_j (c_j - c_true_j)^2, Noll 4..15) on the timed tiles: the step's chosen
    coefficients, the closed form (continuation), the single pass of Eq. 10,
    the surrogate alone and the closed form seeded by the surrogate."""
    import numpy as np
    from paper_2407_20469_amd import apic
    stack = images[:w.n_tiles * w.n_img * w.n * w.n].view(w.n_tiles, w.n_img, w.n, w.n)
    truth = w.coeffs[:, 3:]

    def rmse(z):
        d = z.cpu().numpy()[:, 3:15] - truth
        return float(np.sqrt(np.mean(np.sum(d * d, axis=1))))

    out = {"chosen_in_timed_step": rmse(z_chosen)}
    cf, _, _, _ = apic.estimate_pupil(apic.Plan(plan_geom), stack)
    out["closed_form_continuation"] = rmse(cf)
    one, _, _, _ = apic.estimate_pupil(apic.Plan({**plan_geom, "pupil_bands": 0}), stack)
    out["closed_form_single_pass"] = rmse(one)
    if sur is not None:
        mode = sur.seeds_solve
        sur.seeds_solve = True
        _, zcf, zs, _, _ = apic.estimate_pupil_sur(apic.Plan(plan_geom), stack, pos, sur)
        sur.seeds_solve = mode
        out["surrogate_alone"] = rmse(zs)
        out["closed_form_seeded_by_surrogate"] = rmse(zcf)
    out["unit"] = "rad"
    return out


def slide_stream(args, dev, tiles, steps, warmup):
    """Slide stream (see the module docstring) over the first ``tiles``
    scanned tiles; returns the record."""
    import numpy as np
    import torch
    from apic_synth import slide
    from apic_synth.batch import synth_batch
    from paper_2407_20469_amd import apic

    p_tissue, p_glass = 16, 4
    w = slide.pool_workload(p_tissue, p_glass)
    mask = slide.slide_mask()
    idx, src = slide.scan_order(mask, tiles, p_tissue, p_glass)
    T = len(idx)
    log(f"slide {mask.shape[0]} x {mask.shape[1]} tiles, {mask.mean():.2f} tissue; "
        f"streaming the first {T} scanned tiles from a pool of {w.n_tiles}")
    t0 = time.time()
    pool_dev = synth_batch(w, dev, log=log)
    pool = torch.empty(pool_dev.shape, dtype=torch.float32).pin_memory()
    pool.copy_(pool_dev)
    del pool_dev
    nf = w.n * w.upsample
    ring = args.chunk * (args.buffers + 1)   # more than the tiles in flight
    fields = [torch.empty((nf, nf), dtype=torch.complex64).pin_memory() for _ in range(ring)]
    log(f"pool synthesised and pinned in {time.time() - t0:.1f} s")
    sur = None
    sur_note = None
    if not args.no_surrogate:
        t0 = time.time()
        sur, l0, l1 = train_slide_surrogate(dev)
        sur_note = {"trained_on": "512 closed-form estimates of 512 px content tiles",
                    "loss_first": l0, "loss_last": l1}
        log(f"surrogate trained in {time.time() - t0:.1f} s (loss {l0:.4f} -> {l1:.5f})")
    plan = apic.Plan(w.geometry_kwargs())
    plan.upload()
    st = apic.Streamer(plan, 0, chunk=args.chunk, n_buffers=args.buffers)
    log(f"streamer: chunk {args.chunk}, {args.buffers} buffers, "
        f"{st.device_bytes / 2 ** 30:.1f} GiB device staging")
    host_imgs = [pool[int(k)] for k in src]
    host_flds = [fields[t % ring] for t in range(T)]
    pos = w.positions[src].astype(np.float32)

    def run(n):
        return st.run(host_imgs[:n], host_flds[:n], positions=pos[:n], sur=sur,
                      bg_threshold=args.bg_threshold)

    for i in range(warmup):
        run(min(T, 2 * args.chunk))
        log(f"warmup {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    times = []
    for i in range(steps):
        t0 = time.perf_counter()
        z, status, stat = run(T)
        times.append(time.perf_counter() - t0)
        log(f"stream pass {i + 1}/{steps}: {times[-1]:.2f} s")
    wall = float(np.median(times))
    skipped = (status & apic.TILE_BACKGROUND) != 0
    rec = int((~skipped).sum())
    mpx = rec * nf * nf / 1e6
    used = float(((status & apic.TILE_SURROGATE_USED) != 0)[~skipped].mean()) if rec else 0.0
    bad = int(((status & (apic.TILE_NONFINITE_INPUT | apic.TILE_NONFINITE_OUT)) != 0).sum())
    h2d = T * w.n_img * w.n * w.n * 4
    d2h = rec * nf * nf * 8

    # the same kernels on device-resident tiles: one chunk of tiles (the pool's
    # tissue tiles, cycled) per call
    res = np.arange(args.chunk) % p_tissue
    dev_imgs = pool[torch.as_tensor(res)].to(dev)
    posd = torch.tensor(w.positions[res], dtype=torch.float32, device=dev)
    ws = apic.Workspace()
    call = (lambda: apic.reconstruct_sur(plan, dev_imgs, posd, sur, workspace=ws)) if sur \
        else (lambda: apic.reconstruct(plan, dev_imgs, workspace=ws))
    call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    call()
    torch.cuda.synchronize()
    resident_ms = (time.perf_counter() - t0) * 1e3 / args.chunk

    out = {
        "metric": METRIC, "value": mpx / wall, "unit": "Mpx/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": wall * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"slide stream: first {T} scanned 512x512 tiles (16 NA-matched + "
                               f"32 darkfield, Poisson 1e4) of a 76 x 25 mm slide with 30% "
                               f"tissue, from pinned host memory, 2x complex64 output to "
                               f"pinned host memory",
                   "scanned": T, "reconstructed": rec, "background_skipped": int(skipped.sum()),
                   "chunk": args.chunk, "buffers": args.buffers,
                   "bg_threshold": args.bg_threshold, "surrogate": sur is not None},
        "timing": "host wall-clock of whole stream passes (median), host-device copies included",
        "tiles_per_s": T / wall,
        "pcie": {"h2d_GBps": h2d / wall / 1e9, "d2h_GBps": d2h / wall / 1e9},
        "resident_ms_per_tile": resident_ms,
        "stream_ms_per_reconstructed_tile": wall * 1e3 / max(rec, 1),
        "surrogate": sur_note, "surrogate_used_frac": used,
        "slide_extrapolation": {"scanned_tiles_first_20000_raster": int(mask.ravel()[:20000].sum()),
                                "est_s": float(mask.ravel()[:20000].sum()) * wall / T},
        "nonfinite_tiles": bad,
        "env": run_env(),
    }
    st.close()
    plan.close()
    return out


def run_slide_stream(args, dev):
    print(json.dumps(slide_stream(args, dev, args.tiles, args.steps, args.warmup)), flush=True)


def synth_into(ws_list, order, plan, dev):
    """Synthesise every class of a batch into one flat image buffer laid out by
    the plan's mixed descriptors.  Returns (descs, images, field elements)."""
    import numpy as np
    import torch
    from apic_synth.batch import synth_batch
    from paper_2407_20469_amd import apic
    n_total = sum(w.n_tiles for w in ws_list)
    cls_of = np.zeros(n_total, np.int64)
    for ci, idx in enumerate(order):
        cls_of[idx] = ci
    descs, n_img_el, n_fld_el = apic.mixed_descs(plan, cls_of)
    images = torch.empty(n_img_el, dtype=torch.float32, device=dev)
    for ci, w in enumerate(ws_list):
        log(f"synthesising class {ci}: {w.n_tiles} tiles of {w.n}^2 x {w.n_img} images")
        imgs = synth_batch(w, dev, log=log)
        per = w.n_img * w.n * w.n
        for p_, b in enumerate(order[ci]):
            o = descs[int(b)].image_offset
            images[o:o + per] = imgs[p_].reshape(-1)
        del imgs
    torch.cuda.synchronize()
    return descs, images, n_fld_el


def timed_steps(fn, steps, stream):
    """HIP events on ``stream`` around ``steps`` calls of fn; ms per call."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def uneven_block(dev, ws_gb, warmup=1, steps=1):
    """The uneven batch (4096 tiles, nine geometry classes, closed form) with
    its own warmup and timed passes; chunks fitted to a workspace budget
    without the autotuner's timing runs."""
    import numpy as np
    import torch
    import apic_synth as S
    from paper_2407_20469_amd import apic
    t_start = time.time()
    ws_list = S.uneven_batch(n_tiles=4096)
    order = [w.extra["tiles"] for w in ws_list]
    plan = apic.Plan([w.geometry_kwargs() for w in ws_list])
    plan.upload()
    descs, images, n_fld = synth_into(ws_list, order, plan, dev)
    n_total = sum(w.n_tiles for w in ws_list)
    mpx = sum(w.n_tiles * (w.n * w.upsample) ** 2 for w in ws_list) / 1e6
    field = torch.empty(n_fld, dtype=torch.complex64, device=dev)
    zern = torch.empty((n_total, 15), dtype=torch.float32, device=dev)
    status = torch.empty((n_total,), dtype=torch.int32, device=dev)
    batch = apic.Batch(plan, descs)
    batch.fit(int(ws_gb * 2 ** 30))
    ws = apic.Workspace()
    log(f"uneven: {len(ws_list)} classes, workspace {batch.workspace_bytes / 2 ** 30:.1f} GiB, "
        f"synth + setup {time.time() - t_start:.1f} s")
    for i in range(warmup):
        batch.reconstruct(images, field, zern, status, ws)
        torch.cuda.synchronize()
        log(f"uneven warmup {i + 1}/{warmup} done")
    ms = timed_steps(lambda: batch.reconstruct(images, field, zern, status, ws), steps,
                     torch.cuda.current_stream())
    st = status.cpu().numpy()
    rec = {"value": mpx / (ms * 1e-3), "unit": "Mpx/s", "steps": steps, "warmup": warmup,
           "ms_per_step": ms,
           "workload": f"uneven batch of {n_total} tiles: 128/256/512 px (4:3:1), 8/12/16 "
                       f"NA-matched + 2x darkfield, 40% background, Poisson 1e4, 2x complex64 "
                       f"output",
           "mode": "prepared batch, nine classes on concurrent streams, closed form, chunks "
                   "fitted to the workspace budget",
           "classes": [[w.n, w.n_bf, w.n_df, w.n_tiles, c["chunk"], c["lanes"]]
                       for w, c in zip(ws_list, batch.classes())],
           "workspace_gib": batch.workspace_bytes / 2 ** 30,
           "nonfinite_tiles": int(((st & (apic.TILE_NONFINITE_INPUT
                                         | apic.TILE_NONFINITE_OUT)) != 0).sum()),
           "block_wall_s": None}
    batch.close()
    del images, field, ws
    torch.cuda.empty_cache()
    rec["block_wall_s"] = time.time() - t_start
    log(f"uneven: {ms / 1e3:.1f} s per pass, {rec['value']:.1f} Mpx/s")
    return rec


def surrogate_workload(args, dev):
    """The learned surrogate's workload (see the module docstring).  Returns
    the JSON record."""
    import numpy as np
    import torch
    import apic_synth as S
    from apic_synth.batch import synth_batch
    from paper_2407_20469_amd import apic
    t_start = time.time()
    # training: the closed-form estimates of the training tiles, class by class
    # a label is kept when the closed form trusts itself by the fallback rule's
    # own bound: its linearised residual R(c) at most resid_max = 1 rad^2
    xs, ys, rs, lab_err = [], [], [], []
    tr = S.surrogate_train_batch(args.train_tiles)
    for w in tr:
        imgs = synth_batch(w, dev)
        plan = apic.Plan(w.geometry_kwargs())
        z, diag, feat, _ = apic.estimate_pupil(plan, imgs)
        del imgs
        plan.close()
        pos = torch.tensor(w.positions, dtype=torch.float32, device=dev)
        xs.append(torch.cat([pos, feat], dim=1))
        ys.append(z[:, 3:15])
        rs.append(diag[:, 0])
        lab_err.append(z.cpu().numpy()[:, 3:15] - w.coeffs[:, 3:15])
        log(f"training labels: class {w.name}, {w.n_tiles} tiles")
    torch.cuda.empty_cache()
    x, y, resid = torch.cat(xs), torch.cat(ys), torch.cat(rs)
    ok = torch.isfinite(x).all(1) & torch.isfinite(y).all(1) & (resid <= 1.0)
    lab_err = np.concatenate(lab_err)
    ok_np = ok.cpu().numpy()
    t_lab = time.time() - t_start
    t0 = time.time()
    sur, l0, l1 = fit_surrogate(x[ok].contiguous(), y[ok].contiguous(), seed=47,
                                epochs=args.epochs)
    torch.cuda.synchronize()
    t_fit = time.time() - t0
    log(f"surrogate: labels {t_lab:.1f} s, fit {t_fit:.1f} s on {int(ok.sum())} of "
        f"{len(ok_np)} tiles "
        f"(loss {l0:.4f} -> {l1:.5f})")
    del xs, ys, x, y

    # evaluation: the uneven batch with 70% background, closed form, then with
    # the surrogate and the fallback rule
    ev = S.surrogate_eval_batch(args.tiles)
    order = [w.extra["tiles"] for w in ev]
    plan = apic.Plan([w.geometry_kwargs() for w in ev])
    plan.upload()
    descs, images, n_fld = synth_into(ev, order, plan, dev)
    T = sum(w.n_tiles for w in ev)
    truth, bg, pos = np.zeros((T, 15)), np.zeros(T, bool), np.zeros((T, 2))
    for w, idx in zip(ev, order):
        truth[idx], bg[idx], pos[idx] = w.coeffs, w.extra["background"], w.positions
    pos_dev = torch.tensor(pos, dtype=torch.float32, device=dev)
    mpx = sum(w.n_tiles * (w.n * w.upsample) ** 2 for w in ev) / 1e6
    field = torch.empty(n_fld, dtype=torch.complex64, device=dev)
    zern = torch.empty((T, 15), dtype=torch.float32, device=dev)
    status = torch.empty((T,), dtype=torch.int32, device=dev)
    batch = apic.Batch(plan, descs)
    batch.fit(int(args.ws_gb * 2 ** 30))
    ws = apic.Workspace()
    stream = torch.cuda.current_stream()
    cf_ms = timed_steps(lambda: batch.reconstruct(images, field, zern, status, ws), 1, stream)
    z_cf = zern.cpu().numpy().astype(np.float64)
    log(f"closed-form pass: {cf_ms / 1e3:.1f} s")
    batch.set_surrogate(sur, pos_dev, rho_max=0.05, kappa_max=1e6, resid_max=1.0)
    sur_ms = timed_steps(lambda: batch.reconstruct(images, field, zern, status, ws), 1, stream)
    z_ch = zern.cpu().numpy().astype(np.float64)
    st = status.cpu().numpy()
    log(f"surrogate pass: {sur_ms / 1e3:.1f} s")
    batch.close()
    del field, ws
    # the surrogate alone, from the features of each class's NA-matched images
    z_sur = np.zeros((T, 15))
    for w, idx in zip(ev, order):
        per = w.n_img * w.n * w.n
        stack = torch.stack([images[descs[int(b)].image_offset:descs[int(b)].image_offset + per]
                             .view(w.n_img, w.n, w.n)[:w.n_bf] for b in idx])
        pl = apic.Plan({**w.geometry_kwargs(), "k_df": np.zeros((0, 2), np.int64)})
        _, _, feat, _ = apic.estimate_pupil(pl, stack)
        pl.close()
        del stack
        z_sur[idx, 3:15] = sur.forward(torch.cat([pos_dev[idx], feat], dim=1)).cpu().numpy()
    del images
    torch.cuda.empty_cache()

    def err(z, sel=None, ref=truth):
        d = (z - ref)[:, 3:15]
        if sel is not None:
            d = d[sel]
        return np.sqrt(np.sum(d * d, axis=1))

    def rmse(z, sel=None, ref=truth):
        return float(np.sqrt(np.mean(err(z, sel, ref) ** 2)))

    split = {"all": None, "background": bg, "content": ~bg}
    cands = (("chosen", z_ch), ("closed_form", z_cf), ("surrogate_alone", z_sur))
    acc = {name: {k: rmse(z, sel) for k, sel in split.items()} for name, z in cands}
    acc["surrogate_vs_closed_form"] = {k: rmse(z_sur, sel, z_cf) for k, sel in split.items()}
    med = {name: {k: float(np.median(err(z, sel))) for k, sel in split.items()}
           for name, z in cands}
    kept = (st & apic.TILE_SURROGATE_USED) != 0
    log(f"pupil RMSE vs truth: {acc}")
    log(f"median error vs truth: {med}")
    w_desc = (f"learned surrogate on uneven-recipe tiles: trained on the closed-form estimates "
              f"of {args.train_tiles} content tiles (128/256/512 px 4:3:1, 8/12/16 NA-matched "
              f"LEDs, random field positions, quadratic field model up to 1.5 rad, Poisson 1e4); "
              f"evaluated on {T} tiles of the same recipe with 70% background and 2x darkfield "
              f"images, fallback at 0.05 rad")
    return {"metric": "pupil RMSE vs truth, surrogate with closed-form fallback",
            "value": acc["chosen"]["all"], "unit": "rad", "n_gpus": 1, "steps": 1, "warmup": 0,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16 MLP (fp32 accumulate) + f32/f64 closed form", "data": "synthetic",
            "config": {"workload": w_desc},
            "accuracy_rad": acc,
            "accuracy_note": "RMSE over tiles of the Noll 4..15 error norm; median_rad: the "
                             "median of that norm",
            "median_rad": med,
            "label_rmse_vs_truth": {
                "all": float(np.sqrt(np.mean(np.sum(lab_err ** 2, axis=1)))),
                "kept": float(np.sqrt(np.mean(np.sum(lab_err[ok_np] ** 2, axis=1))))},
            "training": {"tiles": int(ok.sum()), "of": int(len(ok_np)),
                         "rule": "closed-form labels with R(c) <= 1 rad^2",
                         "epochs": args.epochs, "loss_first": l0,
                         "loss_last": l1, "labels_s": t_lab, "fit_s": t_fit},
            "decisions": {"surrogate_kept": int(kept.sum()),
                          "closed_form_kept": int(((st & apic.TILE_FALLBACK_USED) != 0).sum()),
                          "surrogate_kept_background": int((kept & bg).sum()),
                          "surrogate_kept_content": int((kept & ~bg).sum())},
            "rate_Mpx_s": {"closed_form": mpx / (cf_ms * 1e-3),
                           "with_surrogate": mpx / (sur_ms * 1e-3)},
            "wall_s": time.time() - t_start}


def main():
    t_start = time.time()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["grid", "uneven", "slide", "rgb", "surrogate"],
                    default="grid")
    ap.add_argument("--train-tiles", type=int, default=16384, help="surrogate: training tiles")
    ap.add_argument("--epochs", type=int, default=150, help="surrogate: training epochs")
    ap.add_argument("--tiles", type=int, default=None)
    ap.add_argument("--ws-gb", type=float, default=128.0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--graph", dest="graph", action="store_true", default=None)
    ap.add_argument("--no-graph", dest="graph", action="store_false")
    ap.add_argument("--plain-tiles", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="grid: skip the uneven-batch and slide-stream blocks")
    ap.add_argument("--side-steps", type=int, default=5,
                    help="grid: timed steps of the side measurements (closed form, graph)")
    ap.add_argument("--chunk", type=int, default=64, help="slide: tiles per staged chunk")
    ap.add_argument("--buffers", type=int, default=3, help="slide: staging buffers / streams")
    ap.add_argument("--bg-threshold", type=float, default=3e-3,
                    help="slide: background statistic threshold")
    ap.add_argument("--no-surrogate", action="store_true")
    args = ap.parse_args()
    if args.tiles is None:
        args.tiles = {"grid": 1024, "uneven": 4096, "slide": 256, "rgb": 256,
                      "surrogate": 4096}[args.workload]
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the per-tile reconstruction has no "
              "cross-GPU step (tiles shard across GPUs without communication)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import apic_synth as S

    # the oracle's pool runs first, in spawned processes, before anything
    # touches the GPU
    cpu_base = None
    if args.workload == "grid" and not args.no_cpu_baseline:
        log("cpu baseline: FP64 oracle over a tile subset, one process per core")
        cpu_base = cpu_baseline_pool(S.grid_batch(n_tiles=args.tiles))
        log(f"cpu baseline: {cpu_base['sample']}")

    import torch
    from paper_2407_20469_amd import apic

    dev = torch.device("cuda:0")
    if args.workload == "slide":
        return run_slide_stream(args, dev)
    if args.workload == "surrogate":
        print(json.dumps(surrogate_workload(args, dev)), flush=True)
        return
    if args.workload == "grid":
        ws_list = [S.grid_batch(n_tiles=args.tiles)]
        order = [np.arange(ws_list[0].n_tiles)]
    elif args.workload == "rgb":
        from apic_synth.rgb import config_rgb
        ws_list = config_rgb(n_tiles=args.tiles, n=256)
        order = [np.arange(args.tiles) * 3 + c for c in range(3)]   # tile-major R, G, B
    else:
        ws_list = S.uneven_batch(n_tiles=args.tiles or 4096)
        order = [w.extra["tiles"] for w in ws_list]
    n_total = sum(w.n_tiles for w in ws_list)
    plan = apic.Plan([w.geometry_kwargs() for w in ws_list])
    plan.upload()
    t0 = time.time()
    descs, images, n_fld_el = synth_into(ws_list, order, plan, dev)
    log(f"synth done in {time.time() - t0:.1f} s")
    mpx_step = sum(w.n_tiles * (w.n * w.upsample) ** 2 for w in ws_list) / 1e6

    field = torch.empty(n_fld_el, dtype=torch.complex64, device=dev)
    zern = torch.empty((n_total, 15), dtype=torch.float32, device=dev)
    status = torch.empty((n_total,), dtype=torch.int32, device=dev)
    batch = apic.Batch(plan, descs)
    sur = sur_note = sur_pos = None
    if args.workload == "grid" and not args.no_surrogate:
        t0 = time.time()
        sur, sur_note = train_grid_surrogate(ws_list[0], dev)
        sur_pos = torch.tensor(ws_list[0].positions, dtype=torch.float32, device=dev)
        batch.set_surrogate(sur, sur_pos)
        torch.cuda.synchronize()
        log(f"surrogate trained in {time.time() - t0:.1f} s (loss {sur_note['loss_first']:.4f} "
            f"-> {sur_note['loss_last']:.5f}; label RMSE vs truth "
            f"{sur_note['label_rmse_vs_truth']:.4f} rad)")
    budget = int(args.ws_gb * 2 ** 30)
    tune = None
    if not args.no_autotune:
        full = batch.workspace_bytes
        cap = min(full, budget)
        buf = torch.empty(cap + 256, dtype=torch.uint8, device=dev)
        t0 = time.time()
        ms_tile = batch.autotune(images, field, zern, status, (buf.data_ptr() + 255) & ~255, cap,
                                 slack=0.0, log=log)
        del buf
        tune = [{"geom": c["geom"], "tiles": c["n_tiles"], "chunk": c["chunk"],
                 "lanes": c["lanes"], "fft_variant": c.get("fft_variant"),
                 "fft_panel_columns": c.get("fft_panel_columns"), "ms_per_tile": float(m)}
                for c, m in zip(batch.classes(), ms_tile)]
        log(f"autotune {time.time() - t0:.1f} s: (geom, tiles, chunk, lanes, fft variant) "
            f"{[(c['geom'], c['tiles'], c['chunk'], c['lanes'], c['fft_variant']) for c in tune]}")
    elif batch.workspace_bytes > budget:
        batch.fit(budget)
    ws = apic.Workspace()
    log(f"workspace {batch.workspace_bytes / 2 ** 30:.1f} GiB")

    for i in range(args.warmup):
        batch.reconstruct(images, field, zern, status, ws)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    stream = torch.cuda.current_stream()
    apic.profile(True)
    ms = timed_steps(lambda: batch.reconstruct(images, field, zern, status, ws), args.steps,
                     stream)
    prof = apic.profile_read()
    apic.profile(False)
    log(f"timed {args.steps} steps: {ms:.1f} ms/step")
    st = status.cpu().numpy()
    bad = int(((st & (apic.TILE_NONFINITE_INPUT | apic.TILE_NONFINITE_OUT)) != 0).sum())
    if sur_note is not None:
        sur_note["surrogate_kept"] = int(((st & apic.TILE_SURROGATE_USED) != 0).sum())
        sur_note["closed_form_kept"] = int(((st & apic.TILE_FALLBACK_USED) != 0).sum())
        log(f"surrogate kept on {sur_note['surrogate_kept']} tiles, closed form on "
            f"{sur_note['closed_form_kept']}")
    accuracy = None
    if args.workload == "grid":
        accuracy = pupil_accuracy(ws_list[0].geometry_kwargs(), images, ws_list[0], zern, sur,
                                  sur_pos, dev)
        log(f"pupil RMSE vs truth: {accuracy}")

    # the closed-form batch (surrogate off) on the same tiles, timed the same
    # way after the surrogate step: the plain batched method beside it
    closed_form = None
    side = max(1, min(args.side_steps, args.steps))
    if sur_note is not None:
        batch.set_surrogate(None, None)
        batch.reconstruct(images, field, zern, status, ws)
        cf_ms = timed_steps(lambda: batch.reconstruct(images, field, zern, status, ws), side,
                            stream)
        closed_form = {"value": mpx_step / (cf_ms * 1e-3), "unit": "Mpx/s", "ms_per_step": cf_ms,
                       "steps": side}
        log(f"closed-form batch (surrogate off): {cf_ms:.1f} ms/step")

    # a step captured into a graph and replayed: the closed-form batch, since
    # graphs are offered for one-lane batches without the surrogate
    graph_ms = None
    want_graph = args.graph if args.graph is not None else args.workload == "grid"
    if want_graph and any(c["lanes"] != 1 for c in batch.classes()):
        log("graph replay skipped: graphs are offered for one-lane batches only")
        want_graph = False
    if want_graph:
        gstream = torch.cuda.Stream()
        torch.cuda.synchronize()
        batch.capture(images, field, zern, status, ws, gstream)
        with torch.cuda.stream(gstream):
            batch.launch(gstream)
            graph_ms = timed_steps(lambda: batch.launch(gstream), side, gstream)
        log(f"graph replay: {graph_ms:.1f} ms/step")

    # plain path: the same kernels, one tile per call, first class
    w0 = ws_list[0]
    nf0 = w0.n * w0.upsample
    first = [int(b) for b in order[0][:args.plain_tiles]]
    P = len(first)
    per0 = w0.n_img * w0.n * w0.n
    one = [images[descs[b].image_offset:descs[b].image_offset + per0].view(1, w0.n_img, w0.n, w0.n)
           for b in first]
    ws1 = apic.Workspace()
    plan0 = apic.Plan(w0.geometry_kwargs())
    apic.reconstruct(plan0, one[0], workspace=ws1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for x in one:
        apic.reconstruct(plan0, x, workspace=ws1)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / P
    log(f"plain: {plain_s * 1e3:.1f} ms/tile")
    del ws1

    pixel = assembly = None
    if args.workload == "grid":
        assembly = assembly_timing(field, w0)
        log(f"assembly: blend {assembly['blend_ms']:.2f} ms ({assembly['blend_GBps']:.0f} GB/s), "
            f"prepare {assembly['prepare_ms_host']:.1f} ms, phases {assembly['phases_ms_host']:.1f} ms")
        pixel = pixel_pupil_timing(plan0, images, w0)
        log(f"pixel-domain pupil solve: {pixel['ms']:.1f} ms for {pixel['tiles']} tiles "
            f"(mean {pixel['mean_iterations']:.0f} iterations); Zernike basis "
            f"{pixel['ms_zernike_basis']:.1f} ms")

    # gram work per step: nonzero products of the E-sum (the algorithmic
    # count), the dense E-sum, and the products the kernels issue (live
    # (16 x 16 quadrant of a block pair, E row) pairs x 16^2 complex MACs)
    gram_exec = gram_dense = gram_nz = 0.0
    for ci, w in enumerate(ws_list):
        steps_tab = plan.query(6, ci).reshape(-1, 5).astype(np.float64)
        sz = plan.sizes(ci)
        gram_exec += (w.n_tiles * steps_tab[:, 3].sum() * sz["gram_chunk"]
                      * (sz["gram_block"] // 2) ** 2 * 8.0)
        gram_nz += w.n_tiles * gram_nonzero_flops(plan, ci)
    groups = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps,
                  "work_per_step": v[2] / args.steps} for k, v in prof.items()}
    dom = max(prof, key=lambda k: prof[k][0])
    tot_ms, launches, work = prof[dom]
    if dom in FLOP_GROUPS:
        if dom == "gram":
            gram_dense = work / args.steps
            work = gram_nz * args.steps
        achieved = work / (tot_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None}
        if dom == "gram":
            per_step_s = tot_ms / args.steps * 1e-3
            roof["work"] = ("nonzero products of the E-sum (both u + k and u' + k in P), "
                            "8 flops per complex MAC of the Hermitian lower triangle")
            roof["flops_per_step"] = gram_nz
            roof["dense_tflops"] = gram_dense / per_step_s / 1e12
            roof["executed_tflops"] = gram_exec / per_step_s / 1e12
            roof["executed_frac"] = roof["executed_tflops"] / FP64_PEAK_TFLOPS
            roof["executed_over_nonzero"] = gram_exec / gram_nz
            if args.workload == "grid" and n_total == 1024:
                roof["traffic"] = measured_traffic()
    else:
        achieved = work / (tot_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None}

    # HBM-bound groups: algorithmic bytes over their live-timed duration
    hbm_groups = ("kk", "stitch", "df_fft", "df_rhs", "out")
    hbm = {k: {"GB/s": prof[k][2] / (prof[k][0] * 1e-3) / 1e9,
               "frac": prof[k][2] / (prof[k][0] * 1e-3) / 1e9 / HBM_PEAK_GBS}
           for k in hbm_groups if k in prof and prof[k][0] > 0}
    tb = sum(prof[k][2] for k in hbm)
    tt = sum(prof[k][0] for k in hbm) * 1e-3
    hbm["all"] = {"GB/s": tb / tt / 1e9, "frac": tb / tt / 1e9 / HBM_PEAK_GBS}

    rgb = None
    if args.workload == "rgb":
        nf = ws_list[0].n * ws_list[0].upsample
        f3 = field.view(-1, nf, nf)
        chans = [f3[c::3].contiguous() for c in range(3)]
        apic.rgb_combine(*chans)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, gains = apic.rgb_combine(*chans, gains=(1.0, 1.0, 1.0))
        e1.record()
        torch.cuda.synchronize()
        cms = e0.elapsed_time(e1)
        nbytes = 3 * chans[0].numel() * 8 + 3 * chans[0].numel() * 4
        rgb = {"combine_ms": cms, "combine_GBps": nbytes / (cms * 1e-3) / 1e9}
        log(f"colour combination: {cms:.2f} ms ({rgb['combine_GBps']:.0f} GB/s)")
    if args.workload == "rgb":
        w = ws_list[0]
        config = {"workload": f"{w.n_tiles} stained tiles {w.n}x{w.n} x 3 wavelengths "
                              f"(0.63 / 0.52 / 0.47 um), 8 NA-matched + 16 darkfield per channel, "
                              f"Poisson 1e4, 2x complex64 output per channel",
                  "tiles": w.n_tiles, "channels": 3, "n": w.n, "n_bf": w.n_bf, "n_df": w.n_df}
    elif args.workload == "grid":
        w = ws_list[0]
        config = {"workload": f"{w.n_tiles} tiles {w.n}x{w.n}, 16 NA-matched + 32 darkfield "
                              f"(NA 0.25 / 0.30 / 0.38), quadratic field aberrations up to "
                              f"1.5 rad, Poisson 1e4, 2x complex64 output",
                  "tiles": w.n_tiles, "n": w.n, "n_bf": w.n_bf, "n_df": w.n_df,
                  "upsample": w.upsample}
    else:
        config = {"workload": f"uneven batch of {n_total} tiles: 128/256/512 px (4:3:1), "
                              f"8/12/16 NA-matched + 2x darkfield, 40% background, Poisson 1e4, "
                              f"2x complex64 output",
                  "tiles": n_total, "classes": [[w.n, w.n_bf, w.n_df, w.n_tiles] for w in ws_list]}
    config["mode"] = "prepared batch, classes on concurrent streams, autotuned chunks" \
        if tune else "prepared batch, classes on concurrent streams"
    if sur_note is not None:
        config["mode"] += (", surrogate pupil judged by the closed form (continuation), "
                           "closed-form fallback")
        config["surrogate"] = sur_note
    out = {
        "metric": METRIC, "value": mpx_step / (ms * 1e-3), "unit": "Mpx/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": config,
        "pupil_rmse_vs_truth": accuracy,
        "closed_form_batch": closed_form,
        "graph": None if graph_ms is None else {"value": mpx_step / (graph_ms * 1e-3),
                                                "ms_per_step": graph_ms, "steps": side,
                                                "of": "closed-form batch"},
        "plain": {"value": (nf0 * nf0 / 1e6) / plain_s, "unit": "Mpx/s", "tiles_timed": P,
                  "ms_per_tile": plain_s * 1e3, "class": 0},
        "autotune": tune,
        "workspace_gib": batch.workspace_bytes / 2 ** 30,
        "nonfinite_tiles": bad,
        "roofline": roof,
        "hbm_passes": hbm,
        "kernel_groups": groups,
        "pixel_pupil": pixel,
        "assembly": assembly,
        "rgb": rgb,
        "env": run_env(),
    }
    if cpu_base is not None:
        out["cpu_baseline"] = cpu_base

    # the largest configurations beside the headline: the uneven batch (one
    # full pass after one warmup pass) and a subset of the slide stream, each
    # run only while the whole bench stays within its time budget
    if args.workload == "grid" and not args.no_extra:
        batch.close()
        del images, field, ws
        torch.cuda.empty_cache()
        left = 560.0 - (time.time() - t_start)
        out["uneven_batch"] = uneven_block(dev, args.ws_gb) if left > 200 else \
            {"skipped": f"time budget ({left:.0f} s left)"}
        left = 560.0 - (time.time() - t_start)
        if left > 90:
            args.chunk, args.buffers = 64, 3
            rec = slide_stream(args, dev, tiles=128, steps=1, warmup=1)
            out["slide_stream"] = {k: rec[k] for k in ("value", "unit", "steps", "warmup",
                                                       "ms_per_step", "config", "timing",
                                                       "tiles_per_s", "pcie",
                                                       "resident_ms_per_tile",
                                                       "stream_ms_per_reconstructed_tile",
                                                       "surrogate_used_frac",
                                                       "slide_extrapolation")}
            out["slide_stream"]["subset"] = ("the first 128 scanned tiles of the raster order; "
                                             "host wall-clock with the copies (PCIe-inclusive)")
        else:
            out["slide_stream"] = {"skipped": f"time budget ({left:.0f} s left)"}
    out["bench_wall_s"] = time.time() - t_start
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
