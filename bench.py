"""Benchmark of the VDI hot path on one MI355X.

A step is one frame of the whole path on the FHD workload: generate the 8
sub-VDIs of a 512^3 fp32 volume split into z-slabs (per-ray bisection of the
threshold to N=20, regular slot-major layout; --layout compact for the compact
one), composite them into one N=20 VDI and render it from the original view.  The headline metric is composited VDI pixels per
second of that step.  Further legs (same JSON line):
  novel    -- that composited VDI rendered at 5, 20 and 50 degrees from its
              viewpoint: time per frame, SSIM and PSNR against DVR there;
  masks    -- the FHD volume on 8 non-convex domains (wavy z-slabs, owner map):
              generate + composite, rendering checked against the slab one;
  large    -- 1024^3 fp16 volume in 16 bricks (4x2x2): generate + composite,
              and the composite alone on maximally interleaved dense lists
              (16 x 20 supersegments per pixel, 16.6 GB of input);
  dense    -- only that dense composite (implied by large);
  learned  -- learned vs plain threshold search on held-out tiny volumes (N=8)
              and on held-out FHD-generator volumes (N=20), the regressor
              trained here with the project's kernels;
  batched  -- 64 composites of mixed size, k and N in one persistent launch
              replayed from a hipGraph: jobs/s and per-job latency.
Printed: ONE JSON line on stdout (progress goes to stderr).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--legs fhd,novel,masks,large,learned,batched]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# fp32 vector lanes: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one non-packed op per lane and cycle)
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4

# sources of the composite kernels; a traffic figure measured on other sources is not reported
COMPOSITE_SOURCES = ("paper_2206_14503_amd/csrc/vdi_composite.hip", "paper_2206_14503_amd/csrc/vdi_internal.h",
                     "paper_2206_14503_amd/csrc/vdi_kernels.h")
PMC_SUMMARY = "profiles/composite_fhd_pmc.md"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest(paths=COMPOSITE_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each scaled by the
    factor a 1 GiB device copy gives), or None when there is none or it was
    taken on other kernel sources."""
    path = os.path.join(ROOT, PMC_SUMMARY)
    if not os.path.exists(path):
        return None, "no counter summary"
    for line in open(path):
        if line.startswith("pmc: "):
            d = json.loads(line[5:])
            if d.get("source_sha256") != source_digest():
                return None, "kernel sources changed since the counters were taken"
            k = d.get("kernels", {}).get(kernel)
            if not k:
                return None, f"no counters for {kernel}"
            return (k["fetch_kib"] * d["fetch_scale"] + k["write_kib"] * d["write_scale"]) * 1024.0, "measured"
    return None, "no counter line"


def composite_bytes(inputs, out_n, npix, counts_total):
    """Algorithmic bytes of one composite launch: every stored input
    supersegment read once (24 B), each input's count (4 B) and, for compact
    inputs, offset (4 B) per pixel, and the zero-filled regular output written
    once (24 B per slot) plus its count and gamma planes (4 B + 4 B per pixel)."""
    k = len(inputs)
    b = 24 * counts_total + 4 * k * npix
    b += sum(4 * npix for s in inputs if s.offset is not None)
    b += 24 * out_n * npix + 8 * npix
    return b


def ev():
    import torch
    return torch.cuda.Event(enable_timing=True)


def timed_ms(fn, reps):
    """Per-call milliseconds of fn() over reps calls (HIP events on the current stream)."""
    import numpy as np
    import torch
    out = []
    for _ in range(reps):
        a, b = ev(), ev()
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    return np.array(out)


# ---------------------------------------------------------------- FHD (headline)

def leg_fhd(args, result):
    import numpy as np
    import torch
    from paper_2206_14503_amd import synth, vdi

    w = synth.fhd(args.seed)
    log(f"[bench] workload {w.name}: building inputs on the GPU")
    t0 = time.time()
    vol = synth.workload_volume(w, device="cuda")
    bricks = synth.brick_grid((w.n, w.n, w.n), w.grid)
    dbr = vdi.device_bricks(vol, bricks)
    tf = synth.transfer_function()
    tf_d = torch.from_numpy(tf).cuda()
    cam = synth.camera_for(w)
    step_len = 1.0 / w.n
    P = cam.width * cam.height
    layout = vdi.COMPACT if args.layout == "compact" else vdi.REGULAR
    subs = [vdi.VDI.empty(cam.width, cam.height, w.max_n, step_len, layout, capacity=w.max_n * P) for _ in bricks]
    out = vdi.VDI.empty(cam.width, cam.height, w.max_n, step_len, vdi.REGULAR)
    img = torch.empty((P, 4), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    log(f"[bench] inputs ready in {time.time() - t0:.1f}s; {len(bricks)} bricks, {cam.width}x{cam.height}, N={w.max_n}")
    mode = vdi.BISECT if w.mode == "bisect" else vdi.FIXED

    def step(marks=None):
        if marks is not None:
            marks[0].record()
        vdi.generate(dbr, cam, tf_d, step_len, step_len, mode, w.tau, w.max_n, w.iters, layout=layout, outs=subs)
        if marks is not None:
            marks[1].record()
        vdi.composite(subs, mode, w.tau, w.max_n, w.iters, out=out)
        if marks is not None:
            marks[2].record()
        vdi.render_original_view(out, img)
        if marks is not None:
            marks[3].record()

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    flags = vdi.device_status()
    if flags:
        raise RuntimeError(f"device status flags {flags} after warmup")
    marks = [[ev() for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    start, stop = ev(), ev()
    start.record()
    for i in range(args.steps):
        step(marks[i])
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ms_step = total_ms / args.steps
    gen_ms = np.array([m[0].elapsed_time(m[1]) for m in marks])
    comp_ms = np.array([m[1].elapsed_time(m[2]) for m in marks])
    rend_ms = np.array([m[2].elapsed_time(m[3]) for m in marks])
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step; generate {gen_ms.mean():.3f} ms, "
        f"composite {comp_ms.mean():.3f} ms, render {rend_ms.mean():.3f} ms")

    counts_total = int(sum(int(s.count.to(torch.int64).sum()) for s in subs))
    out_total = int(out.count.to(torch.int64).sum())
    cbytes = composite_bytes(subs, w.max_n, P, counts_total)
    comp_gbs = cbytes / (comp_ms.mean() * 1e-3) / 1e9
    log(f"[bench] composite: {counts_total} input supersegments, {out_total} output; algorithmic "
        f"{cbytes / 1e9:.3f} GB -> {comp_gbs:.1f} GB/s ({100 * comp_gbs / HBM_PEAK_GBS:.1f}% of HBM peak)")

    value = P * args.steps / (total_ms * 1e-3)
    result.update({
        "metric": "composited VDI pixels/s (k ranks, N supersegs) + % HBM peak; learned vs plain τ speedup",
        "value": value,
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "volume": f"{w.n}^3 {w.vol_dtype}", "bricks": len(bricks),
                   "grid": list(w.grid), "width": cam.width, "height": cam.height, "max_n": w.max_n,
                   "iters": w.iters, "tau_mode": w.mode, "layout": args.layout, "seed": w.seed},
        "stages_ms": {"generate": float(gen_ms.mean()), "composite": float(comp_ms.mean()),
                      "render": float(rend_ms.mean())},
        "composite_fhd": {"input_supersegments": counts_total, "output_supersegments": out_total,
                          "algorithmic_bytes": cbytes, "ms": float(comp_ms.mean()), "achieved_GBps": comp_gbs,
                          "frac_hbm_peak": comp_gbs / HBM_PEAK_GBS},
    })
    traffic, why = measured_traffic("composite_cat_kernel")
    result["roofline"] = {"kernel": "composite_cat_kernel (composite stage)", "bound": "hbm", "achieved": comp_gbs,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": comp_gbs / HBM_PEAK_GBS,
                          "traffic": traffic, "traffic_note": why, "algorithmic_bytes": cbytes,
                          "workload": w.name}
    return dict(w=w, vol=vol, bricks=bricks, tf=tf, cam=cam, step_len=step_len, dbr=dbr, tf_d=tf_d, out=out)


# ---------------------------------------------------------------- non-convex domains

def leg_masks(args, result, fhd):
    """The FHD volume on 8 non-convex domains (z-slabs with wavy interfaces,
    Sec. 5.3): generation through the owner map, compositing (interleaved
    lists take the general merge) and the original-view rendering, which must
    equal the slab decomposition's (both are DVR of the same samples)."""
    import numpy as np
    import torch
    from paper_2206_14503_amd import synth, vdi

    w, cam, step_len, tf_d, v0 = fhd["w"], fhd["cam"], fhd["step_len"], fhd["tf_d"], fhd["out"]
    owner, bricks, ranks = synth.wavy_slab_owner(w.n, 8, 16, w.seed)
    dbr = vdi.device_bricks(fhd["vol"], bricks, owner=owner, ranks=ranks)
    P = cam.width * cam.height
    subs = [vdi.VDI.empty(cam.width, cam.height, w.max_n, step_len) for _ in bricks]
    out = vdi.VDI.empty(cam.width, cam.height, w.max_n, step_len, vdi.REGULAR)
    gen = lambda: vdi.generate(dbr, cam, tf_d, step_len, step_len, vdi.BISECT, 0.0, w.max_n, w.iters, outs=subs)
    comp = lambda: vdi.composite(subs, vdi.BISECT, 0.0, w.max_n, w.iters, out=out)
    gen()
    comp()
    torch.cuda.synchronize()
    flags = vdi.device_status()
    gen_ms = float(timed_ms(gen, 5).mean())
    comp_ms = float(timed_ms(comp, 5).mean())
    img = vdi.render_original_view(out)
    ref = vdi.render_original_view(v0)
    err = float((img - ref).abs().max())
    torch.cuda.synchronize()
    log(f"[bench] non-convex: generate {gen_ms:.3f} ms, composite {comp_ms:.3f} ms; "
        f"max |render - slab render| {err:.2g}; device flags {flags}")
    result["non_convex"] = {"workload": f"{w.name} volume on 8 wavy z-slab domains (interfaces displaced up to 32 "
                                        f"voxels)", "generate_ms": gen_ms, "composite_ms": comp_ms,
                            "pixels_per_s": P / ((gen_ms + comp_ms) / 1e3), "render_vs_slabs_max_abs": err,
                            "device_flags": flags}
    del dbr, subs, out


# ---------------------------------------------------------------- novel viewpoints

def leg_novel(args, result, fhd):
    """The composited FHD VDI rendered at viewpoint deviations about its
    generation viewpoint (Sec. 7): time per frame, and SSIM and PSNR against
    DVR at the new viewpoint, which is the original-view rendering of a VDI
    generated there (equal to DVR of the same samples, Sec. 2.3)."""
    import torch
    from paper_2206_14503_amd import quality, synth, vdi

    w, cam, step_len, dbr, tf_d, v0 = fhd["w"], fhd["cam"], fhd["step_len"], fhd["dbr"], fhd["tf_d"], fhd["out"]
    out = {}
    for deg in (5.0, 20.0, 50.0):
        view = synth.orbit_camera(10_000 + w.seed, cam.width, cam.height, turn_deg=deg)
        img = torch.empty((view.width * view.height, 4), dtype=torch.float32, device="cuda")
        fn = lambda: vdi.render_novel_view(v0, cam, view, step_len, out=img)
        fn()
        torch.cuda.synchronize()
        ms = float(timed_ms(fn, 5).mean())
        subs = vdi.generate(dbr, view, tf_d, step_len, step_len, vdi.BISECT, 0.0, w.max_n, w.iters)
        gt = vdi.render_original_view(vdi.composite(subs, vdi.BISECT, 0.0, w.max_n, w.iters))
        a, b = img.cpu().numpy(), gt.cpu().numpy()
        del subs, gt
        s, p = quality.ssim(a, b, height=view.height), quality.psnr(a, b, height=view.height)
        out[f"{deg:g}deg"] = {"ms": ms, "mpix_per_s": view.width * view.height / ms / 1e3, "ssim_vs_dvr": s,
                              "psnr_vs_dvr_db": p}
        log(f"[bench] novel view at {deg:g} deg: {ms:.3f} ms; SSIM {s:.4f}, PSNR {p:.2f} dB vs DVR")
    result["novel_view"] = {"workload": f"{w.name} VDI rendered at {cam.width}x{cam.height}, deviations about the "
                                        f"box centre along the orbit", **out}


# ---------------------------------------------------------------- large one-GPU share

def leg_large(args, result):
    import numpy as np
    import torch
    from paper_2206_14503_amd import synth, vdi

    w = synth.large(args.seed)
    log(f"[bench] large: {w.name}")
    t0 = time.time()
    vol = synth.workload_volume(w, device="cuda")
    bricks = synth.brick_grid((w.n, w.n, w.n), w.grid)
    dbr = vdi.device_bricks(vol, bricks)
    del vol
    tf_d = torch.from_numpy(synth.transfer_function()).cuda()
    cam = synth.camera_for(w)
    step_len = 1.0 / w.n
    P = cam.width * cam.height
    subs = [vdi.VDI.empty(cam.width, cam.height, w.max_n, step_len, vdi.REGULAR) for _ in bricks]
    out = vdi.VDI.empty(cam.width, cam.height, w.max_n, step_len, vdi.REGULAR)
    torch.cuda.synchronize()
    log(f"[bench] large inputs ready in {time.time() - t0:.1f}s")
    gen = lambda: vdi.generate(dbr, cam, tf_d, step_len, step_len, vdi.BISECT, 0.0, w.max_n, w.iters, outs=subs)
    comp = lambda: vdi.composite(subs, vdi.BISECT, 0.0, w.max_n, w.iters, out=out)
    gen()
    comp()
    torch.cuda.synchronize()
    g_ms = timed_ms(gen, 3)
    c_ms = timed_ms(comp, 5)
    counts_total = int(sum(int(s.count.to(torch.int64).sum()) for s in subs))
    cbytes = composite_bytes(subs, w.max_n, P, counts_total)
    gbs = cbytes / (np.median(c_ms) * 1e-3) / 1e9
    log(f"[bench] large generated: generate {np.median(g_ms):.2f} ms, composite {np.median(c_ms):.3f} ms, "
        f"{counts_total} input supersegments, {gbs:.0f} GB/s")
    res = {"workload": w.name, "generate_ms": float(np.median(g_ms)), "composite_ms": float(np.median(c_ms)),
           "input_supersegments": counts_total, "algorithmic_bytes": cbytes, "achieved_GBps": gbs,
           "frac_hbm_peak": gbs / HBM_PEAK_GBS, "composited_pixels_per_s": P / (np.median(c_ms) * 1e-3)}
    del subs, dbr
    torch.cuda.empty_cache()
    result["large"] = res
    leg_dense(args, result)


def leg_dense(args, result):
    """The large share's composite on dense maximally interleaved lists:
    16 inputs x 20 supersegments per pixel (16.6 GB of input), N = 20."""
    import numpy as np
    import torch
    from paper_2206_14503_amd import synth, vdi

    w = synth.large(args.seed)
    cam = synth.camera_for(w)
    P = cam.width * cam.height
    res = result.setdefault("large", {"workload": w.name})
    k, n = 16, 20
    color = torch.empty((k, n, P, 4), dtype=torch.float32, device="cuda")
    depth = torch.empty((k, n, P, 2), dtype=torch.float32, device="cuda")
    chunk = 1 << 17
    for p0 in range(0, P, chunk):
        p1 = min(P, p0 + chunk)
        c, d, _ = synth.dense_interleaved_lists(k, n, p1 - p0, seed=args.seed * 1000 + p0 // chunk, device="cuda")
        color[:, :, p0:p1] = c
        depth[:, :, p0:p1] = d
    cnt = torch.full((k, P), n, dtype=torch.int32, device="cuda")
    ins = [vdi.VDI(cam.width, cam.height, n, 0.01, vdi.REGULAR, color[r], depth[r], cnt[r]) for r in range(k)]
    out2 = vdi.VDI.empty(cam.width, cam.height, n, 0.01, vdi.REGULAR)
    comp2 = lambda: vdi.composite(ins, vdi.BISECT, 0.0, n, 10, out=out2)
    comp2()
    torch.cuda.synchronize()
    c2 = timed_ms(comp2, 3)
    b2 = composite_bytes(ins, n, P, k * n * P)
    gbs2 = b2 / (np.median(c2) * 1e-3) / 1e9
    log(f"[bench] large dense interleaved: composite {np.median(c2):.3f} ms, {b2 / 1e9:.2f} GB, {gbs2:.0f} GB/s")
    res["dense_interleaved"] = {"k": k, "n_per_input": n, "composite_ms": float(np.median(c2)),
                                "algorithmic_bytes": b2, "achieved_GBps": gbs2, "frac_hbm_peak": gbs2 / HBM_PEAK_GBS,
                                "composited_pixels_per_s": P / (np.median(c2) * 1e-3)}
    del color, depth, ins, out2
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- learned threshold

def leg_learned(args, result):
    from paper_2206_14503_amd import learned

    for cfg, key, seeds in ((learned.LearnedConfig(), "learned", range(100, 104)),
                            (learned.LearnedConfig.fhd(), "learned_fhd", range(100, 102))):
        if key == "learned_fhd" and not args.learn_fhd:
            continue
        learned_case(args, result, cfg, key, seeds)


def learned_case(args, result, cfg, key, eval_seeds):
    import torch
    from paper_2206_14503_amd import learned, synth

    tf_d = torch.from_numpy(synth.transfer_function()).cuda()
    t0 = time.time()
    X, Y, st = learned.training_pairs(cfg, seeds=range(args.learn_seeds), tf_d=tf_d)
    log(f"[bench] {key}: {X.shape[0]} training pairs (of {st['kept']} served among {st['rays']} brick-rays) "
        f"in {time.time() - t0:.1f}s")
    mlp = learned.init_mlp(0)
    t1 = time.time()
    losses = learned.train(mlp, X, Y, epochs=args.learn_epochs, batch=4096, lr=2e-3, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    del X, Y
    torch.cuda.empty_cache()
    ev_ = learned.evaluate(mlp, cfg, seeds=eval_seeds, tf_d=tf_d, reps=3)
    log(f"[bench] {key} vs plain: {ev_}")
    result[key] = {"train_pairs": st["pairs"], "train_seconds": t_train, "final_loss": losses[-1],
                   "eval_rays": ev_["brick_rays"], "workload": cfg.describe(), **ev_}
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- batched composites

def leg_batched(args, result):
    import numpy as np
    import torch
    from paper_2206_14503_amd import synth, vdi

    specs = synth.batch_jobs(5000, 64)
    pw = synth.batch_pool_workload(5000)
    vol = synth.workload_volume(pw, device="cuda")
    bricks = synth.brick_grid((pw.n,) * 3, pw.grid)
    dbr = vdi.device_bricks(vol, bricks)
    tf_d = torch.from_numpy(synth.transfer_function()).cuda()
    step_len = 1.0 / pw.n
    pool = {}
    t0 = time.time()
    for (wd, ht, k, n) in specs:
        if (wd, ht, n) in pool:
            continue
        cam = synth.orbit_camera(10_000 + 5000, wd, ht)
        subs = vdi.generate(dbr, cam, tf_d, step_len, step_len, vdi.BISECT, 0.0, n, 10, layout=vdi.COMPACT,
                            capacity=n * wd * ht)
        pool[(wd, ht, n)] = subs
    torch.cuda.synchronize()
    log(f"[bench] batched: pooled {len(pool)} sets of 16 compact sub-VDIs in {time.time() - t0:.1f}s")
    jobs = []
    for (wd, ht, k, n) in specs:
        out = vdi.VDI.empty(wd, ht, n, step_len, vdi.REGULAR)
        jobs.append(vdi.Job(pool[(wd, ht, n)][:k], out, mode=vdi.BISECT, iters=10))
    import tempfile
    cache = os.path.join(tempfile.gettempdir(), f"vdi_autotune_tiles_{os.getpid()}.txt")
    t1 = time.time()
    vdi.autotune(jobs, cache)
    t_tune = time.time() - t1
    log(f"[bench] batched: autotuned tile sizes in {t_tune:.1f}s -> {open(cache).read().strip()}")
    b = vdi.Batch(jobs, autotune_cache=cache)
    info = b.info()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.run()
    s.synchronize()
    with torch.cuda.stream(s):
        b.capture(s)
    torch.cuda.synchronize()
    reps = 5
    times, lats = [], []
    for _ in range(reps):
        a, e = ev(), ev()
        a.record(s)
        b.replay(s)
        e.record(s)
        s.synchronize()
        times.append(a.elapsed_time(e))
        lat, span = b.latencies_s()
        lats.append(lat)
    lats = np.concatenate(lats) * 1e3
    ms = float(np.median(times))
    bytes_total = 0
    for j in jobs:
        ct = int(sum(int(v.count.to(torch.int64).sum()) for v in j.inputs))
        bytes_total += composite_bytes(j.inputs, j.out.max_n, j.out.npix, ct)
    gbs = bytes_total / (ms * 1e-3) / 1e9
    log(f"[bench] batched: {len(jobs)} jobs in {ms:.2f} ms -> {len(jobs) / (ms * 1e-3):.0f} jobs/s; "
        f"p50 {np.percentile(lats, 50):.3f} ms p99 {np.percentile(lats, 99):.3f} ms; {gbs:.0f} GB/s")
    result["batched"] = {"jobs": len(jobs), "ms_per_batch": ms, "jobs_per_s": len(jobs) / (ms * 1e-3),
                         "latency_ms_p50": float(np.percentile(lats, 50)),
                         "latency_ms_p99": float(np.percentile(lats, 99)),
                         "algorithmic_bytes": bytes_total, "achieved_GBps": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS,
                         "tiles": info["tiles"], "grid": info["grid"], "autotune_seconds": t_tune,
                         "launch": "one persistent kernel replayed from a hipGraph"}
    b.close()


# ---------------------------------------------------------------- CPU baseline

def cpu_baseline(w, vol, bricks, tf, cam, step_len, target_s):
    """The oracle on a bounded, seeded sample of the same frame's pixels:
    generate all bricks' lists for those pixels, then composite them.  Pixels
    per second of the oracle on the host threads it was given."""
    import numpy as np
    import oracle
    host_vol = vol.float().cpu().numpy() if w.vol_dtype == "f32" else vol.cpu().numpy()
    rng = np.random.default_rng(12345)
    P = cam.width * cam.height
    cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    mode = oracle.BISECT if w.mode == "bisect" else oracle.FIXED

    def run(npx):
        px = np.sort(rng.choice(P, size=npx, replace=False)).astype(np.int32)
        t = time.time()
        g = oracle.generate(host_vol, bricks, cam, tf, step_len, step_len, mode, w.tau, w.max_n, w.iters, pixels=px,
                            nthreads=cores)
        k = len(bricks)
        oracle.composite([g["color"][r] for r in range(k)], [g["depth"][r] for r in range(k)],
                         [g["count"][r] for r in range(k)], step_len, mode, w.tau, w.max_n, w.iters, nthreads=cores)
        return time.time() - t

    npx = 4096
    t = run(npx)
    npx2 = int(min(P, max(npx, npx * target_s / max(t, 1e-3))))
    if npx2 > npx:
        npx, t = npx2, run(npx2)
    log(f"[bench] cpu baseline: oracle on {npx} sampled pixels took {t:.2f}s with {cores} threads")
    return {"value": npx / t, "unit": "pixels/s", "cores": cores, "kind": "oracle",
            "sample": f"{npx} seeded random pixels of the same FHD frame (generate all {len(bricks)} bricks + "
                      f"composite)", "seconds": t}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--layout", choices=["compact", "regular"], default="regular")
    ap.add_argument("--legs", default="fhd,novel,masks,large,learned,batched")
    ap.add_argument("--learn-seeds", type=int, default=32)
    ap.add_argument("--learn-epochs", type=int, default=8)
    ap.add_argument("--no-learn-fhd", dest="learn_fhd", action="store_false",
                    help="skip the learned threshold on FHD-generator volumes (N=20)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device-to-device three times (a kernel of known traffic for counter scaling)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle time for the CPU baseline")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the k bricks of a frame are resident on one device). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    legs = set(args.legs.split(","))
    result = {}
    if args.copy_calibration:
        src = torch.ones((1 << 28,), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 x 1 GiB device-to-device copies")
        del src, dst
    fhd = leg_fhd(args, result)
    if "novel" in legs:
        leg_novel(args, result, fhd)
    if "masks" in legs:
        leg_masks(args, result, fhd)
    if "large" in legs:
        leg_large(args, result)
    elif "dense" in legs:
        leg_dense(args, result)
    if "learned" in legs:
        leg_learned(args, result)
    if "batched" in legs:
        leg_batched(args, result)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(fhd["w"], fhd["vol"], fhd["bricks"], fhd["tf"], fhd["cam"],
                                              fhd["step_len"], args.cpu_seconds)
        result["cpu_baseline"]["gpu_over_cpu"] = result["value"] / result["cpu_baseline"]["value"]
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
