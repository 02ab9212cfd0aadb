"""Benchmark of the VDI hot path on one MI355X.

Headline (the step): the composite of the large one-GPU share on dense,
maximally interleaved inputs -- 16 regular sub-VDIs of 1920x1080 pixels with
20 supersegments per pixel each (15.9 GB), depth-merged and re-segmented by
the per-pixel bisection into one N=20 VDI, then rendered from the original
view.  The metric is composited VDI pixels per second of that step, with the
composite's algorithmic bytes against the 8 TB/s HBM peak.  Further legs
(same JSON line):
  fhd      -- the FHD frame: generate the 8 sub-VDIs of a 512^3 fp32 volume in
              z-slabs (per-ray bisection to N=20), composite, render; per-stage
              times, the composite's HBM roofline and the generation kernel's
              VALU roofline;
  novel    -- that composited VDI rendered at 5, 20 and 50 degrees from its
              viewpoint: time per frame, SSIM and PSNR against DVR there;
  masks    -- the FHD volume on 8 non-convex domains (wavy z-slabs, owner map):
              generate + composite, rendering checked against the slab one;
  large    -- 1024^3 fp16 volume in 16 bricks (4x2x2): generate + composite;
  learned  -- learned vs plain threshold search on held-out tiny volumes (N=8)
              and on held-out FHD-generator volumes (N=20), the regressor
              trained here with the project's kernels;
  batched  -- 64 composites of mixed size, k and N in one persistent launch
              replayed from a hipGraph: jobs/s and per-job latency.
The CPU baseline is the oracle on a seeded pixel sample of the headline frame
(all host threads), its lists compared with the GPU's; the same comparison
runs on a sample of the FHD frame (generation and composite).
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
# fp32 vector issue: 256 CUs x 4 SIMDs x 32 lanes per cycle x 2.4 GHz = 78.6e12
# lane-instructions/s (157.3 TFLOP/s counting an FMA as two)
VALU_PEAK_TLANE = 256 * 4 * 32 * 2.4e9 / 1e12

# sources of the kernels; a counter figure measured on other sources is not reported
COMPOSITE_SOURCES = ("paper_2206_14503_amd/csrc/vdi_composite.hip", "paper_2206_14503_amd/csrc/vdi_internal.h",
                     "paper_2206_14503_amd/csrc/vdi_kernels.h")
GENERATE_SOURCES = ("paper_2206_14503_amd/csrc/vdi_generate.hip", "paper_2206_14503_amd/csrc/vdi_internal.h",
                    "paper_2206_14503_amd/csrc/vdi_kernels.h")
DENSE_PMC = "profiles/composite_dense_pmc.md"
FHD_PMC = "profiles/composite_fhd_pmc.md"
GEN_SQ = "profiles/generate_fhd_sq.md"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest(paths=COMPOSITE_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_line(summary: str, sources):
    """The `pmc: {json}` line of a committed rocprofv3 counter summary, or
    (None, why) when there is none or it was taken on other kernel sources."""
    path = os.path.join(ROOT, summary)
    if not os.path.exists(path):
        return None, f"no counter summary {summary}"
    for line in open(path):
        if line.startswith("pmc: "):
            d = json.loads(line[5:])
            if d.get("source_sha256") != source_digest(sources):
                return None, "kernel sources changed since the counters were taken"
            return d, "measured"
    return None, "no counter line"


def measured_traffic(kernel: str, summary: str = DENSE_PMC):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each scaled by the
    factor a 1 GiB device copy gives), or None with the reason."""
    d, why = counter_line(summary, COMPOSITE_SOURCES)
    if d is None:
        return None, why
    k = d.get("kernels", {}).get(kernel)
    if not k or "fetch_kib" not in k:
        return None, f"no traffic counters for {kernel}"
    return (k["fetch_kib"] * d["fetch_scale"] + k["write_kib"] * d["write_scale"]) * 1024.0, "measured"


def measured_valu(kernel: str, summary: str = GEN_SQ, sources=GENERATE_SOURCES):
    """VALU wave-instructions per launch of `kernel` (SQ_INSTS_VALU) from a
    committed counter summary, or None with the reason."""
    d, why = counter_line(summary, sources)
    if d is None:
        return None, why
    k = d.get("kernels", {}).get(kernel)
    if not k or "valu_insts" not in k:
        return None, f"no VALU counters for {kernel}"
    return float(k["valu_insts"]), "measured"


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


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


# ---------------------------------------------------------------- headline: dense composite

# the composite call on interleaved inputs: the concatenation test, then the
# ordered general merge (merge order, staging, re-segmentation); its counters
# are summed over the call's kernels, its time is the call's
DENSE_CALL = "composite call"
DENSE_KERNEL = "composite_staged_kernel"


def leg_dense(args, result):
    """The step: composite 16 dense interleaved sub-VDIs (20 supersegments per
    pixel each, 1920x1080) into one N=20 VDI and render it.  Returns a seeded
    pixel sample of the inputs and of the GPU's output for the oracle."""
    import numpy as np
    import torch
    from paper_2206_14503_amd import synth, vdi

    w = synth.large(args.seed)
    cam = synth.camera_for(w)
    P = cam.width * cam.height
    k, n, ref = 16, 20, 0.01
    t0 = time.time()
    color, depth, count = synth.dense_frame(k, n, P, seed=args.seed)
    ins = [vdi.VDI(cam.width, cam.height, n, ref, vdi.REGULAR, color[r], depth[r], count[r]) for r in range(k)]
    out = vdi.VDI.empty(cam.width, cam.height, n, ref, vdi.REGULAR)
    img = torch.empty((P, 4), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    log(f"[bench] dense: {k} inputs x {n} supersegments per pixel, {cam.width}x{cam.height}, N={n}; "
        f"inputs ready in {time.time() - t0:.1f}s")

    def step(marks=None):
        if marks is not None:
            marks[0].record()
        vdi.composite(ins, vdi.BISECT, 0.0, n, 10, out=out)
        if marks is not None:
            marks[1].record()
        vdi.render_original_view(out, img)
        if marks is not None:
            marks[2].record()

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] dense warmup step {i + 1}/{args.warmup} done")
    flags = vdi.device_status()
    if flags:
        raise RuntimeError(f"device status flags {flags} after warmup")
    marks = [[ev() for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    start, stop = ev(), ev()
    start.record()
    for i in range(args.steps):
        step(marks[i])
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ms_step = total_ms / args.steps
    comp_ms = np.array([m[0].elapsed_time(m[1]) for m in marks])
    rend_ms = np.array([m[1].elapsed_time(m[2]) for m in marks])
    cbytes = composite_bytes(ins, n, P, k * n * P)
    gbs = cbytes / (comp_ms.mean() * 1e-3) / 1e9
    log(f"[bench] dense: {args.steps} steps, {ms_step:.3f} ms/step; composite {comp_ms.mean():.3f} ms "
        f"({gbs:.0f} GB/s algorithmic, {100 * gbs / HBM_PEAK_GBS:.1f}% of HBM peak), render {rend_ms.mean():.3f} ms")
    result.update({
        "metric": "composited VDI pixels/s (k ranks, N supersegs) + % HBM peak; learned vs plain τ speedup",
        "value": P * args.steps / (total_ms * 1e-3),
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
        "config": {"workload": "large-dense-16x20-1920x1080-N20", "inputs": k, "supersegments_per_input": n,
                   "width": cam.width, "height": cam.height, "max_n": n, "iters": 10, "tau_mode": "bisect",
                   "layout": "regular", "interleaving": "maximal (seeded shuffle of 320 disjoint cells)",
                   "seed": args.seed},
        "stages_ms": {"composite": float(comp_ms.mean()), "render": float(rend_ms.mean())},
    })
    traffic, why = measured_traffic(DENSE_CALL, DENSE_PMC)
    result["roofline"] = {"kernel": f"{DENSE_KERNEL} (composite call)", "bound": "hbm", "achieved": gbs,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                          "traffic_note": why, "algorithmic_bytes": cbytes,
                          "workload": result["config"]["workload"]}
    # the re-segmentation's bisection is arithmetic: VALU lane-instructions of
    # the call (committed counters) per second of the call, against the fp32
    # vector issue peak
    valu, vwhy = measured_valu(DENSE_CALL, DENSE_PMC, COMPOSITE_SOURCES)
    ach = None if valu is None else valu * 64 / (comp_ms.mean() * 1e-3) / 1e12
    result["roofline_alu"] = {"kernel": f"{DENSE_KERNEL} (composite call)", "bound": "alu", "achieved": ach,
                              "peak": VALU_PEAK_TLANE, "unit": "T VALU lane-instructions/s",
                              "frac": None if ach is None else ach / VALU_PEAK_TLANE,
                              "valu_wave_instructions": valu, "counter_note": vwhy}
    # a seeded sample for the oracle: inputs and the GPU's output at those pixels
    px = np.sort(np.random.default_rng(4242).choice(P, size=min(P, args.sample_px), replace=False))
    idx = torch.from_numpy(px).long().cuda()
    sample = {"px": px, "color": color[:, :, idx].cpu().numpy(), "depth": depth[:, :, idx].cpu().numpy(),
              "count": count[:, idx].cpu().numpy(), "k": k, "n": n, "ref": ref,
              "gpu": (out.color[:, idx].cpu().numpy(), out.depth[:, idx].cpu().numpy(),
                      out.count[idx].cpu().numpy(), out.gamma[idx].cpu().numpy())}
    del ins, out, color, depth, count, img
    torch.cuda.empty_cache()
    return sample


# ---------------------------------------------------------------- FHD frame

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

    traffic, why = measured_traffic(DENSE_CALL, FHD_PMC)
    valu, vwhy = measured_valu("gen_kernel<float, 0, false>", GEN_SQ)
    gen_t = float(gen_ms.mean()) * 1e-3
    fhd = {
        "workload": w.name, "volume": f"{w.n}^3 {w.vol_dtype}", "bricks": len(bricks), "grid": list(w.grid),
        "width": cam.width, "height": cam.height, "max_n": w.max_n, "iters": w.iters, "tau_mode": w.mode,
        "layout": args.layout, "steps": args.steps, "ms_per_step": ms_step,
        "pixels_per_s": P * args.steps / (total_ms * 1e-3),
        "stages_ms": {"generate": float(gen_ms.mean()), "composite": float(comp_ms.mean()),
                      "render": float(rend_ms.mean())},
        "composite": {"input_supersegments": counts_total, "output_supersegments": out_total,
                      "algorithmic_bytes": cbytes, "ms": float(comp_ms.mean()), "achieved_GBps": comp_gbs,
                      "frac_hbm_peak": comp_gbs / HBM_PEAK_GBS},
        "roofline_composite": {"kernel": "composite_cat_kernel (composite call)", "bound": "hbm",
                               "achieved": comp_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": comp_gbs / HBM_PEAK_GBS, "traffic": traffic, "traffic_note": why,
                               "algorithmic_bytes": cbytes},
        # generation is bound by its VALU issue (the volume is re-read from
        # cache): lane-instructions per second against the fp32 vector issue peak
        "roofline_generate": {"kernel": "gen_kernel<float, 0, false> (generate call)", "bound": "alu",
                              "achieved": None if valu is None else valu * 64 / gen_t / 1e12,
                              "peak": VALU_PEAK_TLANE, "unit": "T VALU lane-instructions/s",
                              "frac": None if valu is None else valu * 64 / gen_t / 1e12 / VALU_PEAK_TLANE,
                              "valu_wave_instructions": valu, "counter_note": vwhy},
    }
    result["fhd"] = fhd
    # a seeded sample for the oracle: the GPU's sub-VDIs and composite there
    px = np.sort(np.random.default_rng(2525).choice(P, size=min(P, args.fhd_sample_px), replace=False))
    idx = torch.from_numpy(px).long().cuda()
    cols = lambda v: (v.color[:, idx].cpu().numpy(), v.depth[:, idx].cpu().numpy(), v.count[idx].cpu().numpy(),
                      v.gamma[idx].cpu().numpy())
    sample = {"px": px, "subs": [cols(v) for v in subs] if layout == vdi.REGULAR else None, "out": cols(out)}
    return dict(w=w, vol=vol, bricks=bricks, tf=tf, cam=cam, step_len=step_len, dbr=dbr, tf_d=tf_d, out=out,
                sample=sample)


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


def leg_learned_composite(args, result):
    """The compositing bisection's first scan steered by a regressor trained
    here (on dense interleaved frames of other seeds) against the default
    out_n-th-largest-distance rule, on the headline frame: same output, time
    of each."""
    import torch
    from paper_2206_14503_amd import learned, synth, vdi
    t0 = time.time()
    X, Y, st = learned.composite_training_pairs(seeds=range(900, 900 + args.learn_seeds // 4))
    mlp = learned.init_mlp(0)
    losses = learned.train(mlp, X, Y, epochs=args.learn_epochs, batch=4096, lr=2e-3)
    t_train = time.time() - t0
    del X, Y
    w = synth.large(args.seed)
    cam = synth.camera_for(w)
    P = cam.width * cam.height
    color, depth, count = synth.dense_frame(16, 20, P, seed=args.seed)
    ins = [vdi.VDI(cam.width, cam.height, 20, 0.01, vdi.REGULAR, color[r], depth[r], count[r]) for r in range(16)]
    ev_ = learned.evaluate_composite(mlp, ins, 20, reps=3)
    log(f"[bench] learned composite: {st['pairs']} training pairs, loss {losses[-1]:.4f}, {t_train:.1f}s; {ev_}")
    result["learned_composite"] = {"workload": "large-dense-16x20-1920x1080-N20 (the headline frame)",
                                   "train_pairs": st["pairs"], "train_seconds": t_train, "final_loss": losses[-1],
                                   **ev_}
    del ins, color, depth, count
    torch.cuda.empty_cache()
    # the generated frames: the FHD frame's 8 slabs and the large volume's
    # 16 bricks; only their pixels whose lists interleave in depth take the
    # general merge, where the regressor steers
    tf_d = torch.from_numpy(synth.transfer_function()).cuda()
    for key, wl in (("fhd", synth.fhd(args.seed)), ("large_generated", synth.large(args.seed))):
        vol = synth.workload_volume(wl, device="cuda")
        dbr = vdi.device_bricks(vol, synth.brick_grid((wl.n, wl.n, wl.n), wl.grid))
        cam_w = synth.camera_for(wl)
        subs = vdi.generate(dbr, cam_w, tf_d, 1.0 / wl.n, 1.0 / wl.n, vdi.BISECT, 0.0, wl.max_n, wl.iters)
        ev_w = learned.evaluate_composite(mlp, subs, wl.max_n, reps=5)
        log(f"[bench] learned composite on {wl.name}: {ev_w}")
        result["learned_composite"][key] = {"workload": wl.name, **ev_w}
        del subs, dbr, vol
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

def _parity_summary(st):
    return {k: v for k, v in st.items() if k != "fp64_mask"}


def cpu_baseline(dense, fhd, args):
    """The oracle on a bounded, seeded sample of the headline frame's pixels
    (all host threads): composited pixels per second, and its lists compared
    with the GPU's at those pixels.  Then the same comparison (untimed) on a
    sample of the FHD frame: every brick's generated lists, and the composite
    at the pixels whose generated lists all took the oracle's fp64 outcome."""
    import numpy as np
    import oracle
    from oracle.parity import check_lists
    cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    k, n, ref = dense["k"], dense["n"], dense["ref"]

    def run(npx):
        c, d, m = dense["color"][:, :, :npx], dense["depth"][:, :, :npx], dense["count"][:, :npx]
        t = time.time()
        o = oracle.composite([c[r] for r in range(k)], [d[r] for r in range(k)], [m[r] for r in range(k)], ref,
                             oracle.BISECT, 0.0, n, 10, nthreads=cores)
        return time.time() - t, o

    total = len(dense["px"])
    npx = min(1024, total)
    t, o = run(npx)
    npx2 = int(min(total, max(npx, npx * args.cpu_seconds / max(t, 1e-3))))
    if npx2 > npx:
        npx = npx2
        t, o = run(npx)
    g = tuple(x[..., :npx, :] if x.ndim == 3 else x[:npx] for x in dense["gpu"])
    st = check_lists(g, o, "dense sample", strict=False)
    log(f"[bench] cpu baseline: oracle composite of {npx} sampled pixels in {t:.2f}s with {cores} threads; "
        f"vs GPU: {_parity_summary(st)}")
    res = {"value": npx / t, "unit": "pixels/s", "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{npx} seeded random pixels of the headline frame (16 x 20 interleaved supersegments each, "
                     f"merge + bisection to N=20)", "seconds": t, "parity_vs_gpu": _parity_summary(st)}
    if fhd is not None and fhd["sample"]["subs"] is not None:
        w, cam, step_len = fhd["w"], fhd["cam"], fhd["step_len"]
        px = fhd["sample"]["px"].astype(np.int32)
        host = fhd["vol"].float().cpu().numpy()
        t0 = time.time()
        gen = oracle.generate(host, fhd["bricks"], cam, fhd["tf"], step_len, step_len, oracle.BISECT, 0.0, w.max_n,
                              w.iters, pixels=px, nthreads=cores)
        kb = len(fhd["bricks"])
        sts = [check_lists(fhd["sample"]["subs"][r], gen, f"fhd brick {r}", brick=r, strict=False, masks=True)
               for r in range(kb)]
        clean = np.logical_and.reduce([s_["fp64_mask"] for s_ in sts])
        oc = oracle.composite([gen["color"][r] for r in range(kb)], [gen["depth"][r] for r in range(kb)],
                              [gen["count"][r] for r in range(kb)], step_len, oracle.BISECT, 0.0, w.max_n, w.iters,
                              nthreads=cores)
        sel = np.nonzero(clean)[0]
        gsel = tuple(x[:, sel] if x.ndim == 3 else x[sel] for x in fhd["sample"]["out"])
        osel = {key: (v[:, sel] if key in ("color", "depth") else v[sel]) for key, v in oc.items()
                if key in ("color", "depth", "count", "gamma", "nout")}
        alts = oc["alts"]
        keep = np.isin(alts["ray"], sel)
        remap = np.full(len(px), -1, np.int64)
        remap[sel] = np.arange(len(sel))
        osel["alts"] = {key: v[keep] for key, v in alts.items()}
        osel["alts"]["ray"] = remap[alts["ray"][keep]].astype(np.int32)
        cst = check_lists(gsel, osel, "fhd composite", strict=False)
        gen_sum = {key: int(sum(s_[key] for s_ in sts)) for key in ("lists", "nonempty", "fp64_outcome",
                                                                     "near_tie_outcome", "several_outcomes",
                                                                     "unresolved_incomplete", "mismatch")}
        res["fhd_parity_vs_gpu"] = {"sample_pixels": int(len(px)), "generate": gen_sum,
                                    "composite": _parity_summary(cst),
                                    "composite_pixels_skipped": int(len(px) - len(sel)),
                                    "seconds": time.time() - t0}
        log(f"[bench] fhd sample vs oracle: {res['fhd_parity_vs_gpu']}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--layout", choices=["compact", "regular"], default="regular",
                    help="layout of the FHD leg's sub-VDIs")
    ap.add_argument("--legs", default="fhd,novel,masks,large,learned,batched",
                    help="legs after the headline (novel and masks need fhd)")
    ap.add_argument("--learn-seeds", type=int, default=32)
    ap.add_argument("--learn-epochs", type=int, default=8)
    ap.add_argument("--no-learn-fhd", dest="learn_fhd", action="store_false",
                    help="skip the learned threshold on FHD-generator volumes (N=20)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device-to-device three times (a kernel of known traffic for counter scaling)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--sample-px", type=int, default=786432, help="headline pixels kept for the oracle")
    ap.add_argument("--fhd-sample-px", type=int, default=16384, help="FHD pixels compared with the oracle")
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
    dense = leg_dense(args, result)
    fhd = None
    if "fhd" in legs:
        fhd = leg_fhd(args, result)
        if "novel" in legs:
            leg_novel(args, result, fhd)
        if "masks" in legs:
            leg_masks(args, result, fhd)
    if "large" in legs:
        leg_large(args, result)
    if "learned" in legs:
        leg_learned(args, result)
        leg_learned_composite(args, result)
    if "batched" in legs:
        leg_batched(args, result)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(dense, fhd, args)
        result["cpu_baseline"]["gpu_over_cpu"] = result["value"] / result["cpu_baseline"]["value"]
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
