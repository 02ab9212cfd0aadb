"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times: the whole frame runs on the GPU, the oracle computes a
seeded sample of 65,536 pixels one by one, and every sampled list must equal
one of the oracle's outcomes (`parity.check_lists`: the fp64 outcome or
another one near ties admit; invariants on every list).

  * FHD: 512^3 fp32 (200 Gaussians + noise), 8 z-slabs, 1920x1080
    perspective, bisection to N=20: the 8 generated sub-VDIs, then the
    composite, whose inputs at the sampled pixels are the oracle's own lists
    (written into the GPU's sub-VDIs before the launch), so both sides
    composite the same fp32 inputs;
  * large generated: 1024^3 fp16 in 16 bricks (4x2x2), same camera and N;
  * large dense: 16 maximally interleaved inputs of 20 supersegments per pixel
    (the headline compositing case), N=20.
"""
import numpy as np
import pytest

from paper_2206_14503_amd import synth
from conftest import gpu_available
from oracle.parity import check_lists

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="no GPU")]

SAMPLE = 65536


@pytest.fixture(scope="module")
def V():
    import torch
    from paper_2206_14503_amd import vdi
    vdi.lib()
    torch.cuda.init()
    return vdi


def _sample(P, seed):
    return np.sort(np.random.default_rng(seed).choice(P, size=SAMPLE, replace=False)).astype(np.int32)


def _cols(v, idx):
    """GPU regular VDI at pixel columns idx (a device index tensor) as numpy."""
    g = None if v.gamma is None else v.gamma[idx].cpu().numpy()
    return v.color[:, idx].cpu().numpy(), v.depth[:, idx].cpu().numpy(), v.count[idx].cpu().numpy(), g


def _generated_case(V, orc, w, label):
    import torch
    vol = synth.workload_volume(w, device="cuda")
    bricks = synth.brick_grid((w.n,) * 3, w.grid)
    dbr = V.device_bricks(vol, bricks)
    host = vol.cpu().numpy()
    del vol
    tf = synth.transfer_function()
    tf_d = torch.from_numpy(tf).cuda()
    cam = synth.camera_for(w)
    step = 1.0 / w.n
    P = cam.width * cam.height
    print(f"[{label}] {w.name}: GPU generate + composite of the whole frame", flush=True)
    subs = [V.VDI.empty(cam.width, cam.height, w.max_n, step, V.REGULAR) for _ in bricks]
    V.generate(dbr, cam, tf_d, step, step, V.BISECT, 0.0, w.max_n, w.iters, outs=subs)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    px = _sample(P, 2024 + w.n)
    idx = torch.from_numpy(px).long().cuda()
    print(f"[{label}] oracle generate on {len(px)} sampled pixels x {len(bricks)} bricks", flush=True)
    ref = orc.generate(host, bricks, cam, tf, step, step, orc.BISECT, 0.0, w.max_n, w.iters, pixels=px)
    stats = []
    for r in range(len(bricks)):
        stats.append(check_lists(_cols(subs[r], idx), ref, f"{label} brick {r}", brick=r))
    fp64 = sum(s["fp64_outcome"] for s in stats)
    alt = sum(s["near_tie_outcome"] for s in stats)
    ne = sum(s["nonempty"] for s in stats)
    print(f"[{label}] generation: {ne} non-empty sampled lists; {fp64} equal the fp64 outcome, {alt} another "
          f"near-tie outcome; {sum(s['several_outcomes'] for s in stats)} admit several", flush=True)
    # the GPU takes the fp64 branch on all but a few near ties
    assert alt <= 0.005 * ne
    # composite: the oracle's lists at the sampled pixels on both sides
    k = len(bricks)
    for r in range(k):
        subs[r].color[:, idx] = torch.from_numpy(ref["color"][r]).cuda()
        subs[r].depth[:, idx] = torch.from_numpy(ref["depth"][r]).cuda()
        subs[r].count[idx] = torch.from_numpy(ref["count"][r]).cuda()
    out = V.composite(subs, V.BISECT, 0.0, w.max_n, w.iters)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    oref = orc.composite([ref["color"][r] for r in range(k)], [ref["depth"][r] for r in range(k)],
                         [ref["count"][r] for r in range(k)], step, orc.BISECT, 0.0, w.max_n, w.iters)
    st = check_lists(_cols(out, idx), oref, f"{label} composite")
    print(f"[{label}] composite: {st}", flush=True)
    assert st["near_tie_outcome"] <= 0.005 * st["nonempty"]


def test_fhd_frame_sample_parity(V, orc):
    _generated_case(V, orc, synth.fhd(0), "fhd")


def test_large_generated_frame_sample_parity(V, orc):
    _generated_case(V, orc, synth.large(0), "large")


def test_large_dense_frame_sample_parity(V, orc):
    import torch
    w = synth.large(0)
    cam = synth.camera_for(w)
    P = cam.width * cam.height
    k, n = 16, 20
    print(f"[dense] {k} x {n} interleaved supersegments per pixel, {cam.width}x{cam.height}, N={n}", flush=True)
    color, depth, count = synth.dense_frame(k, n, P, seed=0)
    ins = [V.VDI(cam.width, cam.height, n, 0.01, V.REGULAR, color[r], depth[r], count[r]) for r in range(k)]
    out = V.composite(ins, V.BISECT, 0.0, n, 10)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    px = _sample(P, 77)
    idx = torch.from_numpy(px).long().cuda()
    c = color[:, :, idx].cpu().numpy()
    d = depth[:, :, idx].cpu().numpy()
    m = count[:, idx].cpu().numpy()
    print(f"[dense] oracle composite on {len(px)} sampled pixels", flush=True)
    oref = orc.composite([c[r] for r in range(k)], [d[r] for r in range(k)], [m[r] for r in range(k)], 0.01,
                         orc.BISECT, 0.0, n, 10)
    st = check_lists(_cols(out, idx), oref, "dense composite")
    print(f"[dense] composite: {st}", flush=True)
    assert st["near_tie_outcome"] <= 0.005 * st["nonempty"]
