"""Batched persistent compositing: every job equals vdi_composite on its own
(bit for bit), graph replays equal the eager run, per-job device timestamps
are ordered, the autotuner writes a cache the batch reads, and a sampled job
matches the oracle."""
import os

import numpy as np
import pytest

from paper_2206_14503_amd import synth
from conftest import gpu_available
from oracle.parity import check_lists

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="no GPU")]


@pytest.fixture(scope="module")
def V():
    import torch
    from paper_2206_14503_amd import vdi
    vdi.lib()
    torch.cuda.init()
    return vdi


def _stress_inputs(V, k, n_per, w, h, seed, compact_mask=0):
    import torch
    import oracle
    col, dep, cnt = synth.dense_interleaved_lists(k, n_per, w * h, seed=seed)
    # drop a seeded share of each list's tail so counts vary per pixel
    rng = np.random.default_rng(seed)
    cnt = torch.from_numpy(rng.integers(0, n_per + 1, size=(k, w * h)).astype(np.int32))
    col = col.clone()
    dep = dep.clone()
    for r in range(k):
        for s in range(n_per):
            dead = (cnt[r] <= s)
            col[r, s, dead] = 0
            dep[r, s, dead] = 0
    vd = []
    for r in range(k):
        if (compact_mask >> r) & 1:
            off, cc, dd = oracle.to_compact(col[r].numpy(), dep[r].numpy(), cnt[r].numpy())
            v = V.VDI(w, h, n_per, 0.01, V.COMPACT, torch.from_numpy(cc).cuda(), torch.from_numpy(dd).cuda(),
                      cnt[r].cuda(), torch.from_numpy(off.view(np.int32)).cuda())
        else:
            v = V.VDI(w, h, n_per, 0.01, V.REGULAR, col[r].cuda().contiguous(), dep[r].cuda().contiguous(),
                      cnt[r].cuda().contiguous())
        vd.append(v)
    return vd, (col.numpy(), dep.numpy(), cnt.numpy())


def _jobs(V):
    specs = [  # (k, n_per, out_n, w, h, seed, compact_mask, mode)
        (1, 8, 8, 40, 30, 1, 0, 1),
        (3, 6, 8, 64, 48, 2, 0b010, 1),
        (8, 4, 20, 97, 61, 3, 0b10101010, 1),
        (16, 3, 32, 33, 17, 4, 0xFFFF, 1),
        (5, 10, 4, 50, 50, 5, 0, 1),
        (4, 12, 16, 64, 64, 6, 0b1111, 0),
        (20, 2, 12, 30, 20, 7, 0b101, 1),      # more inputs than the depth-disjoint path takes
    ]
    jobs, raw = [], []
    for k, n_per, out_n, w, h, seed, cm, mode in specs:
        ins, arrays = _stress_inputs(V, k, n_per, w, h, seed, cm)
        out = V.VDI.empty(w, h, out_n, 0.01)
        jobs.append(V.Job(ins, out, mode=mode, tau=0.3, iters=10))
        raw.append(arrays)
    return jobs, raw


def _snapshot(v):
    return [t.detach().clone() for t in (v.color, v.depth, v.count, v.gamma)]


def test_batch_matches_single_composites(V):
    import torch
    jobs, _ = _jobs(V)
    refs = []
    for j in jobs:
        out = V.composite(j.inputs, int(j.tau.mode), j.tau.tau, j.out.max_n, 10)
        refs.append(_snapshot(out))
    b = V.Batch(jobs)
    b.run()
    torch.cuda.synchronize()
    assert V.device_status() == 0
    for j, ref in zip(jobs, refs):
        for a, r in zip(_snapshot(j.out), ref):
            assert torch.equal(a, r)
    lat, span = b.latencies_s()
    t = b.t_se.view(-1, 2).cpu().numpy().astype(np.uint64)
    assert np.all(t[:, 0] <= t[:, 1]) and np.all(t[:, 1] > 0)
    assert span > 0 and np.all(lat >= 0)


def test_batch_graph_replay_matches_eager(V):
    """Three replays of the captured graph, with eager work and output resets
    between them, each equal the eager run."""
    import torch
    jobs, _ = _jobs(V)
    b = V.Batch(jobs)
    b.run()
    torch.cuda.synchronize()
    eager = [_snapshot(j.out) for j in jobs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.capture(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for j in jobs:
            j.out.color.fill_(-1.0)
            j.out.count.fill_(-7)
        junk = torch.randn(1 << 20, device="cuda").sum()      # unrelated eager work
        torch.cuda.synchronize()
        b.replay(s)
        s.synchronize()
        for j, ref in zip(jobs, eager):
            for a, r in zip(_snapshot(j.out), ref):
                assert torch.equal(a, r), rep
        assert torch.isfinite(junk)


def test_batch_job_matches_oracle(V, orc):
    """A batched job built from oracle-generated sub-VDIs matches the oracle composite."""
    import torch
    cam = synth.orbit_camera(10_050, 72, 54)
    vol = synth.gaussian_volume(64, 12, 6)
    tf = synth.transfer_function()
    bricks = synth.brick_grid((64, 64, 64), (2, 2, 2))
    ref = orc.generate(vol, bricks, cam, tf, 1 / 64, 1 / 64, 1, 0.0, 8, 10)
    ins = [V.VDI(cam.width, cam.height, 8, 1 / 64, V.REGULAR, torch.from_numpy(ref["color"][r]).cuda(),
                 torch.from_numpy(ref["depth"][r]).cuda(), torch.from_numpy(ref["count"][r]).cuda())
           for r in range(8)]
    out = V.VDI.empty(cam.width, cam.height, 6, 1 / 64)
    jobs, _ = _jobs(V)
    jobs = jobs[:2] + [V.Job(ins, out, mode=V.BISECT, iters=10)]
    V.Batch(jobs).run()
    torch.cuda.synchronize()
    oref = orc.composite([ref["color"][r] for r in range(8)], [ref["depth"][r] for r in range(8)],
                         [ref["count"][r] for r in range(8)], 1 / 64, 1, 0.0, 6, 10)
    g = out.gamma.cpu().numpy() if out.gamma is not None else None
    check_lists((out.color.cpu().numpy(), out.depth.cpu().numpy(), out.count.cpu().numpy(), g), oref, "batched job")


def test_autotune_cache_roundtrip(V, tmp_path):
    import torch
    jobs, _ = _jobs(V)
    path = str(tmp_path / "tiles.txt")
    V.autotune(jobs[:3], path)
    lines = open(path).read().split("\n")
    rows = [l.split() for l in lines if l.strip()]
    assert len(rows) >= 2
    for r in rows:
        assert r[0].startswith("gfx950") and int(r[3]) in (64, 128, 256, 512, 1024) and float(r[4]) > 0
    refs = [_snapshot(j.out) for j in jobs[:3]]
    b = V.Batch(jobs[:3], autotune_cache=path)
    for j in jobs[:3]:
        j.out.count.fill_(-1)
    b.run()
    torch.cuda.synchronize()
    for j, ref in zip(jobs[:3], refs):
        assert torch.equal(j.out.count, ref[2])


def test_batch_rejects_bad_jobs(V):
    import torch
    jobs, _ = _jobs(V)
    bad = V.Job(jobs[0].inputs, V.VDI.empty(41, 30, 8, 0.01))   # size differs from its inputs
    with pytest.raises(V.VdiError):
        V.Batch([jobs[1], bad])
