"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every list must equal one of the oracle's outcomes (`parity.check_lists`):
its fp64 outcome, or, where an Eq. 1 decision's distance lies within the
near-tie band of the threshold, another outcome those near ties admit; the
same count, threshold and merge order, colours, opacities and depths within
ATOL.  Every list also satisfies the invariants of a VDI list.
"""
import numpy as np
import pytest

from paper_2206_14503_amd import synth
from conftest import gpu_available
from oracle.parity import ATOL, check_lists

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="no GPU")]


@pytest.fixture(scope="module")
def V():
    import torch
    from paper_2206_14503_amd import vdi
    vdi.lib()
    torch.cuda.init()
    return vdi


def _np(t):
    return t.detach().cpu().numpy()


def _gpu_regular(v):
    """GPU VDI -> (color [N,P,4], depth [N,P,2], count [P], gamma [P]) as numpy."""
    return _np(v.color), _np(v.depth), _np(v.count), (None if v.gamma is None else _np(v.gamma))


def _tiny_setup(V, mode, grid=(1, 1, 2), cam=None, n=64, seed=0, max_n=8, tau=0.05, dtype="f32"):
    import torch
    vol = synth.gaussian_volume(n, 12, seed)
    if dtype == "f16":
        vol = vol.astype(np.float16)
    tf = synth.transfer_function()
    cam = cam or synth.ortho_camera(256, 256, "+z")
    bricks = synth.brick_grid((n, n, n), grid)
    dbr = V.device_bricks(vol, bricks)
    tf_d = torch.from_numpy(tf).cuda()
    return vol, tf, tf_d, cam, bricks, dbr


# ---------------------------------------------------------------- rays

@pytest.mark.parametrize("cam", [synth.ortho_camera(64, 64, "+z"), synth.ortho_camera(40, 24, "-z"),
                                 synth.orbit_camera(10_000, 96, 54), synth.orbit_camera(10_001, 33, 17)],
                         ids=["ortho+z", "ortho-z", "persp", "persp-ragged"])
def test_rays_bit_exact(V, orc, cam):
    """Ray origin, direction, entry/exit and sample count are fp32 decisions:
    identical to the oracle bit for bit."""
    step = 1.0 / 64
    r = V.debug_rays(cam, step)
    o, d, tn, tf, ns = (_np(r[k]) for k in ("o", "d", "tn", "tf", "samples"))
    for p in range(cam.width * cam.height):
        info = orc.ray_info(cam, p, step)
        assert ns[p] == info["samples"], p
        assert np.array_equal(o[p], info["o"]) and np.array_equal(d[p], info["d"]), p
        if info["samples"] >= 0:
            assert tn[p] == np.float32(info["tn"]) and tf[p] == np.float32(info["tf"]), p


# ---------------------------------------------------------------- generation

@pytest.mark.parametrize("mode", [0, 1], ids=["fixed", "bisect"])
def test_generate_tiny_parity(V, orc, mode):
    """Tiny workload (64^3, 2 z-slabs, 256^2 ortho, N=8): GPU == oracle."""
    import torch
    vol, tf, tf_d, cam, bricks, dbr = _tiny_setup(V, mode)
    outs = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, mode, 0.05, 8, 10)
    torch.cuda.synchronize()
    ref = orc.generate(vol, bricks, cam, tf, 1 / 64, 1 / 64, mode, 0.05, 8, 10)
    for r in range(len(bricks)):
        gc, gd, gn, gg = _gpu_regular(outs[r])
        check_lists((gc, gd, gn, gg), ref, f"brick {r}", brick=r)


@pytest.mark.parametrize("grid,dtype,res", [((1, 1, 4), "f32", (97, 61)), ((2, 2, 2), "f16", (64, 48)),
                                            ((3, 1, 2), "f32", (50, 70))],
                         ids=["slabs-ragged", "octants-f16", "uneven"])
def test_generate_perspective_parity(V, orc, grid, dtype, res):
    """Perspective view, non-slab and uneven bricks, ragged image sizes, fp16 data."""
    import torch
    cam = synth.orbit_camera(10_010, *res)
    vol, tf, tf_d, cam, bricks, dbr = _tiny_setup(V, 1, grid=grid, cam=cam, dtype=dtype)
    outs = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, 1, 0.0, 8, 10)
    torch.cuda.synchronize()
    ref = orc.generate(vol, bricks, cam, tf, 1 / 64, 1 / 64, 1, 0.0, 8, 10)
    for r in range(len(bricks)):
        gc, gd, gn, gg = _gpu_regular(outs[r])
        check_lists((gc, gd, gn, gg), ref, f"brick {r}", brick=r)


@pytest.mark.parametrize("ratio,mode", [(0.6, 1), (1.5, 1), (0.75, 0)], ids=["short-bisect", "long-bisect", "short-fixed"])
def test_generate_step_differs_from_ref_parity(V, orc, ratio, mode):
    """Sampling distance different from the reference distance (Sec. 2.4's
    length-adjusted opacity, R7): per-sample opacity 1 - (1 - a)^(step/ref),
    supersegment lengths in units of ref, on a perspective view."""
    import torch
    cam = synth.orbit_camera(10_013, 71, 53)
    vol, tf, tf_d, cam, bricks, dbr = _tiny_setup(V, mode, grid=(1, 2, 2), cam=cam)
    step, ref_step = ratio / 64, 1 / 64
    outs = V.generate(dbr, cam, tf_d, step, ref_step, mode, 0.05, 8, 10)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    ref = orc.generate(vol, bricks, cam, tf, step, ref_step, mode, 0.05, 8, 10)
    for r in range(len(bricks)):
        gc, gd, gn, gg = _gpu_regular(outs[r])
        check_lists((gc, gd, gn, gg), ref, f"brick {r} step/ref {ratio}", brick=r)


@pytest.mark.parametrize("max_n,mode", [(1, 1), (1, 0), (64, 1)], ids=["N1-bisect", "N1-fixed", "N64-bisect"])
def test_generate_extreme_n_parity(V, orc, max_n, mode):
    """The smallest and largest supersegment budgets (N = 1: one supersegment
    per list; N = VDI_MAX_N = 64)."""
    import torch
    cam = synth.orbit_camera(10_014, 45, 38)
    vol, tf, tf_d, cam, bricks, dbr = _tiny_setup(V, mode, grid=(1, 1, 2), cam=cam)
    outs = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, mode, 0.05, max_n, 10)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    ref = orc.generate(vol, bricks, cam, tf, 1 / 64, 1 / 64, mode, 0.05, max_n, 10)
    for r in range(len(bricks)):
        gc, gd, gn, gg = _gpu_regular(outs[r])
        assert gn.max() <= max_n
        check_lists((gc, gd, gn, gg), ref, f"brick {r} N {max_n}", brick=r)


@pytest.mark.parametrize("nx,dtype", [(1, "f32"), (2, "f32"), (3, "f16")], ids=["x1", "x2", "x3-f16"])
def test_generate_thin_volume_parity(V, orc, nx, dtype):
    """Volumes one to three voxels wide in x: a one-voxel data box (single
    loads) and the x edges where both taps of a stencil row fall on one voxel
    (the first voxel below x = 0.5, the last above x = nx - 0.5)."""
    import torch
    vol = np.ascontiguousarray(synth.gaussian_volume(24, 6, 3)[:, :, :nx])
    if dtype == "f16":
        vol = vol.astype(np.float16)
    tf = synth.transfer_function()
    cam = synth.orbit_camera(10_020 + nx, 40, 30)
    bricks = synth.brick_grid((nx, 24, 24), (1, 1, 2))
    dbr = V.device_bricks(vol, bricks)
    tf_d = torch.from_numpy(tf).cuda()
    outs = V.generate(dbr, cam, tf_d, 1 / 24, 1 / 24, 1, 0.0, 8, 10)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    ref = orc.generate(vol, bricks, cam, tf, 1 / 24, 1 / 24, 1, 0.0, 8, 10)
    for r in range(len(bricks)):
        gc, gd, gn, gg = _gpu_regular(outs[r])
        assert (gn > 0).sum() > 100
        check_lists((gc, gd, gn, gg), ref, f"brick {r} nx {nx}", brick=r)


@pytest.mark.parametrize("mode", [0, 1], ids=["fixed", "bisect"])
def test_generate_compact_matches_regular(V, mode):
    """Compact layout (Sec. 4): offsets are the exclusive prefix sum of the
    counts and the stored supersegments equal the regular layout's (same kernels,
    bit for bit)."""
    import torch
    cam = synth.orbit_camera(10_011, 120, 90)
    vol, tf, tf_d, cam, bricks, dbr = _tiny_setup(V, mode, grid=(1, 2, 2), cam=cam)
    reg = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, mode, 0.05, 8, 10)
    cmp_ = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, mode, 0.05, 8, 10, layout=V.COMPACT)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    for r in range(len(bricks)):
        n = _np(reg[r].count)
        assert np.array_equal(_np(cmp_[r].count), n)
        off = _np(cmp_[r].offset).view(np.uint32)
        assert off[0] == 0 and np.array_equal(off[1:].astype(np.int64), np.cumsum(n))
        rc, rd = _np(reg[r].color), _np(reg[r].depth)
        cc, cd = _np(cmp_[r].color), _np(cmp_[r].depth)
        for p in np.nonzero(n)[0]:
            o = int(off[p])
            assert np.array_equal(cc[o:o + n[p]], rc[:n[p], p]) and np.array_equal(cd[o:o + n[p]], rd[:n[p], p])
        assert np.array_equal(_np(cmp_[r].gamma), _np(reg[r].gamma))


@pytest.mark.parametrize("iters", [10, 3], ids=["iters10", "iters3"])
def test_generate_sequential_bisection_identical(V, orc, iters):
    """BISECT_SEQ (one midpoint per pass) and BISECT (several midpoints per
    pass, decisions replayed) run the same halvings: identical VDIs and
    thresholds, bit for bit, and both match the oracle's bisection."""
    import torch
    cam = synth.orbit_camera(10_012, 83, 57)
    vol, tf, tf_d, cam, bricks, dbr = _tiny_setup(V, 1, grid=(1, 2, 2), cam=cam)
    spec = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, V.BISECT, 0.0, 6, iters)
    seq = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, V.BISECT_SEQ, 0.0, 6, iters)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    ref = orc.generate(vol, bricks, cam, tf, 1 / 64, 1 / 64, 1, 0.0, 6, iters)
    for r in range(len(bricks)):
        a, b = _gpu_regular(spec[r]), _gpu_regular(seq[r])
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        check_lists(b, ref, f"brick {r}", brick=r)


def test_generate_compact_capacity_overflow_flagged(V):
    import torch
    cam = synth.ortho_camera(64, 64, "+z")
    vol, tf, tf_d, cam, bricks, dbr = _tiny_setup(V, 1, cam=cam)
    outs = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, 1, 0.0, 8, 10, layout=V.COMPACT, capacity=100)
    torch.cuda.synchronize()
    assert V.device_status() & 1


def test_generate_empty_views(V, orc):
    """Rays that miss the volume produce empty lists with gamma 2^(1-B)."""
    import torch
    cam = synth.perspective_camera((3.0, 3.0, 3.0), (6.0, 6.0, 6.0), 32, 32)   # looking away
    vol, tf, tf_d, cam, bricks, dbr = _tiny_setup(V, 1, cam=cam)
    outs = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, 1, 0.0, 8, 10)
    torch.cuda.synchronize()
    for o in outs:
        assert int(o.count.abs().sum()) == 0
        assert torch.all(o.gamma == 2.0 ** -9)
        assert float(o.color.abs().sum()) == 0.0


# ---------------------------------------------------------------- compositing

def _oracle_inputs(orc, grid, cam, mode=1, seed=0, max_n=8):
    vol = synth.gaussian_volume(64, 12, seed)
    tf = synth.transfer_function()
    bricks = synth.brick_grid((64, 64, 64), grid)
    ref = orc.generate(vol, bricks, cam, tf, 1 / 64, 1 / 64, mode, 0.05, max_n, 10)
    return vol, tf, bricks, ref


def _to_gpu_vdis(V, ref, cam, max_n):
    import torch
    out = []
    for r in range(ref["color"].shape[0]):
        v = V.VDI(cam.width, cam.height, max_n, 1 / 64, V.REGULAR,
                  torch.from_numpy(ref["color"][r]).cuda(), torch.from_numpy(ref["depth"][r]).cuda(),
                  torch.from_numpy(ref["count"][r]).cuda(), None, None)
        out.append(v)
    return out


@pytest.mark.parametrize("grid,out_n", [((1, 1, 2), 8), ((2, 2, 2), 8), ((1, 1, 4), 5), ((2, 2, 2), 64)],
                         ids=["slabs", "octants", "reduce", "passthrough"])
def test_composite_parity(V, orc, grid, out_n):
    """Same fp32 inputs on both sides: exact merge order (pass-through slots are
    bit-identical), exact counts on tie-free rays, values within ATOL."""
    import torch
    cam = synth.orbit_camera(10_020, 80, 64)
    vol, tf, bricks, ref = _oracle_inputs(orc, grid, cam)
    ins = _to_gpu_vdis(V, ref, cam, 8)
    out = V.composite(ins, V.BISECT, 0.0, out_n, 10)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    k = len(bricks)
    oref = orc.composite([ref["color"][r] for r in range(k)], [ref["depth"][r] for r in range(k)],
                         [ref["count"][r] for r in range(k)], 1 / 64, 1, 0.0, out_n, 10)
    gc, gd, gn, gg = _gpu_regular(out)
    total = ref["count"].sum(axis=0)
    pt = total <= out_n
    assert np.array_equal(gn[pt], total[pt])
    assert np.array_equal(gc[:, pt], oref["color"][:, pt]) and np.array_equal(gd[:, pt], oref["depth"][:, pt])
    check_lists((gc, gd, gn, gg), oref, "composite")


def test_composite_fixed_mode_parity(V, orc):
    import torch
    cam = synth.ortho_camera(128, 128, "+z")
    vol, tf, bricks, ref = _oracle_inputs(orc, (1, 1, 2), cam, mode=0)
    ins = _to_gpu_vdis(V, ref, cam, 8)
    out = V.composite(ins, V.FIXED, 0.05, 8, 10)
    torch.cuda.synchronize()
    oref = orc.composite([ref["color"][r] for r in range(2)], [ref["depth"][r] for r in range(2)],
                         [ref["count"][r] for r in range(2)], 1 / 64, 0, 0.05, 8, 10)
    gc, gd, gn, gg = _gpu_regular(out)
    check_lists((gc, gd, gn, gg), oref, "composite-fixed")


def test_composite_interleaved_stress_parity(V, orc):
    """Maximally interleaved synthetic lists (k=16, 20 each, N=20): every
    pixel needs the full merge and bisection."""
    import torch
    k, n, P = 16, 20, 512
    col, dep, cnt = synth.dense_interleaved_lists(k, n, P, seed=3)
    ins = [V.VDI(32, 16, n, 0.01, V.REGULAR, col[r].cuda().contiguous(), dep[r].cuda().contiguous(),
                 cnt[r].cuda().contiguous()) for r in range(k)]
    out = V.composite(ins, V.BISECT, 0.0, 20, 10)
    torch.cuda.synchronize()
    c, d, m = col.numpy(), dep.numpy(), cnt.numpy()
    oref = orc.composite([c[r] for r in range(k)], [d[r] for r in range(k)], [m[r] for r in range(k)], 0.01, 1, 0.0,
                         20, 10)
    gc, gd, gn, gg = _gpu_regular(out)
    check_lists((gc, gd, gn, gg), oref, "stress")


@pytest.mark.parametrize("k,n,out_n", [(24, 6, 10), (24, 2, 48), (32, 4, 12)],
                         ids=["k24-bisect", "k24-passthrough", "k32-bisect"])
def test_composite_many_inputs_ragged_parity(V, orc, k, n, out_n):
    """k = 24 and k = VDI_MAX_INPUTS = 32 interleaved inputs (above the
    depth-disjoint path's 16), ragged list lengths 0..n and a ragged last
    pixel block (300 pixels): the general merge over every pixel."""
    import torch
    W, H = 20, 15
    P = W * H
    col, dep, cnt = synth.dense_interleaved_lists(k, n, P, seed=7)
    rng = np.random.default_rng(7)
    cnt = torch.from_numpy(rng.integers(0, n + 1, size=(k, P)).astype(np.int32))
    for r in range(k):
        for j in range(n):
            unused = cnt[r] <= j
            col[r, j, unused] = 0.0
            dep[r, j, unused] = 0.0
    ins = [V.VDI(W, H, n, 0.01, V.REGULAR, col[r].cuda().contiguous(), dep[r].cuda().contiguous(),
                 cnt[r].cuda().contiguous()) for r in range(k)]
    out = V.composite(ins, V.BISECT, 0.0, out_n, 10)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    c, d, m = col.numpy(), dep.numpy(), cnt.numpy()
    oref = orc.composite([c[r] for r in range(k)], [d[r] for r in range(k)], [m[r] for r in range(k)], 0.01, 1, 0.0,
                         out_n, 10)
    gc, gd, gn, gg = _gpu_regular(out)
    check_lists((gc, gd, gn, gg), oref, f"k{k} N{out_n}")


@pytest.mark.parametrize("out_n", [4, 30], ids=["bisect", "passthrough"])
def test_composite_mixed_disjoint_and_interleaved(V, orc, out_n):
    """One launch where half of the pixels hold depth-disjoint lists (in a
    seeded per-pixel order, so the depth-disjoint path must sort them) and the
    other half interleaved lists (general merge); one input compact.  Counts,
    merge order and values match the oracle."""
    import torch
    import oracle
    k, n, W, H = 5, 6, 24, 20
    P = W * H
    col, dep, cnt = synth.dense_interleaved_lists(k, n, P, seed=11)
    rng = np.random.default_rng(11)
    cnt = torch.from_numpy(rng.integers(0, n + 1, size=(k, P)).astype(np.int32))
    dep = dep.clone()
    col = col.clone()
    for px in range(0, P, 2):       # even pixels: each input in its own depth band
        perm = rng.permutation(k)
        for r in range(k):
            dep[r, :, px] += float(perm[r]) * 100.0
    for r in range(k):
        for slot in range(n):
            dead = cnt[r] <= slot
            col[r, slot, dead] = 0
            dep[r, slot, dead] = 0
    ins = []
    for r in range(k):
        if r == 2:
            off, cc, dd = oracle.to_compact(col[r].numpy(), dep[r].numpy(), cnt[r].numpy())
            ins.append(V.VDI(W, H, n, 0.01, V.COMPACT, torch.from_numpy(cc).cuda(), torch.from_numpy(dd).cuda(),
                             cnt[r].cuda(), torch.from_numpy(off.view(np.int32)).cuda()))
        else:
            ins.append(V.VDI(W, H, n, 0.01, V.REGULAR, col[r].cuda().contiguous(), dep[r].cuda().contiguous(),
                             cnt[r].cuda().contiguous()))
    out = V.composite(ins, V.BISECT, 0.0, out_n, 10)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    c, d, m = col.numpy(), dep.numpy(), cnt.numpy()
    oref = orc.composite([c[r] for r in range(k)], [d[r] for r in range(k)], [m[r] for r in range(k)], 0.01, 1, 0.0,
                         out_n, 10)
    gc, gd, gn, gg = _gpu_regular(out)
    total = m.sum(axis=0)
    pt = total <= out_n
    assert np.array_equal(gc[:, pt], oref["color"][:, pt]) and np.array_equal(gd[:, pt], oref["depth"][:, pt])
    check_lists((gc, gd, gn, gg), oref, "mixed")


def test_composite_identity_with_empty_inputs(V, orc):
    """Invariant (a) on the GPU: a VDI composited with empty VDIs is returned bit for bit."""
    import torch
    cam = synth.orbit_camera(10_021, 64, 48)
    vol, tf, bricks, ref = _oracle_inputs(orc, (1, 1, 2), cam)
    ins = _to_gpu_vdis(V, ref, cam, 8)
    empty = V.VDI(cam.width, cam.height, 8, 1 / 64, V.REGULAR, torch.zeros_like(ins[0].color),
                  torch.zeros_like(ins[0].depth), torch.zeros_like(ins[0].count))
    for pos in range(3):
        lst = [empty, empty]
        lst.insert(pos, ins[0])
        out = V.composite(lst, V.BISECT, 0.0, 8, 10)
        torch.cuda.synchronize()
        assert torch.equal(out.color, ins[0].color) and torch.equal(out.depth, ins[0].depth)
        assert torch.equal(out.count, ins[0].count)


def test_composite_rejects_invalid_lists(V):
    import torch
    c = torch.zeros((2, 4, 4), device="cuda")
    d = torch.zeros((2, 4, 2), device="cuda")
    d[0, 0] = torch.tensor([2.0, 3.0]); d[1, 0] = torch.tensor([0.0, 1.0])   # unsorted
    c[:, 0, 3] = 0.5
    n = torch.tensor([2, 0, 0, 9], dtype=torch.int32, device="cuda")         # 9 > max_n
    v = V.VDI(2, 2, 2, 1.0, V.REGULAR, c, d, n)
    out = V.composite([v], V.BISECT, 0.0, 2, 10)
    torch.cuda.synchronize()
    assert V.device_status() & 2
    assert out.count[0].item() == 0 and out.count[3].item() == 0


def test_api_argument_errors(V):
    import torch
    c = torch.zeros((2, 4, 4), device="cuda"); d = torch.zeros((2, 4, 2), device="cuda")
    n = torch.zeros(4, dtype=torch.int32, device="cuda")
    v = V.VDI(2, 2, 2, 1.0, V.REGULAR, c, d, n)
    bad = V.VDI(3, 2, 2, 1.0, V.REGULAR, c, d, n)
    with pytest.raises(V.VdiError):
        V.composite([v, bad], V.BISECT, 0.0, 2, 10)
    with pytest.raises(V.VdiError):
        V.composite([v], V.BISECT, 0.0, 2, 0)
    with pytest.raises(V.VdiError):
        V.composite([v], V.BISECT_SEQ, 0.0, 2, 10)   # generation only


# ---------------------------------------------------------------- rendering and end to end

def test_render_parity(V, orc):
    import torch
    cam = synth.orbit_camera(10_030, 80, 60)
    vol, tf, bricks, ref = _oracle_inputs(orc, (1, 1, 2), cam)
    ins = _to_gpu_vdis(V, ref, cam, 8)
    for r in range(2):
        img = _np(V.render_original_view(ins[r]))
        want = orc.render_ov(ref["color"][r], ref["depth"][r], ref["count"][r], 1 / 64)
        assert np.abs(img - want).max() <= ATOL


@pytest.mark.parametrize("grid,mode,out_n", [((1, 1, 2), 0, 8), ((1, 1, 4), 1, 8), ((2, 2, 2), 1, 6)],
                         ids=["tiny-fixed", "slabs-bisect", "octants-bisect"])
def test_end_to_end_equals_dvr(V, orc, grid, mode, out_n):
    """Invariant (b) on the GPU: render(composite(generate(bricks))) equals the
    oracle's DVR of the whole volume (Sec. 2.3 exactness of over)."""
    import torch
    cam = synth.orbit_camera(10_031, 96, 72) if grid != (1, 1, 2) else synth.ortho_camera(256, 256, "+z")
    vol, tf, tf_d, cam, bricks, dbr = _tiny_setup(V, mode, grid=grid, cam=cam)
    outs = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, mode, 0.05, 8, 10)
    comp = V.composite(outs, mode, 0.05, out_n, 10)
    img = _np(V.render_original_view(comp))
    ref = orc.dvr(vol, cam, tf, 1 / 64, 1 / 64)
    assert np.abs(img - ref).max() <= ATOL
    assert int(comp.count.max()) <= out_n


# ---------------------------------------------------------------- novel-view rendering

def _oracle_composited(orc, cam, seed=0):
    vol, tf, bricks, ref = _oracle_inputs(orc, (1, 1, 2), cam, mode=1, seed=seed)
    return orc.composite([ref["color"][r] for r in range(2)], [ref["depth"][r] for r in range(2)],
                         [ref["count"][r] for r in range(2)], 1 / 64, 1, 0.0, 8, 10)


@pytest.mark.parametrize("vcam,view,step", [
    (synth.orbit_camera(10_040, 64, 48), synth.orbit_camera(10_040, 56, 40, turn_deg=10.0), 1 / 64),
    (synth.orbit_camera(10_041, 64, 48), synth.orbit_camera(10_041, 64, 48), 1 / 64),
    (synth.orbit_camera(10_042, 48, 48), synth.orbit_camera(10_042, 40, 30, turn_deg=50.0), 1 / 48),
    (synth.ortho_camera(64, 64, "+z"), synth.orbit_camera(10_043, 50, 38), 1 / 80),
    (synth.orbit_camera(10_046, 64, 48), synth.ortho_camera(40, 40, "-z"), 1 / 64),
], ids=["persp-10deg", "persp-own-view", "persp-50deg-coarse-ragged", "ortho-vdi-fine", "persp-vdi-ortho-view"])
def test_render_novel_view_parity(V, orc, vcam, view, step):
    """A composited VDI (the oracle's, uploaded) rendered from another
    viewpoint: the pixel and supersegment of every sample are fp64 decisions
    taken identically on both sides, so the images agree within ATOL."""
    import torch
    c = _oracle_composited(orc, vcam)
    v = V.VDI(vcam.width, vcam.height, 8, 1 / 64, V.REGULAR, torch.from_numpy(c["color"]).cuda(),
              torch.from_numpy(c["depth"]).cuda(), torch.from_numpy(c["count"]).cuda(), None, None)
    g = _np(V.render_novel_view(v, vcam, view, step))
    torch.cuda.synchronize()
    assert V.device_status() == 0
    ref = orc.novel_view(c["color"], c["depth"], c["count"], 1 / 64, vcam, view, step)
    assert (ref[:, 3] > 0.01).sum() > 100
    err = np.abs(g - ref).max()
    assert err <= ATOL, f"max |gpu - oracle| {err:.3g}"


def test_render_novel_view_compact_parity(V, orc):
    """The same lists in the compact layout (offsets), against the oracle."""
    import torch
    vcam = synth.orbit_camera(10_044, 48, 40)
    c = _oracle_composited(orc, vcam)
    cnt = c["count"]
    P = cnt.size
    off = np.zeros(P + 1, np.int64)
    off[1:] = np.cumsum(cnt)
    m = int(off[-1])
    cc = np.zeros((m, 4), np.float32)
    dd = np.zeros((m, 2), np.float32)
    for q in range(P):
        cc[off[q]:off[q + 1]] = c["color"][:cnt[q], q]
        dd[off[q]:off[q + 1]] = c["depth"][:cnt[q], q]
    v = V.VDI(vcam.width, vcam.height, 8, 1 / 64, V.COMPACT, torch.from_numpy(cc).cuda(),
              torch.from_numpy(dd).cuda(), torch.from_numpy(cnt).cuda(),
              torch.from_numpy(off.astype(np.int32)).cuda(), None)
    view = synth.orbit_camera(10_044, 44, 36, turn_deg=-25.0)
    g = _np(V.render_novel_view(v, vcam, view, 1 / 64))
    torch.cuda.synchronize()
    assert V.device_status() == 0
    ref = orc.novel_view(cc, dd, cnt, 1 / 64, vcam, view, 1 / 64, offset=off[:-1].astype(np.uint32))
    assert (ref[:, 3] > 0.01).sum() > 100
    assert np.abs(g - ref).max() <= ATOL


def test_render_novel_view_from_own_camera_equals_original_view(V, orc):
    """A GPU-generated and composited VDI seen from its own camera on its own
    grid equals its original-view rendering (up to the fp32 depths)."""
    import torch
    vcam = synth.orbit_camera(10_045, 64, 48)
    vol, tf, tf_d, cam, bricks, dbr = _tiny_setup(V, 1, grid=(1, 1, 2), cam=vcam)
    outs = V.generate(dbr, vcam, tf_d, 1 / 64, 1 / 64, 1, 0.0, 8, 10)
    comp = V.composite(outs, 1, 0.0, 8, 10)
    ov = _np(V.render_original_view(comp))
    nv = _np(V.render_novel_view(comp, vcam, vcam, 1 / 64))
    torch.cuda.synchronize()
    assert V.device_status() == 0
    assert (ov[:, 3] > 0.01).sum() > 100
    assert np.abs(nv - ov).max() <= 2e-5
