"""GPU parity on non-convex domains (Sec. 5.3): bricks owning the voxels of an
owner map, so rays leave a domain and enter it again.  Through the C ABI,
against the oracle (counts exact on tie-free rays, values within ATOL), the
box path (bit for bit when the map is the box partition) and whole-volume DVR."""
import numpy as np
import pytest

from paper_2206_14503_amd import synth
from conftest import gpu_available
from oracle.parity import ATOL, check_lists
from test_gpu_parity import _gpu_regular, _np

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="no GPU")]


@pytest.fixture(scope="module")
def V():
    import torch
    from paper_2206_14503_amd import vdi
    vdi.lib()
    torch.cuda.init()
    return vdi


def checker_owner(n, block, ranks=2, seed=None):
    c = np.arange(n) // block
    cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
    if seed is None:
        return ((cx + cy + cz) % ranks).astype(np.uint8)
    nc = (n + block - 1) // block
    table = np.random.default_rng(seed).integers(0, ranks, (nc, nc, nc))
    return table[cz, cy, cx].astype(np.uint8)


def whole_bricks(n, ranks):
    return [synth.Brick((0, 0, 0), (n, n, n), (0, 0, 0), (n, n, n)) for _ in range(ranks)]


def test_box_partition_as_owner_map_is_the_box_path(V):
    import torch
    n = 64
    vol = synth.gaussian_volume(n, 12, 0)
    tf_d = torch.from_numpy(synth.transfer_function()).cuda()
    cam = synth.orbit_camera(10_060, 72, 56)
    bricks = synth.brick_grid((n, n, n), (2, 1, 2))
    owner = np.zeros((n, n, n), np.uint8)
    for r, b in enumerate(bricks):
        owner[b.lo[2]:b.hi[2], b.lo[1]:b.hi[1], b.lo[0]:b.hi[0]] = r
    a = V.generate(V.device_bricks(vol, bricks), cam, tf_d, 1 / n, 1 / n, 1, 0.0, 8, 10)
    m = V.generate(V.device_bricks(vol, bricks, owner=owner, ranks=range(4)), cam, tf_d, 1 / n, 1 / n, 1, 0.0, 8, 10)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    for x, y in zip(a, m):
        for t in ("color", "depth", "count", "gamma"):
            assert torch.equal(getattr(x, t), getattr(y, t)), t


@pytest.mark.parametrize("block,ranks,seed,mode,dtype", [(8, 2, None, 1, "f32"), (6, 3, 11, 1, "f32"),
                                                         (8, 4, 12, 3, "f32"), (5, 2, 14, 1, "f16")],
                         ids=["checker8-2ranks", "random6-3ranks", "random8-4ranks-seq", "random5-2ranks-f16"])
def test_non_convex_generate_parity(V, orc, block, ranks, seed, mode, dtype):
    """Each rank's sub-VDI against the oracle (mode 3: one midpoint per pass,
    the oracle's bisection as is)."""
    import torch
    n = 64
    vol = synth.gaussian_volume(n, 12, 1)
    if dtype == "f16":
        vol = vol.astype(np.float16)
    tf = synth.transfer_function()
    tf_d = torch.from_numpy(tf).cuda()
    cam = synth.orbit_camera(10_061, 64, 48)
    owner = checker_owner(n, block, ranks, seed)
    bricks = whole_bricks(n, ranks)
    outs = V.generate(V.device_bricks(vol, bricks, owner=owner, ranks=range(ranks)), cam, tf_d, 1 / n, 1 / n,
                      mode, 0.0, 16, 10)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    ref = orc.generate(vol, bricks, cam, tf, 1 / n, 1 / n, 1, 0.0, 16, 10, owner=owner, ranks=range(ranks))
    assert (ref["contiguous"] == 0).sum() > 200
    for r in range(ranks):
        gc, gd, gn, gg = _gpu_regular(outs[r])
        check_lists((gc, gd, gn, gg), ref, f"rank {r}", brick=r)


def test_non_convex_composite_equals_dvr(V, orc):
    """Generate on three interleaved domains, composite (general merge: the
    lists interleave in depth) and render: whole-volume DVR within ATOL."""
    import torch
    n = 64
    vol = synth.gaussian_volume(n, 12, 2)
    tf = synth.transfer_function()
    tf_d = torch.from_numpy(tf).cuda()
    cam = synth.orbit_camera(10_062, 60, 44)
    owner = checker_owner(n, 8, 3, 13)
    bricks = whole_bricks(n, 3)
    outs = V.generate(V.device_bricks(vol, bricks, owner=owner, ranks=range(3)), cam, tf_d, 1 / n, 1 / n, 1, 0.0,
                      20, 10)
    comp = V.composite(outs, 1, 0.0, 60, 10)
    img = _np(V.render_original_view(comp))
    torch.cuda.synchronize()
    assert V.device_status() == 0
    ref = orc.dvr(vol, cam, tf, 1 / n, 1 / n)
    assert (ref[:, 3] > 0.05).sum() > 200
    assert np.abs(img - ref).max() <= ATOL


def test_non_convex_compact_matches_regular(V):
    import torch
    n = 64
    vol = synth.gaussian_volume(n, 12, 3)
    tf_d = torch.from_numpy(synth.transfer_function()).cuda()
    cam = synth.orbit_camera(10_063, 56, 40)
    owner = checker_owner(n, 8, 2)
    dbr = V.device_bricks(vol, whole_bricks(n, 2), owner=owner, ranks=[0, 1])
    reg = V.generate(dbr, cam, tf_d, 1 / n, 1 / n, 1, 0.0, 12, 10)
    com = V.generate(dbr, cam, tf_d, 1 / n, 1 / n, 1, 0.0, 12, 10, layout=V.COMPACT)
    torch.cuda.synchronize()
    assert V.device_status() == 0
    for a, b in zip(reg, com):
        assert torch.equal(a.count, b.count) and torch.equal(a.gamma, b.gamma)
        cnt = _np(a.count)
        off = _np(b.offset).astype(np.int64)
        ac, ad, bc, bd = _np(a.color), _np(a.depth), _np(b.color), _np(b.depth)
        for q in np.nonzero(cnt)[0][::7]:
            assert np.array_equal(ac[:cnt[q], q], bc[off[q]:off[q] + cnt[q]])
            assert np.array_equal(ad[:cnt[q], q], bd[off[q]:off[q] + cnt[q]])


def test_more_domain_entries_than_n_keeps_the_first_n(V, orc):
    """N = 2 on a fine checkerboard: rays entering a domain more than twice
    keep their first two supersegments, flagged with device status 4."""
    import torch
    n = 64
    vol = synth.gaussian_volume(n, 12, 4)
    tf = synth.transfer_function()
    tf_d = torch.from_numpy(tf).cuda()
    cam = synth.orbit_camera(10_064, 48, 36)
    owner = checker_owner(n, 4, 2)
    bricks = whole_bricks(n, 2)
    outs = V.generate(V.device_bricks(vol, bricks, owner=owner, ranks=[0, 1]), cam, tf_d, 1 / n, 1 / n, 1, 0.0, 2, 10)
    torch.cuda.synchronize()
    assert V.device_status() & 4
    ref = orc.generate(vol, bricks, cam, tf, 1 / n, 1 / n, 1, 0.0, 2, 10, owner=owner, ranks=[0, 1])
    assert (ref["count"] > 2).sum() > 100
    for r in range(2):
        gc, gd, gn, gg = _gpu_regular(outs[r])
        check_lists((gc, gd, gn, gg), ref, f"rank {r}", brick=r)


def test_owner_maps_need_a_bisection_mode(V):
    import torch
    n = 16
    vol = synth.gaussian_volume(n, 4, 5)
    tf_d = torch.from_numpy(synth.transfer_function()).cuda()
    cam = synth.orbit_camera(10_065, 16, 16)
    dbr = V.device_bricks(vol, whole_bricks(n, 2), owner=checker_owner(n, 4, 2), ranks=[0, 1])
    with pytest.raises(RuntimeError, match="bisection"):
        V.generate(dbr, cam, tf_d, 1 / n, 1 / n, 0, 0.05, 8, 10)
