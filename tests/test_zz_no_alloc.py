"""vdi_composite_noalloc (scratch in the library's fixed device array) against
vdi_composite through the C-ABI: two calls in a row on one device, the second
with a smaller input, each bit for bit equal to vdi_composite on the same
inputs; sizes beyond the fixed array are rejected on the host."""
import pytest
import torch

from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def V():
    from paper_2206_14503_amd import vdi
    return vdi


def _inputs(V, res, grid, seed, N=8):
    from paper_2206_14503_amd import synth
    n = 64
    vol = synth.gaussian_volume(n, 12, seed=seed)
    bricks = synth.brick_grid((n, n, n), grid)
    cam = synth.orbit_camera(10_000 + seed, res[0], res[1])
    tf_d = torch.from_numpy(synth.transfer_function()).cuda()
    return V.generate(V.device_bricks(vol, bricks), cam, tf_d, 1.0 / n, 1.0 / n, V.BISECT, 0.0, N, 10)


def _dense(V, k, n, w, h, seed):
    from paper_2206_14503_amd import synth
    c, d, cnt = synth.dense_interleaved_lists(k, n, w * h, seed=seed, device="cuda")
    return [V.VDI(w, h, n, 0.01, V.REGULAR, c[r].contiguous(), d[r].contiguous(), cnt[r].contiguous())
            for r in range(k)]


def _equal(a, b):
    return (torch.equal(a.color, b.color) and torch.equal(a.depth, b.depth) and torch.equal(a.count, b.count)
            and torch.equal(a.gamma, b.gamma))


@pytest.mark.parametrize("case", ["generated", "interleaved"])
def test_noalloc_equals_composite_twice_second_smaller(V, case):
    if case == "generated":
        big, small = _inputs(V, (160, 120), (2, 2, 2), 5), _inputs(V, (72, 40), (1, 2, 2), 6)
        N = 8
    else:
        big, small = _dense(V, 6, 6, 200, 90, 11), _dense(V, 4, 5, 37, 29, 12)
        N = 10
    for mode in (V.BISECT, V.FIXED):
        for ins in (big, small):
            w, h = ins[0].width, ins[0].height
            ref = V.composite(ins, mode, 0.05, N, 10)
            out = V.VDI.empty(w, h, N, ins[0].ref_step, V.REGULAR)
            out.color.fill_(7.0)
            out.depth.fill_(7.0)
            out.count.fill_(-3)
            out.gamma.fill_(7.0)
            V.composite(ins, mode, 0.05, N, 10, out=out, noalloc=True)
            torch.cuda.synchronize()
            assert _equal(out, ref), f"{case} {w}x{h} mode {mode}: noalloc differs from vdi_composite"
    assert V.device_status() == 0


def test_noalloc_rejects_sizes_beyond_its_array(V):
    w, h = 4096, 2100      # 8.6M pixels: the queue alone exceeds 32 MiB
    c = torch.zeros((1, w * h, 4), dtype=torch.float32, device="cuda")
    d = torch.zeros((1, w * h, 2), dtype=torch.float32, device="cuda")
    cnt = torch.zeros((w * h,), dtype=torch.int32, device="cuda")
    ins = [V.VDI(w, h, 1, 0.01, V.REGULAR, c, d, cnt)]
    out = V.VDI.empty(w, h, 1, 0.01, V.REGULAR)
    with pytest.raises(V.VdiError) as e:
        V.composite(ins, V.BISECT, 0.0, 1, 10, out=out, noalloc=True)
    assert e.value.status == -2 and "fixed" in str(e.value)
