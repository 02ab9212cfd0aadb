"""Workspace of the ops through the C-ABI: the size query, a caller-owned
workspace (no allocation inside the ops), a too-small workspace reported as
VDI_E_WORKSPACE, and generation + compositing captured in a HIP graph straight
after the query, replayed to the eager outputs bit for bit."""
import numpy as np
import pytest
import torch

from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def V():
    from paper_2206_14503_amd import vdi
    return vdi


def _frame(V, n=64, res=96, grid=(1, 1, 2), seed=3):
    from paper_2206_14503_amd import synth
    vol = synth.gaussian_volume(n, 12, seed=seed)
    bricks = synth.brick_grid((n, n, n), grid)
    cam = synth.orbit_camera(10_000 + seed, res, res)
    tf_d = torch.from_numpy(synth.transfer_function()).cuda()
    return V.device_bricks(vol, bricks), cam, tf_d, 1.0 / n


def _same(a, b):
    return torch.equal(a.color, b.color) and torch.equal(a.depth, b.depth) and torch.equal(a.count, b.count)


def test_workspace_query_shapes(V):
    g = V.workspace_size(V.OP_GENERATE, 640, 480, 4, V.REGULAR, V.BISECT)
    assert g == 0                                  # regular bisection needs no scratch
    gc = V.workspace_size(V.OP_GENERATE, 640, 480, 4, V.COMPACT, V.BISECT)
    assert gc >= 640 * 480 * 4                     # gamma planes and scan partials
    gl = V.workspace_size(V.OP_GENERATE, 640, 480, 4, V.REGULAR, V.LEARNED)
    assert gl >= 640 * 480 * 4 * 128               # bf16 histograms of every brick-ray
    c = V.workspace_size(V.OP_COMPOSITE, 640, 480, 4, in_max_n_sum=32)
    assert c >= 640 * 480 * 4                      # the general-merge queue
    m = V.workspace_size(V.OP_MLP_BACKWARD, rows=4096)
    assert m >= V.MLP_PARAMS * 4
    with pytest.raises(V.VdiError):
        V.workspace_size(V.OP_COMPOSITE, 640, 480, 0, in_max_n_sum=8)
    with pytest.raises(V.VdiError):
        V.workspace_size(99, 640, 480, 2)


def test_too_small_workspace_is_reported(V):
    """Below the queues and two minimal chunks the composite reports
    VDI_E_WORKSPACE; just below the recommended size it stages in smaller
    chunks and gives the same output."""
    dbr, cam, tf_d, step = _frame(V)
    need = V.workspace_size(V.OP_COMPOSITE, cam.width, cam.height, 2, in_max_n_sum=16)
    subs = V.generate(dbr, cam, tf_d, step, step, V.BISECT, 0.0, 8, 10)
    ref = V.composite(subs, V.BISECT, 0.0, 8, 10)
    tiny = torch.empty(1024, dtype=torch.uint8, device="cuda")
    V.set_workspace(tiny)
    try:
        with pytest.raises(V.VdiError) as e:
            V.composite(subs, V.BISECT, 0.0, 8, 10)
        assert e.value.status == -6
    finally:
        V.set_workspace(None)
    near = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    V.set_workspace(near)
    try:
        out = V.composite(subs, V.BISECT, 0.0, 8, 10)
        torch.cuda.synchronize()
        assert _same(out, ref)
    finally:
        V.set_workspace(None)


@pytest.mark.parametrize("layout", ["regular", "compact"])
def test_graph_capture_after_workspace_query(V, layout):
    dbr, cam, tf_d, step = _frame(V)
    lay = V.COMPACT if layout == "compact" else V.REGULAR
    k, N, P = len(dbr), 8, cam.width * cam.height
    need = max(V.workspace_size(V.OP_GENERATE, cam.width, cam.height, k, lay, V.BISECT),
               V.workspace_size(V.OP_COMPOSITE, cam.width, cam.height, k, in_max_n_sum=k * N))
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
    V.set_workspace(ws)
    try:
        subs = [V.VDI.empty(cam.width, cam.height, N, step, lay, capacity=N * P) for _ in range(k)]
        out = V.VDI.empty(cam.width, cam.height, N, step, V.REGULAR)
        img = torch.empty((P, 4), dtype=torch.float32, device="cuda")

        def step_fn():
            V.generate(dbr, cam, tf_d, step, step, V.BISECT, 0.0, N, 10, layout=lay, outs=subs)
            V.composite(subs, V.BISECT, 0.0, N, 10, out=out)
            V.render_original_view(out, img)

        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step_fn()
        s.synchronize()
        ref_out = V.VDI(out.width, out.height, N, step, V.REGULAR, out.color.clone(), out.depth.clone(),
                        out.count.clone())
        ref_img = img.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            step_fn()
        for rep in range(3):
            out.color.zero_()
            out.depth.zero_()
            out.count.fill_(-1)
            img.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert _same(out, ref_out), f"replay {rep}: composite differs from the eager run"
            assert torch.equal(img, ref_img), f"replay {rep}: rendering differs from the eager run"
            # eager work between replays
            V.generate(dbr, cam, tf_d, step, step, V.BISECT, 0.0, N, 10, layout=lay)
            torch.cuda.synchronize()
        assert V.device_status() == 0
        del g
    finally:
        V.set_workspace(None)


@pytest.mark.parametrize("W,H", [(480, 400), (1024, 600)], ids=["2chunks", "5chunks"])
def test_graph_capture_of_multi_chunk_general_merge(V, W, H):
    """A general merge spanning several chunks (its staging runs on a second
    stream forked from and joined back to the caller's; with 16 x 20 lists
    per pixel, 192,000 pixels take two chunks and two staging buffers,
    614,400 pixels five chunks and three buffers): captured in a graph and
    replayed, equal to the eager run and to the allocation-free path (no
    staging) bit for bit."""
    from paper_2206_14503_amd import synth
    k, n = 16, 20
    c, d, cnt = synth.dense_frame(k, n, W * H, seed=9)
    ins = [V.VDI(W, H, n, 0.01, V.REGULAR, c[r], d[r], cnt[r]) for r in range(k)]
    need = V.workspace_size(V.OP_COMPOSITE, W, H, k, in_max_n_sum=k * n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    V.set_workspace(ws)
    try:
        out = V.VDI.empty(W, H, n, 0.01, V.REGULAR)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            V.composite(ins, V.BISECT, 0.0, n, 10, out=out)
        s.synchronize()
        ref = V.VDI(W, H, n, 0.01, V.REGULAR, out.color.clone(), out.depth.clone(), out.count.clone(),
                    None, out.gamma.clone())
        alt = V.composite(ins, V.BISECT, 0.0, n, 10, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(alt.color, ref.color) and torch.equal(alt.depth, ref.depth)
        assert torch.equal(alt.count, ref.count) and torch.equal(alt.gamma, ref.gamma)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            V.composite(ins, V.BISECT, 0.0, n, 10, out=out)
        for rep in range(2):
            out.color.zero_()
            out.count.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert _same(out, ref), f"replay {rep} differs from the eager run"
        assert V.device_status() == 0
        del g
    finally:
        V.set_workspace(None)


def test_small_workspace_stages_in_small_chunks(V):
    """A caller workspace far below the recommended size: the general merge
    stages in chunks of a few hundred pixels (hundreds of chunks, and more
    deferred pixels than the deferred round's one chunk holds, so the rest go
    to the unstaged general merge); the output equals the one with the
    recommended workspace and the allocation-free path bit for bit."""
    from paper_2206_14503_amd import synth
    k, n, W, H = 16, 20, 256, 256
    c, d, cnt = synth.dense_frame(k, n, W * H, seed=21)
    ins = [V.VDI(W, H, n, 0.01, V.REGULAR, c[r], d[r], cnt[r]) for r in range(k)]
    ref = V.composite(ins, V.BISECT, 0.0, n, 10)
    alt = V.composite(ins, V.BISECT, 0.0, n, 10, noalloc=True)
    torch.cuda.synchronize()
    assert _same(alt, ref)
    need = V.workspace_size(V.OP_COMPOSITE, W, H, k, in_max_n_sum=k * n)
    # queues and block order (about 1.3 MB here) plus two chunks of 512
    # entries (320 elements of 26 bytes and 76 bytes of per-entry data each)
    small = 2 << 20
    small += 2 * 512 * (320 * 26 + 76) + 8192
    assert small < need // 4
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    V.set_workspace(ws)
    try:
        out = V.composite(ins, V.BISECT, 0.0, n, 10)
        torch.cuda.synchronize()
        assert _same(out, ref)
        assert V.device_status() == 0
    finally:
        V.set_workspace(None)


def test_many_inputs_over_chunks_equals_noalloc(V):
    """24 interleaved inputs of 20 supersegments (above the depth-disjoint
    path's input limit, so every pixel goes to the ordered general merge)
    over 204,800 pixels: three chunks in three staging buffers, deferral and
    the deferred round beside the last chunk; the output equals the
    allocation-free path's (the merge sequence in LDS, no staging) bit for
    bit."""
    from paper_2206_14503_amd import synth
    k, n, W, H = 24, 20, 512, 400
    c, d, cnt = synth.dense_frame(k, n, W * H, seed=5)
    ins = [V.VDI(W, H, n, 0.01, V.REGULAR, c[r], d[r], cnt[r]) for r in range(k)]
    a = V.composite(ins, V.BISECT, 0.0, n, 10)
    b = V.composite(ins, V.BISECT, 0.0, n, 10, noalloc=True)
    torch.cuda.synchronize()
    assert _same(a, b)
    assert torch.equal(a.gamma, b.gamma)
    assert V.device_status() == 0
