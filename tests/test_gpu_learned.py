"""GPU tests of the learned threshold: matrix-core fragment layout, MLP
forward/backward against the oracle (same bf16 operands), features against the
oracle, the learned generation's decisions, and a short training run that shows
what the regressor gains over plain bisection."""
import numpy as np
import pytest

from paper_2206_14503_amd import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="no GPU")]


@pytest.fixture(scope="module")
def V():
    import torch
    from paper_2206_14503_amd import vdi
    vdi.lib()
    torch.cuda.init()
    return vdi


@pytest.fixture(scope="module")
def OL(orc):
    import oracle.learned as learned
    return learned


def _bf16_bits(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).view(torch.int16)


def test_mfma_fragment_layout(V):
    """D = A B through one matrix-core instruction equals the exact product
    (small integers: every product and sum is exact in bf16/fp32)."""
    import torch
    rng = np.random.default_rng(0)
    A = rng.integers(-4, 5, size=(16, 16)).astype(np.float32)
    B = rng.integers(-4, 5, size=(16, 16)).astype(np.float32)
    D = V.debug_mfma(_bf16_bits(A).cuda(), _bf16_bits(B).cuda()).cpu().numpy()
    assert np.array_equal(D, A @ B)


def _random_params(OL, seed):
    p = OL.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    p["b1"] = (rng.standard_normal(128) * 0.1).astype(np.float32)
    p["b2"] = (rng.standard_normal(128) * 0.1).astype(np.float32)
    return p


@pytest.mark.parametrize("rows", [1, 64, 1000, 4099])
def test_mlp_forward_matches_oracle(V, OL, rows):
    import torch
    p = _random_params(OL, rows)
    mlp = V.MLP.from_numpy_params(p)
    rng = np.random.default_rng(rows)
    x = OL.bf16(rng.uniform(0, 1, size=(rows, 64)) * (rng.uniform(size=(rows, 64)) < 0.3))
    y_gpu = V.mlp_forward(mlp, _bf16_bits(x).cuda()).cpu().numpy()
    y_ref, _ = OL.forward(x, p, round_hidden=True)
    # fp32 vs fp64 accumulation can move a hidden activation across a bf16
    # rounding boundary; each such flip changes y by about 2^-8 * |h * w3|
    err = np.abs(y_gpu - y_ref)
    assert np.median(err) < 1e-4 and err.max() < 2e-2, (np.median(err), err.max())


def test_mlp_backward_matches_oracle(V, OL):
    import torch
    rows = 1024
    p = _random_params(OL, 7)
    mlp = V.MLP.from_numpy_params(p)
    rng = np.random.default_rng(7)
    x = OL.bf16(rng.uniform(0, 1, size=(rows, 64)) * (rng.uniform(size=(rows, 64)) < 0.3))
    t = rng.uniform(-9, 0, size=rows)
    xg = _bf16_bits(x).cuda()
    y, acts = V.mlp_forward(mlp, xg, want_acts=True)
    dy = (y - torch.from_numpy(t).float().cuda()) / rows
    g = V.mlp_backward(mlp, xg, acts, dy).cpu().numpy()
    yr, ar = OL.forward(x, p, round_hidden=True)
    gr = OL.backward(ar, dy.cpu().numpy().astype(np.float64))
    o = 0
    for k, shp in (("W1", (128, 64)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)), ("w3", (128,)), ("b3", (1,))):
        n = int(np.prod(shp))
        gk = g[o:o + n].reshape(shp)
        o += n
        bound = 1e-2 * np.abs(gr[k]).max() + 1e-4
        assert np.abs(gk - gr[k]).max() <= bound, (k, np.abs(gk - gr[k]).max(), bound)


def test_mlp_backward_is_deterministic(V, OL):
    import torch
    p = _random_params(OL, 8)
    mlp = V.MLP.from_numpy_params(p)
    x = _bf16_bits(np.random.default_rng(8).uniform(0, 1, size=(777, 64))).cuda()
    y, acts = V.mlp_forward(mlp, x, want_acts=True)
    g1 = V.mlp_backward(mlp, x, acts, y / 777)
    g2 = V.mlp_backward(mlp, x, acts, y / 777)
    assert torch.equal(g1, g2)


def test_adam_matches_oracle(V, OL):
    import torch
    p = _random_params(OL, 9)
    mlp = V.MLP.from_numpy_params(p)
    rng = np.random.default_rng(9)
    m = {k: np.zeros(v.shape) for k, v in p.items()}
    v = {k: np.zeros(v.shape) for k, v in p.items()}
    cur = p
    for step in range(1, 4):
        grads = {k: rng.standard_normal(val.shape) * 1e-2 for k, val in p.items()}
        flat = np.concatenate([grads[k].astype(np.float32).ravel() for k in ("W1", "b1", "W2", "b2", "w3", "b3")])
        V.mlp_adam(mlp, torch.from_numpy(flat).cuda(), lr=1e-3)
        cur = OL.adam(cur, {k: g.astype(np.float32).astype(np.float64) for k, g in grads.items()}, m, v, step)
    got = mlp.to_numpy_params()
    for k in cur:
        np.testing.assert_allclose(got[k], cur[k], rtol=1e-5, atol=1e-6)
    assert torch.equal(mlp.w_bf16, mlp.w_f32.to(torch.bfloat16).view(torch.int16))


def test_features_match_oracle(V, OL):
    """Histogram bins and non-transparent counts are integer decisions: exact.
    cmax agrees exactly up to the saturation at N+1 (tie-free rays)."""
    import torch
    vol = synth.gaussian_volume(64, 12, 3)
    tf = synth.transfer_function()
    cam = synth.orbit_camera(10_040, 96, 72)
    bricks = synth.brick_grid((64, 64, 64), (1, 1, 2))
    dbr = V.device_bricks(vol, bricks)
    tf_d = torch.from_numpy(tf).cuda()
    hist, nnt, cmax = V.tau_features(dbr, cam, tf_d, 1 / 64, 1 / 64, 8, 10, 2.0, 32.0)
    h_ref, n_ref, c_ref = OL.features(vol, bricks, cam, tf, 1 / 64, 1 / 64, 10, 2.0, 32.0)
    h = hist.view(torch.bfloat16).float().cpu().numpy()
    assert np.array_equal(h, h_ref)
    assert np.array_equal(nnt.cpu().numpy(), n_ref)
    g = np.full(n_ref.shape, 2.0 ** -9, np.float32)
    _, margin = OL.count_at(vol, bricks, cam, tf, 1 / 64, 1 / 64, g, 8)
    free = margin >= 2e-5
    assert np.array_equal(cmax.cpu().numpy()[free], np.minimum(c_ref, 9)[free])


def _same_lists(a, b):
    return (np.array_equal(a.count.cpu().numpy(), b.count.cpu().numpy())
            and np.array_equal(a.gamma.cpu().numpy(), b.gamma.cpu().numpy())
            and np.array_equal(a.color.cpu().numpy(), b.color.cpu().numpy())
            and np.array_equal(a.depth.cpu().numpy(), b.depth.cpu().numpy()))


def test_learned_generation_equals_bisection(V, OL):
    """With an arbitrary regressor (random weights, output shifted), the
    learned path's VDIs equal the plain bisection's bit for bit: the
    regressed threshold only orders the scans.  The tallies split the
    brick-rays by their non-transparent samples."""
    import torch
    vol = synth.gaussian_volume(64, 12, 5)
    tf = synth.transfer_function()
    cam = synth.ortho_camera(128, 128, "+z")
    bricks = synth.brick_grid((64, 64, 64), (1, 1, 2))
    dbr = V.device_bricks(vol, bricks)
    tf_d = torch.from_numpy(tf).cuda()
    p = OL.init_params(11)
    p["b3"][:] = -5.0
    mlp = V.MLP.from_numpy_params(p)
    plain = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, V.BISECT, 0.0, 8, 10)
    V.learned_stats()
    lrn = V.generate(dbr, cam, tf_d, 1 / 64, 1 / 64, V.LEARNED, 0.0, 8, 10, mlp=mlp)
    st = V.learned_stats()
    for r in range(2):
        assert _same_lists(plain[r], lrn[r]), r
    _, nnt, _ = V.tau_features(dbr, cam, tf_d, 1 / 64, 1 / 64, 8, 10, 2.0, 32.0)
    n = nnt.cpu().numpy()
    assert st["kept"] + st["refined"] == int((n > 8).sum())
    assert st["shortcut"] == int(((n > 0) & (n <= 8)).sum())
    assert st["fallback"] == 0
    assert sum(st.values()) == 2 * 128 * 128


@pytest.mark.parametrize("camera", ["ortho", "orbit"])
def test_learned_steering_with_any_threshold(V, orc, camera):
    """Caller-supplied log2 thresholds steer the scans: the plain bisection's
    own threshold (a hair below it, so every predicted decision is right),
    the same with seeded noise, and extreme values (NaN, +-inf, far outside
    the range).  Every run equals the plain bisection bit for bit, and on
    tie-free brick-rays the oracle's bisection (threshold and count).  With
    the exact threshold no served list needs a scan beyond the steered one
    unless more than five levels were left after the first scan."""
    import torch
    vol = synth.gaussian_volume(64, 12, 17)
    tf = synth.transfer_function()
    cam = synth.ortho_camera(96, 80, "-z") if camera == "ortho" else synth.orbit_camera(31, 120, 96)
    bricks = synth.brick_grid((64, 64, 64), (1, 1, 2))
    N, step = 8, 1 / 64
    plain_o = orc.generate(vol, bricks, cam, tf, step, step, 1, 0.0, N, 10)
    dbr = V.device_bricks(vol, bricks)
    tf_d = torch.from_numpy(tf).cuda()
    plain = V.generate(dbr, cam, tf_d, step, step, V.BISECT, 0.0, N, 10)
    g_star = np.stack([o.gamma.cpu().numpy() for o in plain]).astype(np.float64)
    rng = np.random.default_rng(3)
    exact = np.log2(g_star * (1.0 - 1e-4)).astype(np.float32)
    noisy = (exact + rng.normal(0.0, 0.4, exact.shape)).astype(np.float32)
    wild = rng.choice(np.float32([np.nan, np.inf, -np.inf, 40.0, -40.0, 0.0]), exact.shape).astype(np.float32)
    free = plain_o["margin"] >= 2e-5
    for name, y in (("exact", exact), ("noisy", noisy), ("wild", wild)):
        V.learned_stats()
        out = V.generate(dbr, cam, tf_d, step, step, V.LEARNED, 0.0, N, 10, y=torch.from_numpy(y).cuda())
        st = V.learned_stats()
        for r in range(len(bricks)):
            assert _same_lists(plain[r], out[r]), (name, r)
        gg = np.stack([o.gamma.cpu().numpy() for o in out])
        gc = np.stack([o.count.cpu().numpy() for o in out])
        assert np.array_equal(gg[free], plain_o["gamma"][free]), name
        assert np.array_equal(gc[free], plain_o["count"][free]), name
        if name == "exact":
            assert st["kept"] > 0
            exact_st = st
        if name == "noisy":
            assert st["kept"] + st["refined"] == exact_st["kept"] + exact_st["refined"]
            assert st["kept"] <= exact_st["kept"]


def test_learned_gain_short_training(V):
    """Train on a few small frames with the project's kernels, evaluate on a
    held-out frame of the config-4 size (1024^2, two bricks): the learned
    path gives the plain bisection's VDIs and is faster than the search as
    the paper runs it (one midpoint per pass); its speed against the
    speculative search, and the ceiling with the exact threshold, are
    reported (the bench records them)."""
    import torch
    from paper_2206_14503_amd import learned
    cfg = learned.LearnedConfig(train_res=(128, 128))
    tf_d = torch.from_numpy(synth.transfer_function()).cuda()
    X, Y, st = learned.training_pairs(cfg, seeds=range(6), tf_d=tf_d)
    assert st["kept"] > 1000
    mlp = learned.init_mlp(0)
    losses = learned.train(mlp, X, Y, epochs=6, batch=1024, lr=3e-3)
    assert losses[-1] < 0.5 * losses[0]
    ev = learned.evaluate(mlp, cfg, seeds=[100], tf_d=tf_d, reps=3)
    print("learned vs plain:", ev)
    assert ev["identical_to_plain"]
    assert ev["rgba_mae_vs_plain_render"] == 0.0
    assert ev["kept"] > 0
    assert ev["speedup_vs_seq"] > 1.0


def test_mlp_mse_gradient_and_loss(V):
    """The training step's loss kernel: dy = scale (y - log2 gamma) and the
    per-256-row loss sums of 0.5 (y - log2 gamma)^2, against fp64 numpy."""
    import torch
    rng = np.random.default_rng(21)
    rows = 1000
    y = rng.normal(-4.0, 1.5, rows).astype(np.float32)
    gam = np.exp2(rng.uniform(-9.0, 1.0, rows)).astype(np.float32)
    dy, parts = V.mlp_mse(torch.from_numpy(y).cuda(), torch.from_numpy(gam).cuda(), 1.0 / 64)
    d = y.astype(np.float64) - np.log2(gam.astype(np.float64))
    np.testing.assert_allclose(dy.cpu().numpy(), d / 64, rtol=1e-6, atol=1e-7)
    p = parts.cpu().numpy()
    assert p.shape == ((rows + 255) // 256,)
    want = [0.5 * (d[i:i + 256] ** 2).sum() for i in range(0, rows, 256)]
    np.testing.assert_allclose(p, want, rtol=1e-5)


def test_mlp_checkpoint_resume_equals_continuous(V, tmp_path):
    """Training resumed from a checkpoint (fp32 weights, Adam moments, step)
    after two epochs reaches the same parameters, bit for bit, as four epochs
    in one run."""
    import torch
    from paper_2206_14503_amd import learned
    rng = np.random.default_rng(3)
    R = 8192
    X = torch.from_numpy(rng.integers(0, 40, (R, 64)).astype(np.float32) / 32.0).cuda()
    X = X.to(torch.bfloat16).view(torch.int16).contiguous()
    Y = torch.from_numpy(np.exp2(rng.uniform(-8.0, 0.0, R)).astype(np.float32)).cuda()
    a = learned.init_mlp(5)
    la = learned.train(a, X, Y, epochs=4, batch=1024, lr=2e-3)
    b = learned.init_mlp(5)
    lb = learned.train(b, X, Y, epochs=2, batch=1024, lr=2e-3)
    path = str(tmp_path / "mlp.safetensors")
    b.save(path)
    c = V.MLP.load(path)
    lc = learned.train(c, X, Y, epochs=4, batch=1024, lr=2e-3, start_epoch=2)
    torch.cuda.synchronize()
    assert c.step == a.step == 4 * (R // 1024)
    for name in ("w_f32", "m", "v", "w_bf16"):
        assert torch.equal(getattr(a, name), getattr(c, name)), name
    assert lb + lc == la


def _interleaved_inputs(V, k, n, W, H, seed):
    cc, dd, cnt = synth.dense_interleaved_lists(k, n, W * H, seed=seed, device="cuda")
    ins = [V.VDI(W, H, n, 0.01, V.REGULAR, cc[r].contiguous(), dd[r].contiguous(), cnt[r].contiguous())
           for r in range(k)]
    return ins, cc.cpu().numpy(), dd.cpu().numpy(), cnt.cpu().numpy()


def test_composite_features_match_oracle(V, OL):
    """The compositing threshold-prediction features (64-bin histogram of
    log2 consecutive-operand distances, over N) against the oracle's, up to
    distances within 1e-4 of a bin boundary in log2 (the kernels take log2 in
    fp32 with the hardware instruction)."""
    import torch
    k, n, W, H, N = 6, 8, 40, 30, 10
    ins, c, d, m = _interleaved_inputs(V, k, n, W, H, 31)
    feat = torch.full((W * H, 64), -1, dtype=torch.int16, device="cuda")
    V.composite(ins, V.BISECT, 0.0, N, 10, features=feat)
    torch.cuda.synchronize()
    g = feat.view(torch.bfloat16).float().cpu().numpy().astype(np.float64)
    f, have, near = OL.composite_features([c[r] for r in range(k)], [d[r] for r in range(k)],
                                          [m[r] for r in range(k)], N)
    assert have.all()
    o = OL.bf16(f)
    diff = np.abs(g - o).sum(axis=1) * N
    assert np.all(diff <= 2 * near + 1e-6), (diff.max(), near[diff.argmax()])
    assert np.array_equal(g[near == 0], o[near == 0])


@pytest.mark.parametrize("seed", [0, 7])
def test_learned_composite_equals_bisection(V, orc, seed):
    """LEARNED compositing steers only the bisection's first scan: for any
    regressor (here untrained weights) the composite equals BISECT's bit for
    bit, and the oracle's."""
    import torch
    from paper_2206_14503_amd import learned
    from oracle.parity import check_lists
    k, n, W, H, N = 8, 10, 48, 40, 12
    ins, c, d, m = _interleaved_inputs(V, k, n, W, H, 40 + seed)
    mlp = learned.init_mlp(seed)
    a = V.composite(ins, V.BISECT, 0.0, N, 10)
    b = V.composite(ins, V.LEARNED, 0.0, N, 10, mlp=mlp)
    torch.cuda.synchronize()
    for name in ("color", "depth", "count", "gamma"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name
    oref = orc.composite([c[r] for r in range(k)], [d[r] for r in range(k)], [m[r] for r in range(k)], 0.01,
                         orc.BISECT, 0.0, N, 10)
    check_lists((b.color.cpu().numpy(), b.depth.cpu().numpy(), b.count.cpu().numpy(), b.gamma.cpu().numpy()),
                oref, "learned composite")


def test_learned_composite_equals_bisection_over_chunks(V):
    """The same at a size whose general merge spans five chunks in three
    staging buffers (16 x 20 lists per pixel, 1024 x 600 pixels): the MLP's
    forward pass runs per chunk on the second stream over the chunk's queue
    entries, and mispredicted lanes are deferred; the composite still equals
    BISECT's bit for bit."""
    import torch
    from paper_2206_14503_amd import learned
    k, n, W, H = 16, 20, 1024, 600
    c, d, cnt = synth.dense_frame(k, n, W * H, seed=12)
    ins = [V.VDI(W, H, n, 0.01, V.REGULAR, c[r], d[r], cnt[r]) for r in range(k)]
    mlp = learned.init_mlp(3)
    a = V.composite(ins, V.BISECT, 0.0, n, 10)
    b = V.composite(ins, V.LEARNED, 0.0, n, 10, mlp=mlp)
    torch.cuda.synchronize()
    for name in ("color", "depth", "count", "gamma"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name
    assert V.device_status() == 0
