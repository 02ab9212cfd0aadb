"""Pins for the learned-threshold oracle: finite differences for the
backward pass, torch's own bf16 rounding, GELU and Adam as independent
references, and closed-form histogram features.  CPU only."""
import math

import numpy as np
import pytest
import torch

from paper_2206_14503_amd import synth


@pytest.fixture(scope="module")
def L(orc):
    import oracle.learned as learned
    return learned


def test_bf16_rounding_matches_torch(L):
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 20000),
                        np.float32([0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0, 3.0e38])])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(L.bf16(x), want)


def test_gelu_matches_torch_exact_form(L):
    z = np.linspace(-8, 8, 4001)
    want = torch.nn.functional.gelu(torch.from_numpy(z), approximate="none").numpy()
    np.testing.assert_allclose(L.gelu(z), want, rtol=0, atol=1e-15)
    zt = torch.from_numpy(z).requires_grad_(True)
    torch.nn.functional.gelu(zt, approximate="none").sum().backward()
    np.testing.assert_allclose(L.gelu_grad(z), zt.grad.numpy(), rtol=0, atol=1e-14)


def test_backward_matches_central_differences(L):
    """Reverse mode of the fp64 network (no rounding) against central differences, rel. err <= 1e-6."""
    rng = np.random.default_rng(1)
    p = {k: v.astype(np.float64) for k, v in L.init_params(3).items()}
    p["b1"] = rng.standard_normal(128) * 0.1
    p["b2"] = rng.standard_normal(128) * 0.1
    x = rng.uniform(0, 0.5, size=(7, 64))
    t = rng.uniform(-8, 0, size=7)

    def f(pp):
        y, _ = L.forward(x, pp, round_hidden=False, round_weights=False)
        return L.loss(y, t)

    y, acts = L.forward(x, p, round_hidden=False, round_weights=False)
    g = L.backward(acts, L.mse_grad(y, t))
    h = 1e-6
    for k, idxs in (("W1", [(0, 0), (77, 13), (127, 63)]), ("b1", [(5,), (100,)]), ("W2", [(0, 1), (127, 64)]),
                    ("b2", [(9,)]), ("w3", [(0,), (127,)]), ("b3", [(0,)])):
        for idx in idxs:
            pp, pm = {a: b.copy() for a, b in p.items()}, {a: b.copy() for a, b in p.items()}
            pp[k][idx] += h
            pm[k][idx] -= h
            fd = (f(pp) - f(pm)) / (2 * h)
            an = g[k][idx]
            assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (k, idx, fd, an)


def test_adam_matches_torch(L):
    rng = np.random.default_rng(2)
    p = L.init_params(4)
    tp = {k: torch.tensor(v.astype(np.float64), requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = {k: np.zeros_like(v, dtype=np.float64) for k, v in p.items()}
    v = {k: np.zeros_like(v, dtype=np.float64) for k, v in p.items()}
    cur = {k: val.astype(np.float64) for k, val in p.items()}
    for step in range(1, 4):
        grads = {k: rng.standard_normal(val.shape) for k, val in p.items()}
        for k in tp:
            tp[k].grad = torch.from_numpy(grads[k])
        opt.step()
        cur = L.adam(cur, grads, m, v, step)
        cur = {k: val.astype(np.float64) for k, val in cur.items()}
    for k in tp:
        np.testing.assert_allclose(cur[k], tp[k].detach().numpy(), rtol=1e-6, atol=1e-7)


def test_features_constant_volume(L, orc):
    """Constant volume: every owned sample has the same opacity, so one bin
    holds them all, nnt = owned samples, and the count at any positive
    threshold is one supersegment per brick-ray."""
    s = np.float32(0.5)
    vol = np.full((32, 32, 32), s, np.float32)
    tf = synth.transfer_function()
    cam = synth.ortho_camera(16, 16, "+z")
    bricks = synth.brick_grid((32, 32, 32), (1, 1, 2))
    hist, nnt, cmax = L.features(vol, bricks, cam, tf, 1 / 32, 1 / 32, s_ref=16.0)
    a = orc.classify(tf, s)[3]
    j = min(63, math.ceil(64 * np.float32(a)) - 1)
    assert np.all(nnt == 16)
    assert np.all(cmax == 1)
    assert np.all(hist[:, :, j] == 1.0) and hist.sum() == hist.shape[0] * hist.shape[1]


def test_features_histogram_counts(L, orc):
    """Bins sum to the non-transparent count; nnt matches the oracle's own stream."""
    vol = synth.gaussian_volume(64, 12, 0)
    tf = synth.transfer_function()
    cam = synth.ortho_camera(64, 64, "+z")
    bricks = synth.brick_grid((64, 64, 64), (1, 1, 2))
    hist, nnt, cmax = L.features(vol, bricks, cam, tf, 1 / 64, 1 / 64, s_ref=1.0)
    assert np.array_equal(hist.sum(axis=2).astype(np.int64), nnt)
    for p in (0, 1000, 2080, 4095):
        for r, b in enumerate(bricks):
            e, a32, _ = orc.stream(vol, b, cam, tf, 1 / 64, p)
            assert nnt[r, p] == int((a32 > 0).sum())
            bins = np.minimum(63, np.ceil(64 * a32[a32 > 0].astype(np.float64)).astype(int) - 1)
            assert np.array_equal(np.bincount(bins, minlength=64), hist[r, p].astype(int))


def test_composite_features_hand_example():
    """Two interleaved lists of three elements, N = 2: merged by front the
    per-step colours are 0, 0.5, 0.5, 1, 1, 1.5 (red only), so the five
    consecutive distances are 0.5, 0, 0.5, 0, 0.5: three in the bin of
    log2 0.5 = -1 (bin floor((-1 + 8) / (9 / 64)) = 49), two zeros in bin 0;
    counts divided by N.  The second pixel (empty lists) has no features, nor
    would a pixel whose merged list fits N."""
    from oracle import learned as OL
    c = [np.zeros((3, 2, 4), np.float32) for _ in range(2)]
    d = [np.zeros((3, 2, 2), np.float32) for _ in range(2)]
    for r in range(2):
        for j in range(3):
            c[r][j, 0] = [0.5 * (r + j), 0.0, 0.0, 1.0]
            d[r][j, 0] = [2 * j + r, 2 * j + r + 0.5]
    cnt = [np.array([3, 0]), np.array([3, 0])]
    f, have, near = OL.composite_features(c, d, cnt, 2)
    assert have.tolist() == [True, False]
    want = np.zeros(64)
    want[49], want[0] = 3 / 2, 2 / 2
    np.testing.assert_array_equal(f[0], want)
    assert near[0] == 0
    f6, have6, _ = OL.composite_features(c, d, cnt, 6)
    assert not have6.any()
