"""Pins for the oracle's novel-view rendering of a VDI.

The VDI is read as the piecewise-constant field it encodes (each
supersegment fills its pixel's view frustum between its front and back
depths); a ray of the new view is sampled on the generation grid.  Checked
against: the original-view rendering (exact when the new view is the VDI's own
camera, since every sample then lies inside the supersegments it was made
of), closed forms for a constant slab seen from the side and a constant shell
seen from the VDI's eye, the empty VDI, and the compact layout.
"""
import math

import numpy as np
import pytest

from paper_2206_14503_amd import synth


def _one_segment_vdi(npix, f0, b0, rgb, a):
    color = np.zeros((1, npix, 4), np.float32)
    color[0, :, :3] = rgb
    color[0, :, 3] = a
    depth = np.zeros((1, npix, 2), np.float32)
    depth[0, :, 0] = f0
    depth[0, :, 1] = b0
    return color, depth, np.ones(npix, np.int32)


def _tiny_vdi(orc, cam, n=24, seed=3):
    vol = synth.gaussian_volume(n, 6, seed)
    tf = synth.transfer_function()
    bricks = synth.brick_grid((n, n, n), (1, 1, 2))
    step = 1.0 / n
    g = orc.generate(vol, bricks, cam, tf, step, step, 1, 0.0, 8, 10)
    c = orc.composite([g["color"][r] for r in range(2)], [g["depth"][r] for r in range(2)],
                      [g["count"][r] for r in range(2)], step, 1, 0.0, 8, 10)
    return c, step


@pytest.mark.parametrize("cam", [synth.orbit_camera(10_031, 40, 30), synth.ortho_camera(32, 32, "+z")],
                         ids=["persp", "ortho"])
def test_novel_view_from_the_vdi_camera_is_the_original_view(orc, cam):
    """Seen from its own camera on its own sample grid, every sample lies inside
    the supersegment it was accumulated into, so the point-sampled integral of
    each supersegment is its total opacity: novel view == original view, up to
    the fp32 rounding of the stored depths (the original view takes each
    length from them, the novel view counts samples)."""
    c, step = _tiny_vdi(orc, cam)
    ov = orc.render_ov(c["color"], c["depth"], c["count"], step)
    nv = orc.novel_view(c["color"], c["depth"], c["count"], step, cam, cam, step)
    assert (c["count"] > 1).sum() > 50
    assert np.abs(nv - ov).max() <= 2e-6


def test_novel_view_ortho_slab_from_the_side(orc):
    """A +z orthographic VDI whose every list is one supersegment [0.3, 0.7) is a
    constant slab; an orthographic view along +x sees, on rows with z in the
    slab, all of its ray's samples at opacity 1-(1-a)^(step/ref) each."""
    vcam = synth.ortho_camera(32, 32, "+z")
    color, depth, count = _one_segment_vdi(32 * 32, 0.3, 0.7, (0.2, 0.5, 0.9), 0.1)
    W, H = 40, 24
    view = synth.Camera(1, (0.0, 0.5, 0.5), (1.0, 0.0, 0.0), (0.0, 0.0, 0.5), (0.0, 0.5, 0.0), W, H).as_f32()
    step = 1.0 / 64
    nv = orc.novel_view(color, depth, count, step, vcam, view, step).reshape(H, W, 4)
    for i in range(W):
        z = (2 * i + 1) / (2 * W)
        for j in range(H):
            ns = orc.ray_info(view, j * W + i, step)["samples"]
            alpha = 1.0 - (1.0 - float(np.float32(0.1))) ** ns if 0.3 <= z < 0.7 else 0.0
            assert nv[j, i, 3] == pytest.approx(alpha, abs=1e-12)
            assert np.allclose(nv[j, i, :3], np.array([0.2, 0.5, 0.9], np.float32).astype(np.float64) * alpha,
                               atol=1e-12)


def test_novel_view_perspective_shell_from_the_vdi_eye(orc):
    """A perspective VDI whose every list is one supersegment [1.3, 1.9) is a
    shell of radii 1.3 and 1.9 about its eye.  A narrower view from the same
    eye, turned by 5 degrees, stays inside the VDI's frustum, so a ray's
    samples inside the shell are those with 1.3 <= t_k < 1.9."""
    eye = (0.5, 0.5, -1.0)
    vcam = synth.perspective_camera(eye, (0.5, 0.5, 0.5), 32, 32, 60.0)
    color, depth, count = _one_segment_vdi(32 * 32, 1.3, 1.9, (0.7, 0.3, 0.1), 0.05)
    turn = math.radians(5.0)
    target = (0.5 + 1.5 * math.sin(turn), 0.5, -1.0 + 1.5 * math.cos(turn))
    view = synth.perspective_camera(eye, target, 24, 20, 30.0)
    step = 1.0 / 48
    nv = orc.novel_view(color, depth, count, step, vcam, view, step)
    checked = 0
    for pix in range(24 * 20):
        info = orc.ray_info(view, pix, step)
        if info["samples"] <= 0:
            assert np.all(nv[pix] == 0)
            continue
        t = info["tn"] + (np.arange(info["samples"]) + 0.5) * step
        if np.min(np.abs(t - 1.3)) < 1e-5 or np.min(np.abs(t - 1.9)) < 1e-5:
            continue
        n_in = int(((t >= 1.3) & (t < 1.9)).sum())
        alpha = 1.0 - (1.0 - float(np.float32(0.05))) ** n_in
        assert nv[pix, 3] == pytest.approx(alpha, abs=1e-12), pix
        assert np.allclose(nv[pix, :3], np.array([0.7, 0.3, 0.1], np.float32).astype(np.float64) * alpha, atol=1e-12)
        checked += 1
    assert checked > 300


def test_novel_view_of_an_empty_vdi_is_empty(orc):
    cam = synth.orbit_camera(10_032, 16, 12)
    color = np.zeros((4, 16 * 12, 4), np.float32)
    depth = np.zeros((4, 16 * 12, 2), np.float32)
    count = np.zeros(16 * 12, np.int32)
    view = synth.orbit_camera(10_033, 20, 10)
    nv = orc.novel_view(color, depth, count, 1 / 32, cam, view, 1 / 32)
    assert np.all(nv == 0)


def test_novel_view_compact_equals_regular(orc):
    """The same lists in the compact layout give the same image, bit for bit."""
    cam = synth.orbit_camera(10_034, 36, 28)
    c, step = _tiny_vdi(orc, cam)
    cnt = c["count"]
    off = np.concatenate([[0], np.cumsum(cnt)[:-1]]).astype(np.uint32)
    m = int(cnt.sum())
    cc = np.zeros((m, 4), np.float32)
    dd = np.zeros((m, 2), np.float32)
    for q in range(cnt.size):
        cc[off[q]:off[q] + cnt[q]] = c["color"][:cnt[q], q]
        dd[off[q]:off[q] + cnt[q]] = c["depth"][:cnt[q], q]
    view = synth.orbit_camera(10_035, 30, 22)
    a = orc.novel_view(c["color"], c["depth"], cnt, step, cam, view, step)
    b = orc.novel_view(cc, dd, cnt, step, cam, view, step, offset=off)
    assert (a[:, 3] > 0).sum() > 50
    assert np.array_equal(a, b)
