"""Oracle for the learned threshold (an extension beyond the paper: a small
MLP predicts the threshold the per-ray bisection of Sec. 2.4 finds, and the
prediction steers the order of the bisection's scans; the result stays the
bisection's, so the generation's expected output is the oracle's BISECT).

TEST INFRASTRUCTURE (see oracle/__init__.py).

Network: 64 -> 128 -> 128 -> 1, GELU (exact erf form) after both hidden
layers, linear output y, regressed onto log2(gamma*) with mean squared error.
Weight matrices are stored (out, in): z1 = x W1^T + b1, z2 = h1 W2^T + b2.
Weights and inputs are bf16; products accumulate in fp64 here.  With
`round_hidden=True` the hidden activations are rounded to bf16 before the next
layer, where the kernels round them; with False the network is a plain fp64
function (used for the finite-difference pin of the backward pass).

Features per brick-ray (`features`): a 64-bin histogram of the sample
opacities, bin j holding the non-transparent samples with a in (j/64,
(j+1)/64], divided by s_ref and rounded to bf16; plus the number of
non-transparent samples and the count at the smallest bisection threshold.
"""
from __future__ import annotations

import ctypes
import math
from typing import Dict, Optional

import numpy as np
from scipy.special import erf

from . import _cam, _dims, _ptr, _vol, lib

SQRT1_2 = 1.0 / math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def bf16(x) -> np.ndarray:
    """Round to bf16 (nearest, ties to even) through fp32; returns float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    r = np.where(finite, r, u.astype(np.uint32))
    return r.view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z * SQRT1_2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z * SQRT1_2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def init_params(seed: int = 0) -> Dict[str, np.ndarray]:
    """fp32 master weights (He-style scale); the forward uses their bf16 copies."""
    rng = np.random.default_rng(seed)
    return {
        "W1": (rng.standard_normal((128, 64)) * math.sqrt(2.0 / 64)).astype(np.float32),
        "b1": np.zeros(128, np.float32),
        "W2": (rng.standard_normal((128, 128)) * math.sqrt(2.0 / 128)).astype(np.float32),
        "b2": np.zeros(128, np.float32),
        "w3": (rng.standard_normal(128) * math.sqrt(1.0 / 128)).astype(np.float32),
        "b3": np.full(1, -4.0, np.float32),
    }


def forward(x, params, round_hidden: bool = True, round_weights: bool = True):
    """y [R] and the saved activations.  x [R, 64] (bf16 values)."""
    q = bf16 if round_weights else (lambda a: np.asarray(a, np.float64))
    W1, W2, w3 = q(params["W1"]), q(params["W2"]), q(params["w3"])
    b1, b2, b3 = (np.asarray(params[k], np.float64) for k in ("b1", "b2", "b3"))
    x = np.asarray(x, np.float64)
    z1 = x @ W1.T + b1
    h1 = gelu(z1)
    if round_hidden:
        h1 = bf16(h1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    if round_hidden:
        h2 = bf16(h2)
    y = h2 @ w3 + b3[0]
    return y, {"x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "W1": W1, "W2": W2, "w3": w3}


def loss(y, target):
    """0.5 * mean squared error."""
    d = np.asarray(y, np.float64) - np.asarray(target, np.float64)
    return 0.5 * float(np.mean(d * d))


def backward(acts, dy) -> Dict[str, np.ndarray]:
    """Reverse mode through the network for output gradients dy [R] (fp64)."""
    dy = np.asarray(dy, np.float64)
    g = {}
    g["w3"] = acts["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(dy, acts["w3"])
    dz2 = dh2 * gelu_grad(acts["z2"])
    g["W2"] = dz2.T @ acts["h1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ acts["W2"]
    dz1 = dh1 * gelu_grad(acts["z1"])
    g["W1"] = dz1.T @ acts["x"]
    g["b1"] = dz1.sum(axis=0)
    return g


def mse_grad(y, target):
    y = np.asarray(y, np.float64)
    return (y - np.asarray(target, np.float64)) / len(y)


def adam(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on fp32 master weights (fp64 arithmetic)."""
    out = {}
    for k in params:
        m[k] = b1 * m[k] + (1 - b1) * grads[k]
        v[k] = b2 * v[k] + (1 - b2) * grads[k] ** 2
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        out[k] = (params[k].astype(np.float64) - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
    return out


def features(vol, bricks, cam, tf, step: float, ref: float, iters: int = 10, gmax: float = 2.0,
             s_ref: float = 32.0, pixels: Optional[np.ndarray] = None, nthreads: int = 0):
    """Histogram features, non-transparent counts and counts at the smallest threshold."""
    vol, dt = _vol(vol)
    n = _dims(vol)
    nb = len(bricks)
    lo = np.ascontiguousarray([b.lo for b in bricks], dtype=np.int32)
    hi = np.ascontiguousarray([b.hi for b in bricks], dtype=np.int32)
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    px = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int32)
    npix = cam.width * cam.height if px is None else len(px)
    hist = np.zeros((nb, npix, 64), np.float32)
    nnt = np.zeros((nb, npix), np.int32)
    cmax = np.zeros((nb, npix), np.int32)
    c = _cam(cam)
    L = lib()
    L.orc_features.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_float,
                               ctypes.c_float, ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_void_p,
                               ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    rc = L.orc_features(_ptr(vol), dt, _ptr(n), _ptr(lo), _ptr(hi), nb, ctypes.byref(c), _ptr(tf), tf.shape[0],
                        step, ref, iters, gmax, s_ref, _ptr(px), npix, _ptr(hist), _ptr(nnt), _ptr(cmax), nthreads)
    if rc != 0:
        raise RuntimeError("orc_features failed")
    return hist, nnt, cmax


def count_at(vol, bricks, cam, tf, step: float, ref: float, gamma: np.ndarray, limit: int,
             pixels: Optional[np.ndarray] = None, nthreads: int = 0):
    """Supersegment count of each brick-ray at the given thresholds [nb, npix] and the decision margin."""
    vol, dt = _vol(vol)
    n = _dims(vol)
    nb = len(bricks)
    lo = np.ascontiguousarray([b.lo for b in bricks], dtype=np.int32)
    hi = np.ascontiguousarray([b.hi for b in bricks], dtype=np.int32)
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    px = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int32)
    npix = cam.width * cam.height if px is None else len(px)
    g = np.ascontiguousarray(gamma, dtype=np.float32).reshape(nb, npix)
    count = np.zeros((nb, npix), np.int32)
    margin = np.zeros((nb, npix), np.float64)
    c = _cam(cam)
    L = lib()
    L.orc_count_at.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_float,
                               ctypes.c_float, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    rc = L.orc_count_at(_ptr(vol), dt, _ptr(n), _ptr(lo), _ptr(hi), nb, ctypes.byref(c), _ptr(tf), tf.shape[0],
                        step, ref, _ptr(g), limit, _ptr(px), npix, _ptr(count), _ptr(margin), nthreads)
    if rc != 0:
        raise RuntimeError("orc_count_at failed")
    return count, margin


# ---------------------------------------------------------------- compositing features
#
# Threshold prediction for the compositing bisection (an extension beyond the
# paper: Sec. 5.2 runs the per-pixel search again in compositing).  For each
# pixel whose merged list is longer than out_n: the distances between
# consecutive merged elements' per-step premultiplied colours (rgb * a, the
# Eq. 1 operands), binned by 0.5 log2 of the squared distance over [-8, 1) in
# 64 bins (below the range: bin 0; above: bin 63), counts divided by out_n.

PRED_BINS, PRED_LO, PRED_HI = 64, -8.0, 1.0


def composite_features(colors, depths, counts, out_n: int):
    """Features [npix, 64] (fp64, before bf16 rounding) and a mask of the
    pixels that have them; also the per-pixel number of distances within
    1e-4 (in log2) of a bin boundary, where an fp32 evaluation may bin the
    distance on the other side."""
    k = len(colors)
    npix = colors[0].shape[1]
    feats = np.zeros((npix, PRED_BINS))
    have = np.zeros(npix, bool)
    near = np.zeros(npix, np.int64)
    width = (PRED_HI - PRED_LO) / PRED_BINS
    for p in range(npix):
        el = []
        for r in range(k):
            for j in range(int(counts[r][p])):
                # merge key (front, input); the slot keeps each list's order
                el.append((float(depths[r][j, p, 0]), r, j))
        if len(el) <= out_n:
            continue
        el.sort()
        rep = np.array([colors[r][j, p, :3].astype(np.float64) * float(colors[r][j, p, 3]) for _, r, j in el])
        d2 = ((rep[1:] - rep[:-1]) ** 2).sum(axis=1)
        with np.errstate(divide="ignore"):
            l2 = 0.5 * np.log2(d2)
        x = (l2 - PRED_LO) / width
        b = np.where(x > 0, np.minimum(np.floor(np.where(np.isfinite(x), x, 0)), PRED_BINS - 1), 0).astype(int)
        np.add.at(feats[p], b, 1.0)
        xf = np.where(np.isfinite(x), x, -1.0)
        frac = np.abs(xf - np.round(xf)) * width
        near[p] = int(np.sum((frac < 1e-4) & (xf > 0.5) & (xf < PRED_BINS - 0.5)))
        have[p] = True
    return feats / out_n, have, near
