"""CPU oracle for VDI generation, compositing and rendering (fp64, plain C).

TEST INFRASTRUCTURE.  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import this package.  The product path
(`paper_2206_14503_amd`) never does, and this package never imports the product
path: the two share only the seeded input generators.

The arithmetic lives in `vdi_oracle.c` (see its header for the readings of the
paper it encodes); this module builds it with gcc, loads it with ctypes and
moves numpy arrays in and out.  The learned-threshold reference (histogram
features and the MLP forward/backward) lives in `oracle.learned`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vdi_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libvdi_oracle.so")
_lib = None

FIXED, BISECT = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (fp32 steps need -ffp-contract=off)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", _LIB_PATH, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


class Camera(ctypes.Structure):
    _fields_ = [("ortho", ctypes.c_int32), ("eye", ctypes.c_float * 3), ("fwd", ctypes.c_float * 3),
                ("right", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


def _cam(c) -> Camera:
    return Camera(int(c.ortho), (ctypes.c_float * 3)(*c.eye), (ctypes.c_float * 3)(*c.fwd),
                  (ctypes.c_float * 3)(*c.right), (ctypes.c_float * 3)(*c.up), int(c.width), int(c.height))


# Near-tie band of the Eq. 1 decisions: an fp32 evaluation of the distance
# may take the other branch where |d - gamma| < TIE * max(1, L / 128), L the
# open supersegment's element count (see vdi_oracle.c).  Lists whose decisions
# meet such near ties carry every outcome the near ties admit.
TIE = 2e-5


class Alts(ctypes.Structure):
    _fields_ = [("ray", ctypes.c_void_p), ("count", ctypes.c_void_p), ("gamma", ctypes.c_void_p),
                ("color", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("cap", ctypes.c_int32),
                ("n", ctypes.c_int32)]


def _alloc_alts(cap: int, max_n: int):
    cap = max(int(cap), 1)
    a = {"ray": np.zeros(cap, np.int32), "count": np.zeros(cap, np.int32), "gamma": np.zeros(cap, np.float32),
         "color": np.zeros((cap, max_n, 4), np.float32), "depth": np.zeros((cap, max_n, 2), np.float32)}
    st = Alts(a["ray"].ctypes.data, a["count"].ctypes.data, a["gamma"].ctypes.data, a["color"].ctypes.data,
              a["depth"].ctypes.data, cap, 0)
    return a, st


def _with_alts(call, rays: int, max_n: int):
    """Run call(alts_struct) with a buffer for alternative outcomes, growing
    it when the oracle reports it too small (-3); returns (rc, alts) with the
    alternatives trimmed to those written."""
    cap = max(64, rays // 16)
    while True:
        a, st = _alloc_alts(cap, max_n)
        rc = call(ctypes.byref(st))
        if rc == -3:
            cap = int(st.n) + 16
            continue
        n = min(int(st.n), cap)
        return rc, {k: v[:n] for k, v in a.items()}


def lib():
    global _lib
    if _lib is None:
        # VDI_ORACLE_LIBRARY: another build of the same source (the
        # sanitizer test loads an AddressSanitizer/UBSan build this way)
        path = os.environ.get("VDI_ORACLE_LIBRARY")
        if not path:
            path = _LIB_PATH
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
                build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, f32, f64 = ctypes.c_int32, ctypes.c_float, ctypes.c_double
        L.orc_generate.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_int, ctypes.POINTER(Camera), P, ctypes.c_int,
                                   f32, f32, ctypes.c_int, f32, ctypes.c_int, ctypes.c_int, P, ctypes.c_int,
                                   P, P, P, P, P, P, P, P, f64, P, P, ctypes.c_int]
        L.orc_composite.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int, ctypes.c_int, f32, ctypes.c_int, f32,
                                    ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, f64, P, P, ctypes.c_int]
        L.orc_render_ov.argtypes = [P, P, P, ctypes.c_int, ctypes.c_int, f32, P, ctypes.c_int]
        L.orc_dvr.argtypes = [P, ctypes.c_int, P, ctypes.POINTER(Camera), P, ctypes.c_int, f32, f32, P,
                              ctypes.c_int, P, ctypes.c_int]
        L.orc_seg.argtypes = [P, ctypes.c_int, ctypes.c_int, f64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_int, f64, P, ctypes.c_int, P, P]
        L.orc_seg_outcomes.argtypes = [P, ctypes.c_int, ctypes.c_int, f64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       f64, f64, P, P, P, ctypes.c_int]
        L.orc_seg_outcomes.restype = ctypes.c_int
        L.orc_ray_info.argtypes = [ctypes.POINTER(Camera), ctypes.c_int, f32, P, P, P, P]
        L.orc_stream.argtypes = [P, ctypes.c_int, P, P, P, ctypes.POINTER(Camera), P, ctypes.c_int, f32,
                                 ctypes.c_int, P, ctypes.c_int, P]
        L.orc_novel_view.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, f32,
                                     ctypes.POINTER(Camera), ctypes.POINTER(Camera), f32, P, ctypes.c_int]
        L.orc_trilinear.argtypes = [P, ctypes.c_int, P, P]
        L.orc_trilinear.restype = f64
        L.orc_classify.argtypes = [P, ctypes.c_int, f32, P]
        L.orc_classify.restype = None
        for name in ("orc_generate", "orc_composite", "orc_render_ov", "orc_novel_view", "orc_dvr", "orc_seg",
                     "orc_ray_info", "orc_stream"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _vol(vol: np.ndarray):
    vol = np.ascontiguousarray(vol)
    if vol.dtype == np.float16:
        return vol, 1
    if vol.dtype != np.float32:
        raise TypeError("volume must be float32 or float16")
    return vol, 0


def _dims(vol: np.ndarray) -> np.ndarray:
    nz, ny, nx = vol.shape
    return np.array([nx, ny, nz], dtype=np.int32)


def generate(vol: np.ndarray, bricks: Sequence, cam, tf: np.ndarray, step: float, ref: float,
             mode: int, tau: float, max_n: int, iters: int = 10,
             pixels: Optional[np.ndarray] = None, nthreads: int = 0, owner: Optional[np.ndarray] = None,
             ranks: Optional[Sequence[int]] = None, tie: float = TIE) -> Dict[str, np.ndarray]:
    """Generate one regular sub-VDI per brick over `pixels` (default: all).
    owner: optional rank per voxel ([nz, ny, nx] uint8, like the volume) with
    ranks[r] brick r's rank: brick r owns the samples whose voxel lies in its
    box and carries its rank (non-convex domains; bisection modes only).
    Besides the fp64 outcome, "nout" [nb, npix] holds each list's number of
    outcomes under near ties (negative: not all enumerated) and "alts" the
    others (ray = r * npix + q)."""
    vol, dt = _vol(vol)
    n = _dims(vol)
    nb = len(bricks)
    lo = np.ascontiguousarray([b.lo for b in bricks], dtype=np.int32)
    hi = np.ascontiguousarray([b.hi for b in bricks], dtype=np.int32)
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    if pixels is None:
        npix = cam.width * cam.height
        px = None
    else:
        px = np.ascontiguousarray(pixels, dtype=np.int32)
        npix = len(px)
    out = {
        "color": np.zeros((nb, max_n, npix, 4), np.float32),
        "depth": np.zeros((nb, max_n, npix, 2), np.float32),
        "count": np.zeros((nb, npix), np.int32),
        "gamma": np.zeros((nb, npix), np.float32),
        "margin": np.zeros((nb, npix), np.float64),
        "contiguous": np.zeros((nb, npix), np.int32),
        "nout": np.zeros((nb, npix), np.int32),
    }
    own = None if owner is None else np.ascontiguousarray(owner, dtype=np.uint8)
    rk = None if ranks is None else np.ascontiguousarray(ranks, dtype=np.int32)
    if own is not None:
        assert own.shape == vol.shape and rk is not None and len(rk) == nb
    c = _cam(cam)
    call = lambda alts: lib().orc_generate(
        _ptr(vol), dt, _ptr(n), _ptr(lo), _ptr(hi), nb, ctypes.byref(c), _ptr(tf), tf.shape[0], step, ref, mode,
        tau, max_n, iters, _ptr(px), npix, _ptr(out["color"]), _ptr(out["depth"]), _ptr(out["count"]),
        _ptr(out["gamma"]), _ptr(out["margin"]), _ptr(out["contiguous"]), _ptr(own), _ptr(rk), tie,
        _ptr(out["nout"]), alts, nthreads)
    rc, out["alts"] = _with_alts(call, nb * npix, max_n)
    if rc != 0:
        raise RuntimeError(f"orc_generate failed ({rc})")
    return out


def composite(colors: Sequence[np.ndarray], depths: Sequence[np.ndarray], counts: Sequence[np.ndarray],
              ref: float, mode: int, tau: float, out_n: int, iters: int = 10,
              want_order: bool = False, nthreads: int = 0, tie: float = TIE) -> Dict[str, np.ndarray]:
    """Composite k regular lists ([in_n, npix, 4], [in_n, npix, 2], [npix]) into one.
    "nout" and "alts" as for generate (ray = pixel)."""
    k = len(colors)
    in_n, npix = colors[0].shape[0], colors[0].shape[1]
    cs = [np.ascontiguousarray(c, dtype=np.float32) for c in colors]
    ds = [np.ascontiguousarray(d, dtype=np.float32) for d in depths]
    ns = [np.ascontiguousarray(c, dtype=np.int32) for c in counts]
    for c, d, m in zip(cs, ds, ns):
        assert c.shape == (in_n, npix, 4) and d.shape == (in_n, npix, 2) and m.shape == (npix,)
    arr = lambda xs: (ctypes.c_void_p * k)(*[x.ctypes.data for x in xs])
    out = {
        "color": np.zeros((out_n, npix, 4), np.float32),
        "depth": np.zeros((out_n, npix, 2), np.float32),
        "count": np.zeros((npix,), np.int32),
        "gamma": np.zeros((npix,), np.float32),
        "margin": np.zeros((npix,), np.float64),
        "nout": np.zeros((npix,), np.int32),
    }
    order = np.zeros((npix, k * in_n), np.int32) if want_order else None
    call = lambda alts: lib().orc_composite(
        k, arr(cs), arr(ds), arr(ns), in_n, npix, ref, mode, tau, out_n, iters, _ptr(out["color"]),
        _ptr(out["depth"]), _ptr(out["count"]), _ptr(out["gamma"]), _ptr(out["margin"]), _ptr(order), tie,
        _ptr(out["nout"]), alts, nthreads)
    rc, out["alts"] = _with_alts(call, npix, out_n)
    if rc == -2:
        raise ValueError("composite input is not a valid depth-sorted supersegment list")
    if rc != 0:
        raise RuntimeError(f"orc_composite failed ({rc})")
    if want_order:
        out["order"] = order
    return out


def render_ov(color: np.ndarray, depth: np.ndarray, count: np.ndarray, ref: float,
              nthreads: int = 0) -> np.ndarray:
    """Premultiplied RGBA [npix, 4] (fp64) of a regular VDI seen from its own viewpoint."""
    max_n, npix = color.shape[0], color.shape[1]
    color = np.ascontiguousarray(color, dtype=np.float32)
    depth = np.ascontiguousarray(depth, dtype=np.float32)
    count = np.ascontiguousarray(count, dtype=np.int32)
    rgba = np.zeros((npix, 4), np.float64)
    rc = lib().orc_render_ov(_ptr(color), _ptr(depth), _ptr(count), max_n, npix, ref, _ptr(rgba), nthreads)
    if rc != 0:
        raise RuntimeError("orc_render_ov failed")
    return rgba


def novel_view(color: np.ndarray, depth: np.ndarray, count: np.ndarray, ref: float, vdi_cam, view, step: float,
               offset: Optional[np.ndarray] = None, nthreads: int = 0) -> np.ndarray:
    """Premultiplied RGBA [view pixels, 4] (fp64) of a VDI rendered from camera
    `view` (the VDI as a piecewise-constant field over its camera's pixel
    frusta, sampled on each new ray's grid).  Regular layout: color [N, P, 4],
    depth [N, P, 2]; compact (offset given): color [M, 4], depth [M, 2], pixel
    q's list at offset[q]."""
    color = np.ascontiguousarray(color, dtype=np.float32)
    depth = np.ascontiguousarray(depth, dtype=np.float32)
    count = np.ascontiguousarray(count, dtype=np.int32)
    if offset is None:
        max_n = color.shape[0]
        off = None
    else:
        max_n = max(int(count.max()) if count.size else 1, 1)
        off = np.ascontiguousarray(offset, dtype=np.uint32)
    rgba = np.zeros((view.width * view.height, 4), np.float64)
    vc, nv = _cam(vdi_cam), _cam(view)
    rc = lib().orc_novel_view(_ptr(color), _ptr(depth), _ptr(count), _ptr(off), max_n, vdi_cam.width,
                              vdi_cam.height, ref, ctypes.byref(vc), ctypes.byref(nv), step, _ptr(rgba), nthreads)
    if rc != 0:
        raise RuntimeError("orc_novel_view failed")
    return rgba


def dvr(vol: np.ndarray, cam, tf: np.ndarray, step: float, ref: float,
        pixels: Optional[np.ndarray] = None, nthreads: int = 0) -> np.ndarray:
    """Emission-absorption raycast of the whole volume; premultiplied RGBA [npix, 4] (fp64)."""
    vol, dt = _vol(vol)
    n = _dims(vol)
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    px = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int32)
    npix = cam.width * cam.height if px is None else len(px)
    rgba = np.zeros((npix, 4), np.float64)
    c = _cam(cam)
    rc = lib().orc_dvr(_ptr(vol), dt, _ptr(n), ctypes.byref(c), _ptr(tf), tf.shape[0], step, ref, _ptr(px),
                       npix, _ptr(rgba), nthreads)
    if rc != 0:
        raise RuntimeError("orc_dvr failed")
    return rgba


def seg(elems: np.ndarray, mode: int, gamma: float = 0.0, cap: int = 0, max_n: int = 0, iters: int = 10,
        gaps: bool = False, ref: float = 1.0, max_out: Optional[int] = None):
    """Segment explicit elements [n, 6] = (f, b, r, g, b, a).

    Returns (supersegments [c, 6], count, gamma_used, margin)."""
    elems = np.ascontiguousarray(elems, dtype=np.float64).reshape(-1, 6)
    n = elems.shape[0]
    max_out = max_out if max_out is not None else max(n, 1)
    out = np.zeros((max_out, 6), np.float64)
    g = np.zeros(1, np.float64)
    m = np.zeros(1, np.float64)
    c = lib().orc_seg(_ptr(elems), n, mode, gamma, cap, max_n, iters, int(gaps), ref, _ptr(out), max_out,
                      _ptr(g), _ptr(m))
    return out[:min(c, max_out)], c, float(g[0]), float(m[0])


def seg_outcomes(elems: np.ndarray, mode: int, gamma: float = 0.0, max_n: int = 8, iters: int = 10,
                 gaps: bool = False, ref: float = 1.0, tie: float = TIE, max_outcomes: int = 256):
    """Every outcome of segmenting explicit elements [n, 6] when each near-tie
    Eq. 1 decision may go either way: a list of (count, gamma, supersegments
    [min(count, max_n), 6]), the fp64 outcome first, and whether the
    enumeration was complete."""
    elems = np.ascontiguousarray(elems, dtype=np.float64).reshape(-1, 6)
    counts = np.zeros(max_outcomes, np.int32)
    gammas = np.zeros(max_outcomes, np.float64)
    lists = np.zeros((max_outcomes, max_n, 6), np.float64)
    no = lib().orc_seg_outcomes(_ptr(elems), elems.shape[0], mode, gamma, max_n, iters, int(gaps), ref, tie,
                                _ptr(counts), _ptr(gammas), _ptr(lists), max_outcomes)
    tot = min(abs(no), max_outcomes)
    return [(int(counts[i]), float(gammas[i]), lists[i, :min(int(counts[i]), max_n)]) for i in range(tot)], no > 0


def ray_info(cam, pix: int, step: float):
    o = np.zeros(3, np.float32)
    d = np.zeros(3, np.float32)
    tn = np.zeros(1, np.float32)
    tf = np.zeros(1, np.float32)
    c = _cam(cam)
    ns = lib().orc_ray_info(ctypes.byref(c), pix, step, _ptr(o), _ptr(d), _ptr(tn), _ptr(tf))
    return dict(o=o, d=d, tn=float(tn[0]), tf=float(tf[0]), samples=ns)


def stream(vol: np.ndarray, brick, cam, tf: np.ndarray, step: float, pix: int):
    """Owned element stream (f, b, r, g, b, a) of one brick along one pixel's ray."""
    vol, dt = _vol(vol)
    n = _dims(vol)
    cap = int(1.7320509 / step) + 4
    e = np.zeros((cap, 6), np.float64)
    a32 = np.zeros(cap, np.float32)
    lo = np.array(brick.lo, np.int32)
    hi = np.array(brick.hi, np.int32)
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    c = _cam(cam)
    ne = lib().orc_stream(_ptr(vol), dt, _ptr(n), _ptr(lo), _ptr(hi), ctypes.byref(c), _ptr(tf), tf.shape[0],
                          step, pix, _ptr(e), cap, _ptr(a32))
    contiguous = ne >= 0
    ne = ne if ne >= 0 else -ne - 1
    return e[:ne], a32[:ne], contiguous


def trilinear(vol: np.ndarray, p) -> float:
    vol, dt = _vol(vol)
    n = _dims(vol)
    pp = np.asarray(p, dtype=np.float32)
    return lib().orc_trilinear(_ptr(vol), dt, _ptr(n), _ptr(pp))


def classify(tf: np.ndarray, s: float) -> np.ndarray:
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    out = np.zeros(4, np.float64)
    lib().orc_classify(_ptr(tf), tf.shape[0], s, _ptr(out))
    return out


def to_compact(color: np.ndarray, depth: np.ndarray, count: np.ndarray):
    """Regular [N, P, *] layout -> compact: offset = exclusive prefix sum of the
    counts (Sec. 4), supersegments of list p stored at offset[p] + j."""
    max_n, npix = color.shape[0], color.shape[1]
    offset = np.zeros(npix + 1, np.uint64)
    offset[1:] = np.cumsum(count.astype(np.uint64))
    total = int(offset[-1])
    cc = np.zeros((total, 4), np.float32)
    dd = np.zeros((total, 2), np.float32)
    for p in np.nonzero(count)[0]:
        o = int(offset[p])
        cc[o:o + count[p]] = color[:count[p], p]
        dd[o:o + count[p]] = depth[:count[p], p]
    return offset.astype(np.uint32), cc, dd


def from_compact(offset: np.ndarray, color: np.ndarray, depth: np.ndarray, max_n: int):
    npix = len(offset) - 1
    count = (offset[1:].astype(np.int64) - offset[:-1].astype(np.int64)).astype(np.int32)
    rc = np.zeros((max_n, npix, 4), np.float32)
    rd = np.zeros((max_n, npix, 2), np.float32)
    for p in np.nonzero(count)[0]:
        o = int(offset[p])
        rc[:count[p], p] = color[o:o + count[p]]
        rd[:count[p], p] = depth[o:o + count[p]]
    return rc, rd, count
