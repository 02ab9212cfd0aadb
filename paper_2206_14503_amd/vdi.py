"""ctypes binding of libvdi (include/vdi.h).

Argument marshalling only: every step of generation, compositing and
rendering runs in the HIP kernels of libvdi.so.  torch tensors supply device
memory and the current HIP stream.  If libvdi.so is missing the calls raise;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvdi.so")

REGULAR, COMPACT = 0, 1
FIXED, BISECT, LEARNED, BISECT_SEQ = 0, 1, 2, 3
F32, F16 = 0, 1

_STATUS = {0: "VDI_OK", -1: "VDI_E_INVALID", -2: "VDI_E_UNSUPPORTED", -3: "VDI_E_HIP", -4: "VDI_E_INPUT",
           -5: "VDI_E_CAPACITY", -6: "VDI_E_WORKSPACE"}


class VdiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


# ---------------------------------------------------------------- C structs (mirror include/vdi.h)

class vdi_t(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("max_n", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("ref_step", ctypes.c_float), ("color", ctypes.c_void_p),
                ("depth", ctypes.c_void_p), ("count", ctypes.c_void_p), ("offset", ctypes.c_void_p),
                ("gamma", ctypes.c_void_p), ("capacity", ctypes.c_uint64)]


class vdi_brick_t(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("full_dim", ctypes.c_int32 * 3),
                ("lo", ctypes.c_int32 * 3), ("hi", ctypes.c_int32 * 3), ("data_lo", ctypes.c_int32 * 3),
                ("data_dim", ctypes.c_int32 * 3), ("owner", ctypes.c_void_p), ("rank", ctypes.c_int32)]


class vdi_camera_t(ctypes.Structure):
    _fields_ = [("ortho", ctypes.c_int32), ("eye", ctypes.c_float * 3), ("fwd", ctypes.c_float * 3),
                ("right", ctypes.c_float * 3), ("up", ctypes.c_float * 3), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32)]


class vdi_tf_t(ctypes.Structure):
    _fields_ = [("rgba", ctypes.c_void_p), ("entries", ctypes.c_int32)]


class vdi_tau_t(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tau", ctypes.c_float), ("iters", ctypes.c_int32),
                ("gamma_max", ctypes.c_float), ("mlp", ctypes.c_void_p), ("fallback_tol", ctypes.c_float),
                ("feature_scale", ctypes.c_float), ("y", ctypes.c_void_p), ("features", ctypes.c_void_p)]


class vdi_shape_t(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("k", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("tau_mode", ctypes.c_int32), ("in_max_n_sum", ctypes.c_int32),
                ("rows", ctypes.c_int32)]


OP_GENERATE, OP_COMPOSITE, OP_MLP_BACKWARD = 0, 1, 2


class vdi_mlp_t(ctypes.Structure):
    _fields_ = [("w_bf16", ctypes.c_void_p), ("w_f32", ctypes.c_void_p)]


MLP_PARAMS = 24961
MLP_ACT_FLOATS = 384


_lib = None


def lib():
    """Load libvdi.so (raises if it has not been built).  VDI_LIBRARY names
    another build of the same sources (the sanitizer test loads a build
    with host-side AddressSanitizer/UBSan this way)."""
    global _lib
    if _lib is None:
        path = os.environ.get("VDI_LIBRARY") or LIB_PATH
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_2206_14503_amd.build`")
        L = ctypes.CDLL(path)
        P, I = ctypes.c_void_p, ctypes.c_int
        L.vdi_last_error.restype = ctypes.c_char_p
        L.vdi_ctx_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), I]
        L.vdi_ctx_destroy.argtypes = [P]
        L.vdi_ctx_device_status.argtypes = [P, ctypes.POINTER(ctypes.c_int32), P]
        L.vdi_generate.argtypes = [P, ctypes.POINTER(vdi_brick_t), I, ctypes.POINTER(vdi_camera_t),
                                   ctypes.POINTER(vdi_tf_t), ctypes.c_float, ctypes.POINTER(vdi_tau_t),
                                   ctypes.POINTER(vdi_t), P]
        L.vdi_composite.argtypes = [P, ctypes.POINTER(vdi_t), I, ctypes.POINTER(vdi_tau_t), ctypes.POINTER(vdi_t), P]
        L.vdi_composite_noalloc.argtypes = [P, ctypes.POINTER(vdi_t), I, ctypes.POINTER(vdi_tau_t),
                                            ctypes.POINTER(vdi_t), P]
        L.vdi_composite_noalloc.restype = ctypes.c_int
        L.vdi_render_original_view.argtypes = [P, ctypes.POINTER(vdi_t), P, P]
        L.vdi_render_novel_view.argtypes = [P, ctypes.POINTER(vdi_t), ctypes.POINTER(vdi_camera_t),
                                            ctypes.POINTER(vdi_camera_t), ctypes.c_float, P, P]
        L.vdi_debug_rays.argtypes = [P, ctypes.POINTER(vdi_camera_t), ctypes.c_float, P, P, P, P, P, P]
        L.vdi_tau_features.argtypes = [P, ctypes.POINTER(vdi_brick_t), I, ctypes.POINTER(vdi_camera_t),
                                       ctypes.POINTER(vdi_tf_t), ctypes.c_float, ctypes.c_float, I,
                                       ctypes.POINTER(vdi_tau_t), P, P, P, P]
        L.vdi_mlp_forward.argtypes = [P, ctypes.POINTER(vdi_mlp_t), P, I, P, P, P]
        L.vdi_mlp_backward.argtypes = [P, ctypes.POINTER(vdi_mlp_t), P, P, P, I, P, P]
        L.vdi_mlp_adam.argtypes = [P, ctypes.POINTER(vdi_mlp_t), P, P, P, I, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, P]
        L.vdi_learned_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64), P]
        L.vdi_debug_mfma.argtypes = [P, P, P, P, P]
        L.vdi_mlp_mse.argtypes = [P, P, P, I, ctypes.c_float, P, P, P]
        L.vdi_mlp_pack.argtypes = [P, ctypes.POINTER(vdi_mlp_t), P]
        for name in ("vdi_mlp_mse", "vdi_mlp_pack"):
            getattr(L, name).restype = ctypes.c_int
        L.vdi_workspace_size.argtypes = [P, ctypes.POINTER(vdi_shape_t), ctypes.POINTER(ctypes.c_size_t)]
        L.vdi_ctx_set_workspace.argtypes = [P, P, ctypes.c_size_t]
        L.vdi_ctx_reserve_workspace.argtypes = [P, ctypes.c_size_t]
        for name in ("vdi_workspace_size", "vdi_ctx_set_workspace", "vdi_ctx_reserve_workspace"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("vdi_ctx_create", "vdi_ctx_destroy", "vdi_ctx_device_status", "vdi_generate", "vdi_composite",
                     "vdi_render_original_view", "vdi_render_novel_view", "vdi_debug_rays", "vdi_tau_features",
                     "vdi_mlp_forward", "vdi_mlp_backward", "vdi_mlp_adam", "vdi_learned_stats", "vdi_debug_mfma"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise VdiError(rc, lib().vdi_last_error().decode())


_ctx = {}


def context(device: Optional[int] = None) -> ctypes.c_void_p:
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _ctx:
        h = ctypes.c_void_p()
        _check(lib().vdi_ctx_create(ctypes.byref(h), dev))
        _ctx[dev] = h
    return _ctx[dev]


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous"
    return ctypes.c_void_p(t.data_ptr())


def workspace_size(op: int, width: int = 0, height: int = 0, k: int = 0, layout: int = REGULAR,
                   tau_mode: int = BISECT, in_max_n_sum: int = 0, rows: int = 0) -> int:
    """Bytes of device scratch memory the op needs at this shape (vdi_workspace_size)."""
    sh = vdi_shape_t(op, width, height, k, layout, tau_mode, in_max_n_sum, rows)
    n = ctypes.c_size_t()
    _check(lib().vdi_workspace_size(context(), ctypes.byref(sh), ctypes.byref(n)))
    return int(n.value)


_workspace = {}


def set_workspace(ws: Optional[torch.Tensor]):
    """Make `ws` (a device uint8 tensor, kept referenced here) the workspace of
    every later op on this device's context; None returns to the context's own."""
    dev = torch.cuda.current_device()
    if ws is None:
        _check(lib().vdi_ctx_set_workspace(context(), None, 0))
        _workspace.pop(dev, None)
        return
    assert ws.is_cuda and ws.is_contiguous() and ws.dtype == torch.uint8
    _check(lib().vdi_ctx_set_workspace(context(), _ptr(ws), ws.numel()))
    _workspace[dev] = ws


def reserve_workspace(nbytes: int):
    """Grow the context's own workspace to nbytes now (vdi_ctx_reserve_workspace)."""
    _check(lib().vdi_ctx_reserve_workspace(context(), int(nbytes)))


# ---------------------------------------------------------------- Python-side VDI

@dataclasses.dataclass
class VDI:
    """A VDI held in torch tensors.

    regular: color [max_n, H*W, 4], depth [max_n, H*W, 2]
    compact: color [capacity, 4], depth [capacity, 2], offset [H*W+1] (int32 storage of uint32)
    count [H*W] int32, gamma [H*W] float32 or None."""
    width: int
    height: int
    max_n: int
    ref_step: float
    layout: int
    color: torch.Tensor
    depth: torch.Tensor
    count: torch.Tensor
    offset: Optional[torch.Tensor] = None
    gamma: Optional[torch.Tensor] = None

    @property
    def npix(self) -> int:
        return self.width * self.height

    def c(self) -> vdi_t:
        cap = self.color.shape[0] if self.layout == COMPACT else 0
        return vdi_t(self.width, self.height, self.max_n, self.layout, self.ref_step, _ptr(self.color),
                     _ptr(self.depth), _ptr(self.count), _ptr(self.offset), _ptr(self.gamma), cap)

    @staticmethod
    def empty(width: int, height: int, max_n: int, ref_step: float, layout: int = REGULAR,
              capacity: Optional[int] = None, device=None, with_gamma: bool = True) -> "VDI":
        dev = device or torch.device("cuda", torch.cuda.current_device())
        P = width * height
        if layout == REGULAR:
            color = torch.empty((max_n, P, 4), dtype=torch.float32, device=dev)
            depth = torch.empty((max_n, P, 2), dtype=torch.float32, device=dev)
            offset = None
        else:
            cap = capacity if capacity is not None else max_n * P
            color = torch.empty((max(cap, 1), 4), dtype=torch.float32, device=dev)
            depth = torch.empty((max(cap, 1), 2), dtype=torch.float32, device=dev)
            offset = torch.empty((P + 1,), dtype=torch.int32, device=dev)
        count = torch.empty((P,), dtype=torch.int32, device=dev)
        gamma = torch.empty((P,), dtype=torch.float32, device=dev) if with_gamma else None
        return VDI(width, height, max_n, ref_step, layout, color, depth, count, offset, gamma)


def camera_c(cam) -> vdi_camera_t:
    f3 = lambda v: (ctypes.c_float * 3)(*v)
    return vdi_camera_t(int(cam.ortho), f3(cam.eye), f3(cam.fwd), f3(cam.right), f3(cam.up), int(cam.width),
                        int(cam.height))


def tau_c(mode: int, tau: float = 0.0, iters: int = 10, gamma_max: float = 2.0, mlp=None,
          fallback_tol: float = 0.1, feature_scale: float = 32.0, y=None) -> vdi_tau_t:
    return vdi_tau_t(mode, tau, iters, gamma_max, mlp, fallback_tol, feature_scale, y, None)


@dataclasses.dataclass
class DeviceBrick:
    """A brick's halo'd data on the device plus its placement (synth.Brick)."""
    data: torch.Tensor        # [dz, dy, dx] float32 or float16
    lo: Sequence[int]
    hi: Sequence[int]
    data_lo: Sequence[int]
    full_dim: Sequence[int]
    owner: Optional[torch.Tensor] = None   # [nz, ny, nx] uint8 rank per voxel (non-convex domains)
    rank: int = 0

    def c(self) -> vdi_brick_t:
        dz, dy, dx = self.data.shape
        dt = F16 if self.data.dtype == torch.float16 else F32
        i3 = lambda v: (ctypes.c_int32 * 3)(*[int(x) for x in v])
        return vdi_brick_t(_ptr(self.data), dt, i3(self.full_dim), i3(self.lo), i3(self.hi), i3(self.data_lo),
                           i3((dx, dy, dz)), _ptr(self.owner), int(self.rank))


def device_bricks(vol, bricks, device=None, owner=None, ranks=None) -> List[DeviceBrick]:
    """Copy each brick's halo'd block of a [nz, ny, nx] volume (numpy or torch) to
    the device.  owner: optional [nz, ny, nx] uint8 rank per voxel (copied once
    to the device) with ranks[r] brick r's rank (non-convex domains)."""
    import numpy as np
    dev = device or torch.device("cuda", torch.cuda.current_device())
    nz, ny, nx = vol.shape
    own = None
    if owner is not None:
        own = torch.from_numpy(np.ascontiguousarray(owner, dtype=np.uint8)) if isinstance(owner, np.ndarray) \
            else owner.to(torch.uint8)
        own = own.to(dev).contiguous()
        assert tuple(own.shape) == (nz, ny, nx) and ranks is not None and len(ranks) == len(bricks)
    out = []
    for i, b in enumerate(bricks):
        blk = vol[b.data_lo[2]:b.data_hi[2], b.data_lo[1]:b.data_hi[1], b.data_lo[0]:b.data_hi[0]]
        t = torch.from_numpy(np.ascontiguousarray(blk)) if isinstance(blk, np.ndarray) else blk
        out.append(DeviceBrick(t.to(dev).contiguous(), b.lo, b.hi, b.data_lo, (nx, ny, nz), own,
                               int(ranks[i]) if own is not None else 0))
    return out


# ---------------------------------------------------------------- entry points

def generate(bricks: Sequence[DeviceBrick], cam, tf: torch.Tensor, step: float, ref_step: float, mode: int,
             tau: float = 0.0, max_n: int = 8, iters: int = 10, layout: int = REGULAR,
             capacity: Optional[int] = None, outs: Optional[List[VDI]] = None, gamma_max: float = 2.0,
             mlp: Optional["MLP"] = None, fallback_tol: float = 0.1, feature_scale: float = 32.0,
             y: Optional[torch.Tensor] = None) -> List[VDI]:
    """vdi_generate: one sub-VDI per brick (mode LEARNED needs `mlp`, or `y`:
    float32 [k, H*W] log2 thresholds on the device used instead of the MLP)."""
    k = len(bricks)
    if outs is None:
        outs = [VDI.empty(cam.width, cam.height, max_n, ref_step, layout, capacity) for _ in range(k)]
    bc = (vdi_brick_t * k)(*[b.c() for b in bricks])
    oc = (vdi_t * k)(*[o.c() for o in outs])
    cc = camera_c(cam)
    tfc = vdi_tf_t(_ptr(tf), tf.shape[0])
    mc = mlp.c() if mlp is not None else None
    if y is not None:
        if y.dtype != torch.float32 or not y.is_cuda or y.numel() != k * cam.width * cam.height:
            raise ValueError("y must be a float32 device tensor of k*H*W log2 thresholds")
        y = y.contiguous()
    tc = tau_c(mode, tau, iters, gamma_max, ctypes.cast(ctypes.pointer(mc), ctypes.c_void_p) if mc else None,
               fallback_tol, feature_scale, _ptr(y) if y is not None else None)
    _check(lib().vdi_generate(context(), bc, k, ctypes.byref(cc), ctypes.byref(tfc), step, ctypes.byref(tc), oc,
                              _stream()))
    return outs


def composite(vdis: Sequence[VDI], mode: int, tau: float = 0.0, max_n: int = 8, iters: int = 10,
              out: Optional[VDI] = None, gamma_max: float = 2.0, noalloc: bool = False,
              mlp: Optional["MLP"] = None, features: Optional[torch.Tensor] = None) -> VDI:
    """vdi_composite: k-way merge + re-segmentation into one regular VDI
    (noalloc: vdi_composite_noalloc, scratch in the library's fixed array).
    mode LEARNED needs `mlp` (the threshold predictor of the general merge;
    same result as BISECT); features: optional int16 [H*W, 64] device tensor
    receiving the prediction features (bf16 bits) of general-merge pixels."""
    k = len(vdis)
    v0 = vdis[0]
    if out is None:
        out = VDI.empty(v0.width, v0.height, max_n, v0.ref_step, REGULAR)
    ic = (vdi_t * k)(*[v.c() for v in vdis])
    oc = out.c()
    mc = mlp.c() if mlp is not None else None
    tc = tau_c(mode, tau, iters, gamma_max, ctypes.cast(ctypes.pointer(mc), ctypes.c_void_p) if mc else None)
    if features is not None:
        assert features.is_cuda and features.is_contiguous() and features.numel() == out.npix * 64
        tc.features = features.data_ptr()
    fn = lib().vdi_composite_noalloc if noalloc else lib().vdi_composite
    _check(fn(context(), ic, k, ctypes.byref(tc), ctypes.byref(oc), _stream()))
    return out


def render_original_view(v: VDI, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """vdi_render_original_view: premultiplied RGBA [H*W, 4]."""
    if out is None:
        out = torch.empty((v.npix, 4), dtype=torch.float32, device=v.color.device)
    vc = v.c()
    _check(lib().vdi_render_original_view(context(), ctypes.byref(vc), _ptr(out), _stream()))
    return out


def render_novel_view(v: VDI, vdi_cam, view, step: float, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """vdi_render_novel_view: the VDI (generated through vdi_cam) seen from
    camera `view`; premultiplied RGBA [view H*W, 4]."""
    if out is None:
        out = torch.empty((view.width * view.height, 4), dtype=torch.float32, device=v.color.device)
    vc, c0, c1 = v.c(), camera_c(vdi_cam), camera_c(view)
    _check(lib().vdi_render_novel_view(context(), ctypes.byref(vc), ctypes.byref(c0), ctypes.byref(c1), step,
                                       _ptr(out), _stream()))
    return out


def device_status() -> int:
    flags = ctypes.c_int32(0)
    _check(lib().vdi_ctx_device_status(context(), ctypes.byref(flags), _stream()))
    return int(flags.value)


def debug_rays(cam, step: float):
    P = cam.width * cam.height
    dev = torch.device("cuda", torch.cuda.current_device())
    o = torch.empty((P, 3), dtype=torch.float32, device=dev)
    d = torch.empty((P, 3), dtype=torch.float32, device=dev)
    tn = torch.empty((P,), dtype=torch.float32, device=dev)
    tf = torch.empty((P,), dtype=torch.float32, device=dev)
    ns = torch.empty((P,), dtype=torch.int32, device=dev)
    cc = camera_c(cam)
    _check(lib().vdi_debug_rays(context(), ctypes.byref(cc), step, _ptr(o), _ptr(d), _ptr(tn), _ptr(tf), _ptr(ns),
                                _stream()))
    return dict(o=o, d=d, tn=tn, tf=tf, samples=ns)


# ---------------------------------------------------------------- learned threshold

class MLP:
    """The threshold regressor's parameters on the device: a flat fp32 master
    copy and its bf16 bits (VDI_MLP_PARAMS values each), plus Adam moments."""

    def __init__(self, w_f32: torch.Tensor):
        assert w_f32.shape == (MLP_PARAMS,) and w_f32.dtype == torch.float32 and w_f32.is_cuda
        self.w_f32 = w_f32.contiguous()
        self.w_bf16 = torch.empty((MLP_PARAMS,), dtype=torch.int16, device=w_f32.device)
        self.m = torch.zeros_like(self.w_f32)
        self.v = torch.zeros_like(self.w_f32)
        self.step = 0
        mc = self.c()
        _check(lib().vdi_mlp_pack(context(), ctypes.byref(mc), _stream()))

    def save(self, path: str):
        """Checkpoint: fp32 master parameters, Adam moments and step (safetensors)."""
        from safetensors.torch import save_file
        save_file({"w_f32": self.w_f32.cpu(), "m": self.m.cpu(), "v": self.v.cpu(),
                   "step": torch.tensor([self.step], dtype=torch.int64)}, path)

    @staticmethod
    def load(path: str, device=None) -> "MLP":
        """Resume from a checkpoint written by save()."""
        from safetensors.torch import load_file
        d = load_file(path)
        dev = device or torch.device("cuda", torch.cuda.current_device())
        mlp = MLP(d["w_f32"].to(dev))
        mlp.m.copy_(d["m"].to(dev))
        mlp.v.copy_(d["v"].to(dev))
        mlp.step = int(d["step"][0])
        return mlp

    def c(self) -> vdi_mlp_t:
        return vdi_mlp_t(_ptr(self.w_bf16), _ptr(self.w_f32))

    @staticmethod
    def from_numpy_params(params: dict, device=None) -> "MLP":
        import numpy as np
        flat = np.concatenate([params[k].astype(np.float32).ravel() for k in ("W1", "b1", "W2", "b2", "w3", "b3")])
        dev = device or torch.device("cuda", torch.cuda.current_device())
        return MLP(torch.from_numpy(flat).to(dev))

    def to_numpy_params(self) -> dict:
        w = self.w_f32.detach().cpu().numpy()
        sizes = (("W1", (128, 64)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)), ("w3", (128,)), ("b3", (1,)))
        out, o = {}, 0
        for k, shp in sizes:
            n = 1
            for d in shp:
                n *= d
            out[k] = w[o:o + n].reshape(shp).copy()
            o += n
        return out


def tau_features(bricks: Sequence[DeviceBrick], cam, tf: torch.Tensor, step: float, ref_step: float, max_n: int,
                 iters: int = 10, gamma_max: float = 2.0, feature_scale: float = 32.0):
    """vdi_tau_features: (hist bf16 bits [k, P, 64] int16, nnt [k, P], cmax [k, P])."""
    k = len(bricks)
    P = cam.width * cam.height
    dev = bricks[0].data.device
    hist = torch.empty((k, P, 64), dtype=torch.int16, device=dev)
    nnt = torch.empty((k, P), dtype=torch.int32, device=dev)
    cmax = torch.empty((k, P), dtype=torch.int32, device=dev)
    bc = (vdi_brick_t * k)(*[b.c() for b in bricks])
    cc = camera_c(cam)
    tfc = vdi_tf_t(_ptr(tf), tf.shape[0])
    tc = tau_c(LEARNED, 0.0, iters, gamma_max, None, 0.1, feature_scale)
    _check(lib().vdi_tau_features(context(), bc, k, ctypes.byref(cc), ctypes.byref(tfc), step, ref_step, max_n,
                                  ctypes.byref(tc), _ptr(hist), _ptr(nnt), _ptr(cmax), _stream()))
    return hist, nnt, cmax


def mlp_forward(mlp: MLP, x: torch.Tensor, want_acts: bool = False):
    """vdi_mlp_forward on x ([R, 64] bf16 bits as int16 or bfloat16): y [R] (and activations)."""
    x = x.view(torch.int16) if x.dtype == torch.bfloat16 else x
    rows = x.shape[0]
    y = torch.empty((rows,), dtype=torch.float32, device=x.device)
    acts = torch.empty((rows, MLP_ACT_FLOATS), dtype=torch.float32, device=x.device) if want_acts else None
    mc = mlp.c()
    _check(lib().vdi_mlp_forward(context(), ctypes.byref(mc), _ptr(x), rows, _ptr(y), _ptr(acts), _stream()))
    return (y, acts) if want_acts else y


def mlp_backward(mlp: MLP, x: torch.Tensor, acts: torch.Tensor, dy: torch.Tensor) -> torch.Tensor:
    x = x.view(torch.int16) if x.dtype == torch.bfloat16 else x
    grad = torch.empty((MLP_PARAMS,), dtype=torch.float32, device=x.device)
    mc = mlp.c()
    _check(lib().vdi_mlp_backward(context(), ctypes.byref(mc), _ptr(x), _ptr(acts), _ptr(dy.contiguous()),
                                  x.shape[0], _ptr(grad), _stream()))
    return grad


def mlp_adam(mlp: MLP, grad: torch.Tensor, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8):
    mlp.step += 1
    mc = mlp.c()
    _check(lib().vdi_mlp_adam(context(), ctypes.byref(mc), _ptr(grad), _ptr(mlp.m), _ptr(mlp.v), mlp.step, lr,
                              beta1, beta2, eps, _stream()))


def mlp_mse(y: torch.Tensor, gamma: torch.Tensor, scale: float):
    """vdi_mlp_mse: dy = scale * (y - log2 gamma) and the per-block loss sums
    (fp64, 0.5 (y - log2 gamma)^2 over each 256 rows)."""
    rows = y.numel()
    dy = torch.empty_like(y)
    parts = torch.empty(((rows + 255) // 256,), dtype=torch.float64, device=y.device)
    _check(lib().vdi_mlp_mse(context(), _ptr(y), _ptr(gamma), rows, scale, _ptr(dy), _ptr(parts), _stream()))
    return dy, parts


def learned_stats():
    st = (ctypes.c_int64 * 5)()
    _check(lib().vdi_learned_stats(context(), st, _stream()))
    return {"kept": st[0], "shortcut": st[1], "fallback": st[2], "empty": st[3], "refined": st[4]}


def debug_mfma(A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    D = torch.empty((16, 16), dtype=torch.float32, device=A.device)
    _check(lib().vdi_debug_mfma(context(), _ptr(A.contiguous()), _ptr(B.contiguous()), _ptr(D), _stream()))
    return D


# ---------------------------------------------------------------- batched compositing

class vdi_job_t(ctypes.Structure):
    _fields_ = [("in_", ctypes.POINTER(vdi_t)), ("k", ctypes.c_int32), ("out", vdi_t), ("tau", vdi_tau_t)]


def _batch_lib():
    L = lib()
    if not getattr(L, "_batch_ready", False):
        P, I = ctypes.c_void_p, ctypes.c_int
        L.vdi_batch_create.argtypes = [P, ctypes.POINTER(vdi_job_t), I, ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]
        L.vdi_batch_run.argtypes = [P, P, P]
        L.vdi_batch_capture.argtypes = [P, P, P]
        L.vdi_batch_replay.argtypes = [P, P]
        L.vdi_batch_info.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
        L.vdi_batch_destroy.argtypes = [P]
        L.vdi_autotune.argtypes = [P, ctypes.POINTER(vdi_job_t), I, ctypes.c_char_p, P]
        for name in ("vdi_batch_create", "vdi_batch_run", "vdi_batch_capture", "vdi_batch_replay", "vdi_batch_info",
                     "vdi_batch_destroy", "vdi_autotune"):
            getattr(L, name).restype = ctypes.c_int
        L._batch_ready = True
    return L


class Job:
    """One composite of a batch: k input VDIs -> one regular output VDI."""

    def __init__(self, inputs: Sequence[VDI], out: VDI, mode: int = BISECT, tau: float = 0.0, iters: int = 10,
                 gamma_max: float = 2.0):
        self.inputs = list(inputs)
        self.out = out
        self.tau = tau_c(mode, tau, iters, gamma_max)
        self._arr = (vdi_t * len(self.inputs))(*[v.c() for v in self.inputs])

    def c(self) -> vdi_job_t:
        return vdi_job_t(ctypes.cast(self._arr, ctypes.POINTER(vdi_t)), len(self.inputs), self.out.c(), self.tau)


def _jobs_c(jobs: Sequence[Job]):
    return (vdi_job_t * len(jobs))(*[j.c() for j in jobs])


class Batch:
    """vdi_batch_*: a persistent launch over many composites."""

    def __init__(self, jobs: Sequence[Job], autotune_cache: Optional[str] = None):
        self.jobs = list(jobs)
        self._jc = _jobs_c(self.jobs)
        h = ctypes.c_void_p()
        path = autotune_cache.encode() if autotune_cache else None
        _check(_batch_lib().vdi_batch_create(context(), self._jc, len(self.jobs), path, ctypes.byref(h)))
        self.h = h
        self.t_se = torch.zeros((2 * len(self.jobs),), dtype=torch.int64, device="cuda")
        self._graph_stream = None

    def info(self):
        nt, gr, lds = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        hz = ctypes.c_double()
        _check(_batch_lib().vdi_batch_info(self.h, ctypes.byref(nt), ctypes.byref(gr), ctypes.byref(lds),
                                           ctypes.byref(hz)))
        return {"tiles": nt.value, "grid": gr.value, "lds_bytes": lds.value, "clock_hz": hz.value}

    def run(self, timestamps: bool = True):
        _check(_batch_lib().vdi_batch_run(self.h, _ptr(self.t_se) if timestamps else None, _stream()))

    def capture(self, stream: torch.cuda.Stream, timestamps: bool = True):
        """Capture run() into a hipGraph on `stream` (a non-default stream)."""
        self._graph_stream = stream
        _check(_batch_lib().vdi_batch_capture(self.h, _ptr(self.t_se) if timestamps else None,
                                              ctypes.c_void_p(stream.cuda_stream)))

    def replay(self, stream: Optional[torch.cuda.Stream] = None):
        s = stream or self._graph_stream
        _check(_batch_lib().vdi_batch_replay(self.h, ctypes.c_void_p(s.cuda_stream)))

    def latencies_s(self):
        """Per-job (last tile end - first tile start) in seconds, and the batch span."""
        hz = self.info()["clock_hz"]
        t = self.t_se.view(-1, 2).cpu().numpy().astype("uint64")
        lat = (t[:, 1] - t[:, 0]).astype("float64") / hz
        span = float(t[:, 1].max() - t[:, 0].min()) / hz
        return lat, span

    def close(self):
        if self.h:
            _batch_lib().vdi_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(jobs: Sequence[Job], cache_path: str):
    jc = _jobs_c(jobs)
    _check(_batch_lib().vdi_autotune(context(), jc, len(jobs), cache_path.encode(), _stream()))
