"""Seeded synthetic inputs for VDI generation and compositing.

This module produces *inputs only*: scalar volumes, the 1D transfer-function
table, camera descriptions, brick decompositions and synthetic supersegment
lists.  It contains none of the method's arithmetic (no ray setup, sampling,
segmentation, merging or compositing), so it may serve both the CPU oracle and
the HIP path.

The paper evaluates on real scans and simulations (Table 1) that are not
available here; the generators below stand in for them with smooth Gaussian
blobs plus value noise, the same kind of multi-scale structure a turbulence or
CT volume presents to a raycaster.

Camera convention (shared by every consumer): a camera is the fp32 tuple
(ortho, eye, fwd, right, up, width, height).  For a pixel (i, j), with j = 0
the top row, sx = (2i+1)/W - 1 and sy = 1 - (2j+1)/H.  A perspective ray starts
at `eye` with direction normalize(fwd + sx*right + sy*up); an orthographic ray
starts at eye + sx*right + sy*up with direction `fwd`.  `right` and `up` are
pre-scaled (tan(fovy/2)*aspect and tan(fovy/2) for perspective, the half
extents for orthographic) so that consumers never evaluate a trigonometric
function.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Transfer function
# --------------------------------------------------------------------------


def transfer_function(entries: int = 256, ramp: Tuple[float, float] = (0.2, 0.9)) -> np.ndarray:
    """256-entry RGBA table sampled at s = i/(entries-1).

    Opacity ramps linearly from 0 at s=ramp[0] to 1 at s=ramp[1] (0 below,
    1 above).  RGB is a three-knot multi-hue ramp blue -> green -> red, so the
    colour is never black.  Returned as float32 [entries, 4].
    """
    s = np.arange(entries, dtype=np.float64) / (entries - 1)
    a = np.clip((s - ramp[0]) / (ramp[1] - ramp[0]), 0.0, 1.0)
    r = np.clip((s - 0.5) / 0.5, 0.0, 1.0)
    b = np.clip((0.5 - s) / 0.5, 0.0, 1.0)
    g = 1.0 - r - b
    return np.stack([r, g, b, a], axis=1).astype(np.float32)


# --------------------------------------------------------------------------
# Volumes
# --------------------------------------------------------------------------


def _gaussian_params(rng: np.random.Generator, n: int, count: int, sigma=(4.0, 10.0)):
    centres = rng.uniform(0.0, n, size=(count, 3))          # voxel units, (x, y, z)
    sigmas = rng.uniform(sigma[0], sigma[1], size=count)
    amps = rng.uniform(0.2, 1.0, size=count)
    return centres, sigmas, amps


def _add_gaussians(vol, n: int, centres, sigmas, amps, xp, window: float = 5.0):
    """Accumulate isotropic Gaussians, each truncated to a +-window*sigma box.

    exp(-|x-c|^2/(2 s^2)) separates into per-axis factors, so each Gaussian is
    an outer product over its window.  The truncation (value < 4e-6 outside)
    is part of this generator's definition.
    """
    for (cx, cy, cz), sg, amp in zip(centres, sigmas, amps):
        r = int(math.ceil(window * sg))
        lo = [max(int(math.floor(c)) - r, 0) for c in (cx, cy, cz)]
        hi = [min(int(math.floor(c)) + r + 1, n) for c in (cx, cy, cz)]
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        g = []
        for ax, c in enumerate((cx, cy, cz)):
            idx = xp.arange(lo[ax], hi[ax], dtype=xp.float64) if xp is np else \
                xp.arange(lo[ax], hi[ax], dtype=xp.float64, device=vol.device)
            g.append(xp.exp(-((idx - c) ** 2) / (2.0 * sg * sg)))
        plane = amp * g[1][:, None] * g[0][None, :]
        if xp is not np:
            plane = plane.to(vol.dtype)
            gz = g[2].to(vol.dtype)
        else:
            gz = g[2]
        for z0 in range(lo[2], hi[2], 32):          # bounded temporaries
            z1 = min(z0 + 32, hi[2])
            vol[z0:z1, lo[1]:hi[1], lo[0]:hi[0]] += gz[z0 - lo[2]:z1 - lo[2], None, None] * plane[None]


def _interp_matrix(n: int, cells: int) -> np.ndarray:
    """[n, cells+1] linear-interpolation weights of voxel i at lattice coordinate i*cells/n."""
    u = np.arange(n, dtype=np.float64) * cells / n
    i0 = np.minimum(np.floor(u).astype(np.int64), cells - 1)
    w = u - i0
    m = np.zeros((n, cells + 1), dtype=np.float64)
    m[np.arange(n), i0] = 1.0 - w
    m[np.arange(n), i0 + 1] += w
    return m


def gaussian_volume(n: int, n_gauss: int, seed: int, noise_amp: float = 0.0,
                    dtype: str = "f32", device: str = "cpu", sigma=(4.0, 10.0)):
    """Seeded scalar volume [n, n, n] (z, y, x; x fastest) with values in [0, 1].

    value = clamp(sum_i amp_i * exp(-|x - c_i|^2 / (2 sigma_i^2)) + noise, 0, 1)
    with centres U[0,n)^3 (voxel units), sigma U(sigma) voxels (default 4..10),
    amplitude U(0.2,1).  Noise (if noise_amp > 0) is 4 octaves of trilinearly
    interpolated lattice values U(-1,1) on 8, 16, 32, 64 cells per axis with
    octave weights 1, 1/2, 1/4, 1/8 scaled to a total of noise_amp.

    Small volumes are built with numpy; `device="cuda"` builds large volumes
    with torch on the GPU (random draws always come from numpy's PCG64, so the
    parameters do not depend on the device).  Returns a numpy array for
    device="cpu", else a torch tensor on that device.  dtype "f32" or "f16".
    """
    rng = np.random.default_rng(seed)
    centres, sigmas, amps = _gaussian_params(rng, n, n_gauss, sigma)
    lattices = []
    if noise_amp > 0.0:
        weights = np.array([1.0, 0.5, 0.25, 0.125])
        weights = noise_amp * weights / weights.sum()
        for octave in range(4):
            cells = 8 << octave
            lat = rng.uniform(-1.0, 1.0, size=(cells + 1,) * 3)
            lattices.append((cells, weights[octave], lat))

    if device == "cpu":
        vol = np.zeros((n, n, n), dtype=np.float64 if n <= 256 else np.float32)
        _add_gaussians(vol, n, centres, sigmas, amps, np)
        for cells, wgt, lat in lattices:
            m = _interp_matrix(n, cells).astype(vol.dtype)
            lt = lat.astype(vol.dtype)
            # separable trilinear interpolation: contract x, then y, then z
            t = np.tensordot(lt, m, axes=([2], [1]))                    # [cz, cy, x]
            t = np.ascontiguousarray(np.tensordot(t, m, axes=([1], [1])).transpose(0, 2, 1))  # [cz, y, x]
            for z0 in range(0, n, 64):
                vol[z0:z0 + 64] += wgt * np.tensordot(m[z0:z0 + 64], t, axes=([1], [0]))
        np.clip(vol, 0.0, 1.0, out=vol)
        return vol.astype(np.float16 if dtype == "f16" else np.float32)

    import torch
    dev = torch.device(device)
    vol = torch.zeros((n, n, n), dtype=torch.float32, device=dev)
    _add_gaussians(vol, n, centres, sigmas, amps, torch)
    for cells, wgt, lat in lattices:
        m = torch.from_numpy(_interp_matrix(n, cells)).to(dev, torch.float32)
        lt = torch.from_numpy(lat).to(dev, torch.float32)
        t = torch.tensordot(lt, m, dims=([2], [1]))                  # [cz, cy, x]
        t = torch.tensordot(t, m, dims=([1], [1])).permute(0, 2, 1).contiguous()  # [cz, y, x]
        for z0 in range(0, n, 128):
            vol[z0:z0 + 128] += wgt * torch.tensordot(m[z0:z0 + 128].contiguous(), t, dims=([1], [0]))
    vol.clamp_(0.0, 1.0)
    return vol.to(torch.float16 if dtype == "f16" else torch.float32)


# --------------------------------------------------------------------------
# Bricks (domain decomposition)
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Brick:
    """An owned voxel box [lo, hi) (x, y, z order) and the halo'd data box."""
    lo: Tuple[int, int, int]
    hi: Tuple[int, int, int]
    data_lo: Tuple[int, int, int]
    data_hi: Tuple[int, int, int]


def brick_grid(n: Sequence[int], grid: Sequence[int], halo: int = 1) -> List[Brick]:
    """Split an (nx, ny, nz) voxel grid into gx*gy*gz boxes of near-equal size.

    Bricks are ordered x fastest, then y, then z.  Each brick's data box is its
    owned box grown by `halo` voxels and clipped to the volume.
    """
    cuts = []
    for ax in range(3):
        cuts.append([(n[ax] * i) // grid[ax] for i in range(grid[ax] + 1)])
    out = []
    for bz in range(grid[2]):
        for by in range(grid[1]):
            for bx in range(grid[0]):
                lo = (cuts[0][bx], cuts[1][by], cuts[2][bz])
                hi = (cuts[0][bx + 1], cuts[1][by + 1], cuts[2][bz + 1])
                dlo = tuple(max(l - halo, 0) for l in lo)
                dhi = tuple(min(h + halo, n[a]) for a, h in enumerate(hi))
                out.append(Brick(lo, hi, dlo, dhi))
    return out


def wavy_slab_owner(n: int, slabs: int, amplitude: int, seed: int):
    """Non-convex decomposition of an n^3 volume into `slabs` z-slabs whose
    interfaces are displaced per (x, y) column by a smooth seeded wave of up
    to `amplitude` voxels (as the domains of a simulation that moves its
    interfaces), and each domain's bricks: the bounding box of its voxels with
    a one-voxel halo.  Returns (owner [n, n, n] uint8 (z, y, x), bricks, ranks)."""
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) / n
    cuts = []
    for i in range(1, slabs):
        a = rng.uniform(0.5, 1.0, 2) * amplitude
        f = rng.uniform(1.0, 3.0, 2)
        ph = rng.uniform(0.0, 2.0 * math.pi, 2)
        wave = (a[0] * np.sin(2 * math.pi * f[0] * x[None, :] + ph[0]) +
                a[1] * np.sin(2 * math.pi * f[1] * x[:, None] + ph[1]))   # [y, x]
        cuts.append(np.clip(np.round(n * i / slabs + wave), 1, n - 1).astype(np.int64))
    z = np.arange(n)[:, None, None]
    owner = np.zeros((n, n, n), np.uint8)
    for c in cuts:
        owner += (z >= c[None, :, :]).astype(np.uint8)
    bricks = []
    for r in range(slabs):
        zs = np.nonzero((owner == r).any(axis=(1, 2)))[0]
        lo, hi = (0, 0, int(zs.min())), (n, n, int(zs.max()) + 1)
        dlo = tuple(max(l - 1, 0) for l in lo)
        dhi = tuple(min(h + 1, n) for h in hi)
        bricks.append(Brick(lo, hi, dlo, dhi))
    return owner, bricks, list(range(slabs))


def brick_data(vol, b: Brick):
    """The halo'd block of `vol` ([z, y, x]) a brick holds, as a contiguous copy."""
    blk = vol[b.data_lo[2]:b.data_hi[2], b.data_lo[1]:b.data_hi[1], b.data_lo[0]:b.data_hi[0]]
    return blk.copy() if isinstance(blk, np.ndarray) else blk.contiguous()


# --------------------------------------------------------------------------
# Cameras
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Camera:
    ortho: int
    eye: Tuple[float, float, float]
    fwd: Tuple[float, float, float]
    right: Tuple[float, float, float]
    up: Tuple[float, float, float]
    width: int
    height: int

    def as_f32(self) -> "Camera":
        f = lambda v: tuple(float(np.float32(x)) for x in v)
        return Camera(self.ortho, f(self.eye), f(self.fwd), f(self.right), f(self.up),
                      self.width, self.height)


def _normalize(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def ortho_camera(width: int, height: int, axis: str = "+z") -> Camera:
    """Orthographic view of the unit box along +z or -z, image covering [0,1]^2."""
    if axis == "+z":
        eye, fwd = (0.5, 0.5, 0.0), np.array([0.0, 0.0, 1.0])
    elif axis == "-z":
        eye, fwd = (0.5, 0.5, 1.0), np.array([0.0, 0.0, -1.0])
    else:
        raise ValueError(axis)
    up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    return Camera(1, eye, tuple(fwd), tuple(0.5 * right), tuple(0.5 * up), width, height).as_f32()


def perspective_camera(eye, target, width: int, height: int, fovy_deg: float = 60.0) -> Camera:
    fwd = _normalize(np.asarray(target, np.float64) - np.asarray(eye, np.float64))
    right = _normalize(np.cross(fwd, [0.0, 1.0, 0.0]))
    up = np.cross(right, fwd)
    th = math.tan(math.radians(fovy_deg) / 2.0)
    return Camera(0, tuple(eye), tuple(fwd), tuple(th * (width / height) * right), tuple(th * up),
                  width, height).as_f32()


def orbit_camera(seed: int, width: int, height: int, radius: float = 1.8,
                 max_elev_deg: float = 30.0, fovy_deg: float = 60.0, turn_deg: float = 0.0) -> Camera:
    """Perspective camera on a seeded orbit about the box centre, looking at it;
    turn_deg moves it along the orbit (azimuth) by that angle, a viewpoint
    deviation about the box centre."""
    rng = np.random.default_rng(seed)
    az = rng.uniform(0.0, 2.0 * math.pi) + math.radians(turn_deg)
    el = math.radians(rng.uniform(-max_elev_deg, max_elev_deg))
    c = np.array([0.5, 0.5, 0.5])
    eye = c + radius * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    return perspective_camera(tuple(eye), tuple(c), width, height, fovy_deg)


# --------------------------------------------------------------------------
# Synthetic supersegment lists (compositing stress inputs)
# --------------------------------------------------------------------------


def dense_interleaved_lists(k: int, n_per: int, npix: int, seed: int, depth_range: float = 3.0,
                            device: str = "cpu", alpha_range=(0.02, 0.6)):
    """k rank lists of exactly n_per supersegments for each of npix pixels.

    Per pixel, 2*k*n_per increasing cut points in (0, depth_range) give
    k*n_per disjoint intervals (gaps between consecutive cuts are U(0.05,1.05)
    before normalisation, so no two cuts coincide in fp32); a seeded shuffle
    assigns the intervals to ranks, so the ranks interleave along every ray.
    Colour is U(0,1)^3, per-unit opacity U(alpha_range).  Returns torch tensors
    (color [k, n_per, npix, 4], depth [k, n_per, npix, 2], count [k, npix]) in
    slot-major regular layout.
    """
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    total = k * n_per
    gaps = torch.rand((npix, 2 * total + 1), generator=gen, device=device, dtype=torch.float64) + 0.05
    cuts = torch.cumsum(gaps, dim=1)
    cuts = (cuts[:, :-1] / cuts[:, -1:] * depth_range).to(torch.float32)
    front, back = cuts[:, 0::2], cuts[:, 1::2]                  # [npix, total]
    keys = torch.rand((npix, total), generator=gen, device=device)
    perm = torch.argsort(keys, dim=1)                            # cell ids in rank-major order
    sel = perm.view(npix, k, n_per).sort(dim=2).values           # each rank's cells, depth-sorted
    f = torch.gather(front, 1, sel.view(npix, total)).view(npix, k, n_per)
    b = torch.gather(back, 1, sel.view(npix, total)).view(npix, k, n_per)
    rgb = torch.rand((npix, k, n_per, 3), generator=gen, device=device)
    a = alpha_range[0] + (alpha_range[1] - alpha_range[0]) * torch.rand((npix, k, n_per, 1), generator=gen, device=device)
    color = torch.cat([rgb, a], dim=3).permute(1, 2, 0, 3).contiguous()
    depth = torch.stack([f, b], dim=3).permute(1, 2, 0, 3).contiguous()
    count = torch.full((k, npix), n_per, dtype=torch.int32, device=device)
    return color, depth, count


def dense_frame(k: int, n_per: int, npix: int, seed: int, device: str = "cuda", chunk: int = 1 << 17):
    """dense_interleaved_lists for a whole frame, generated in pixel chunks of
    `chunk` (chunk c seeded seed*1000 + c) into preallocated slot-major
    tensors: color [k, n_per, npix, 4], depth [k, n_per, npix, 2], count [k, npix]."""
    import torch
    color = torch.empty((k, n_per, npix, 4), dtype=torch.float32, device=device)
    depth = torch.empty((k, n_per, npix, 2), dtype=torch.float32, device=device)
    for p0 in range(0, npix, chunk):
        p1 = min(npix, p0 + chunk)
        c, d, _ = dense_interleaved_lists(k, n_per, p1 - p0, seed=seed * 1000 + p0 // chunk, device=device)
        color[:, :, p0:p1] = c
        depth[:, :, p0:p1] = d
    count = torch.full((k, npix), n_per, dtype=torch.int32, device=device)
    return color, depth, count


# --------------------------------------------------------------------------
# Workload presets
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    n_gauss: int
    noise: float
    vol_dtype: str
    grid: Tuple[int, int, int]
    sigma: Tuple[float, float]
    width: int
    height: int
    mode: str          # "fixed" | "bisect"
    tau: float
    max_n: int
    iters: int
    seed: int


def tiny(seed: int = 0) -> Workload:
    """64^3 fp32, 12 Gaussians, 2 z-slabs, 256^2 ortho along +z, fixed tau 0.05, N=8."""
    return Workload("tiny-64c-2slab-256sq-fixed", 64, 12, 0.0, "f32", (1, 1, 2), (4.0, 10.0), 256, 256,
                    "fixed", 0.05, 8, 10, seed)


def scaled_sigma(n: int) -> Tuple[float, float]:
    """Gaussian widths that keep the feature size a fixed fraction of the box:
    U(4,10) voxels at 128^3, i.e. 16..40 voxels at 512^3 and 32..80 at 1024^3.
    With widths fixed in voxels the large volumes would be nearly empty
    (mean value 0.013 at 512^3), unlike any of the paper's datasets."""
    return (4.0 * n / 128, 10.0 * n / 128)


def fhd(seed: int = 0) -> Workload:
    """512^3 fp32, 200 Gaussians + noise 0.1, 8 z-slabs, 1920x1080 orbit view, bisection N=20."""
    return Workload("fhd-512c-8slab-1920x1080-bisect-N20", 512, 200, 0.1, "f32", (1, 1, 8), scaled_sigma(512),
                    1920, 1080, "bisect", 0.0, 20, 10, seed)


def large(seed: int = 0) -> Workload:
    """1024^3 fp16, same generator, 16 bricks 4x2x2, 1920x1080 orbit view, bisection N=20."""
    return Workload("large-1024c-f16-16brick-1920x1080-bisect-N20", 1024, 200, 0.1, "f16", (4, 2, 2),
                    scaled_sigma(1024), 1920, 1080, "bisect", 0.0, 20, 10, seed)


def workload_volume(w: Workload, device: str = "cpu"):
    return gaussian_volume(w.n, w.n_gauss, w.seed, w.noise, w.vol_dtype, device=device, sigma=w.sigma)


def camera_for(w: Workload) -> Camera:
    if w.mode == "fixed" and w.width == w.height and w.n <= 64:
        return ortho_camera(w.width, w.height, "+z")
    return orbit_camera(10_000 + w.seed, w.width, w.height)


# --------------------------------------------------------------------------
# Batched compositing workload
# --------------------------------------------------------------------------

BATCH_RESOLUTIONS = ((256, 256), (512, 512), (1280, 720), (1920, 1080))
BATCH_N = (8, 16, 20, 32)


def batch_jobs(seed: int = 5000, n_jobs: int = 64):
    """Seeded job list of the batched workload: (width, height, k, N) per job,
    resolution from BATCH_RESOLUTIONS, k uniform in 2..16, N from BATCH_N."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_jobs):
        w, h = BATCH_RESOLUTIONS[int(rng.integers(0, len(BATCH_RESOLUTIONS)))]
        k = int(rng.integers(2, 17))
        n = int(BATCH_N[int(rng.integers(0, len(BATCH_N)))])
        out.append((w, h, k, n))
    return out


def batch_pool_workload(seed: int = 5000) -> Workload:
    """Source of the pooled sub-VDIs of the batched workload: a 256^3 fp32
    volume of 200 Gaussians (+ noise) in 16 bricks (4x2x2)."""
    return Workload("batch-pool-256c-16brick", 256, 200, 0.1, "f32", (4, 2, 2), scaled_sigma(256), 0, 0,
                    "bisect", 0.0, 0, 10, seed)
