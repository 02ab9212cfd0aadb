"""Learned per-ray threshold: training-pair generation, training and evaluation.

An extension beyond the paper.  The per-ray bisection of Sec. 2.4 costs up to
B+1 passes over a brick-ray; the regressor predicts log2(gamma*) from a 64-bin
histogram of the ray's sample opacities so that generation needs a feature
pass and one generation pass, falling back to the bisection on rays whose
count misses the target.  Every numeric step runs in libvdi's kernels
(features, MLP forward/backward/Adam, generation); this module only schedules
them.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Sequence, Tuple

import numpy as np
import torch

from . import synth, vdi


@dataclasses.dataclass
class LearnedConfig:
    """Setting of the learned threshold.

    kind "tiny": the tiny volumes (64^3 fp32, 12 Gaussians, 2 z-slabs),
    orthographic views along +z (even seeds) or -z (odd seeds), N=8, B=10.
    Training frames are train_res, evaluation frames res (1024^2 x 2 bricks =
    2.1M brick-rays per frame).

    kind "fhd": the FHD generator (512^3 fp32, 200 Gaussians + noise, 8
    z-slabs) under seeded orbit cameras, N=20 as in the FHD workload; the
    rays are ten times longer."""
    kind: str = "tiny"
    n: int = 64
    n_gauss: int = 12
    res: Tuple[int, int] = (1024, 1024)
    train_res: Tuple[int, int] = (640, 640)
    grid: Tuple[int, int, int] = (1, 1, 2)
    max_n: int = 8
    iters: int = 10
    gamma_max: float = 2.0
    feature_scale: float = 32.0
    max_pairs: int = 8 << 20

    @staticmethod
    def fhd() -> "LearnedConfig":
        return LearnedConfig(kind="fhd", n=512, n_gauss=200, res=(1920, 1080), train_res=(640, 360),
                             grid=(1, 1, 8), max_n=20)

    def describe(self) -> str:
        view = "ortho +-z" if self.kind == "tiny" else "orbit perspective"
        return (f"{self.n}^3, {self.grid} bricks, {self.res[0]}x{self.res[1]} {view} views, N={self.max_n}")


def frame_inputs(cfg: LearnedConfig, seed: int, res: Tuple[int, int]):
    """Volume (host array for tiny, device tensor for fhd), bricks and camera of one frame."""
    if cfg.kind == "tiny":
        vol = synth.gaussian_volume(cfg.n, cfg.n_gauss, seed)
        bricks = synth.brick_grid((cfg.n,) * 3, cfg.grid)
        cam = synth.ortho_camera(res[0], res[1], "+z" if seed % 2 == 0 else "-z")
        return vol, bricks, cam
    w = dataclasses.replace(synth.fhd(seed), width=res[0], height=res[1])
    vol = synth.workload_volume(w, device="cuda")
    bricks = synth.brick_grid((cfg.n,) * 3, cfg.grid)
    return vol, bricks, synth.camera_for(w)


def training_pairs(cfg: LearnedConfig, seeds: Sequence[int], tf_d: torch.Tensor
                   ) -> Tuple[torch.Tensor, torch.Tensor, Dict[str, int]]:
    """(histogram, gamma*) pairs from the plain bisection on the GPU, at most
    cfg.max_pairs (a seeded subsample when there are more); the regressor's
    target is log2 gamma* (taken in the loss kernel).

    Brick-rays with at most N non-transparent samples are left out: every
    threshold is feasible there and the learned path resolves them exactly
    without the regressor."""
    xs, ys = [], []
    stats = {"rays": 0, "kept": 0}
    step = 1.0 / cfg.n
    for seed in seeds:
        vol, bricks, cam = frame_inputs(cfg, seed, cfg.train_res)
        dbr = vdi.device_bricks(vol, bricks)
        outs = vdi.generate(dbr, cam, tf_d, step, step, vdi.BISECT, 0.0, cfg.max_n, cfg.iters,
                            gamma_max=cfg.gamma_max)
        hist, nnt, cmax = vdi.tau_features(dbr, cam, tf_d, step, step, cfg.max_n, cfg.iters, cfg.gamma_max,
                                           cfg.feature_scale)
        gam = torch.stack([o.gamma for o in outs])            # [k, P]
        keep = nnt > cfg.max_n
        stats["rays"] += int(nnt.numel())
        stats["kept"] += int(keep.sum())
        xs.append(hist[keep])
        ys.append(gam[keep])
        del dbr, outs, vol
    X, Y = torch.cat(xs), torch.cat(ys)
    if X.shape[0] > cfg.max_pairs:
        g = torch.Generator(device=X.device)
        g.manual_seed(1)
        idx = torch.randperm(X.shape[0], generator=g, device=X.device)[:cfg.max_pairs]
        X, Y = X[idx].contiguous(), Y[idx].contiguous()
    stats["pairs"] = int(X.shape[0])
    return X, Y, stats


def train(mlp: vdi.MLP, X: torch.Tensor, Y: torch.Tensor, epochs: int = 4, batch: int = 4096, lr: float = 2e-3,
          seed: int = 0, log=None, start_epoch: int = 0) -> List[float]:
    """Adam on 0.5 * mean squared error of log2(gamma) (Y holds gamma*);
    returns per-epoch mean loss.  Epoch e draws its batch order from seed + e
    and halves the rate every two epochs, so training resumed at start_epoch
    from a checkpoint taken after epoch start_epoch - 1 continues exactly."""
    import numpy as np
    R = X.shape[0]
    hist = []
    for ep in range(start_epoch, epochs):
        g = torch.Generator(device=X.device)
        g.manual_seed(seed + ep)
        perm = torch.randperm(R, generator=g, device=X.device)
        parts = []
        for b0 in range(0, R - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb = X[idx].contiguous()
            tb = Y[idx].contiguous()
            y, acts = vdi.mlp_forward(mlp, xb, want_acts=True)
            dy, lp = vdi.mlp_mse(y, tb, 1.0 / batch)
            parts.append(lp)
            grad = vdi.mlp_backward(mlp, xb, acts, dy)
            vdi.mlp_adam(mlp, grad, lr=lr * (0.5 ** (ep // 2)))
        loss = float(np.sum([p.cpu().numpy().sum() for p in parts])) / max(len(parts) * batch, 1)
        hist.append(loss)
        if log:
            log(f"[learned] epoch {ep + 1}/{epochs}: loss {hist[-1]:.4f}")
    return hist


def init_mlp(seed: int = 0, device=None) -> vdi.MLP:
    """He-initialised weights (fp32 master); output bias at the mean log2 gamma range."""
    rng = np.random.default_rng(seed)
    params = {
        "W1": (rng.standard_normal((128, 64)) * math.sqrt(2.0 / 64)).astype(np.float32),
        "b1": np.zeros(128, np.float32),
        "W2": (rng.standard_normal((128, 128)) * math.sqrt(2.0 / 128)).astype(np.float32),
        "b2": np.zeros(128, np.float32),
        "w3": (rng.standard_normal(128) * math.sqrt(1.0 / 128)).astype(np.float32),
        "b3": np.full(1, -4.0, np.float32),
    }
    return vdi.MLP.from_numpy_params(params, device)


def timed(fn, reps: int = 3) -> float:
    """Median milliseconds of fn() measured with HIP events on the current stream."""
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def evaluate(mlp: vdi.MLP, cfg: LearnedConfig, seeds: Sequence[int], tf_d: torch.Tensor,
             reps: int = 3) -> Dict[str, float]:
    """Plain bisection vs learned generation on held-out frames: time, the
    share of served lists whose steered scan settled every remaining level,
    and whether the VDIs are identical (they must be: the learned path only
    reorders the bisection's scans).  The learned path is also timed with the
    exact threshold supplied as the regressed one (log2 of the bisection's
    result, a hair below it, so every steered decision is right): the ceiling
    any regressor can reach.  The plain search is timed twice:
    speculative (several midpoints per pass, the library's BISECT) and one
    midpoint per pass (BISECT_SEQ, the search as the paper runs it); both give
    the same VDIs.  The original-view renderings of the composited VDIs are
    compared as well."""
    step = 1.0 / cfg.n
    t_plain = t_learned = t_seq = t_exact = 0.0
    agg = {"kept": 0, "refined": 0, "shortcut": 0, "empty": 0}
    mae_learned = 0.0
    identical = True
    frames = 0
    rays = 0
    for seed in seeds:
        vol, bricks, cam = frame_inputs(cfg, seed, cfg.res)
        dbr = vdi.device_bricks(vol, bricks)
        P = cam.width * cam.height
        outs_p = [vdi.VDI.empty(cam.width, cam.height, cfg.max_n, step) for _ in bricks]
        outs_l = [vdi.VDI.empty(cam.width, cam.height, cfg.max_n, step) for _ in bricks]
        run_p = lambda: vdi.generate(dbr, cam, tf_d, step, step, vdi.BISECT, 0.0, cfg.max_n, cfg.iters,
                                     outs=outs_p, gamma_max=cfg.gamma_max)
        run_l = lambda: vdi.generate(dbr, cam, tf_d, step, step, vdi.LEARNED, 0.0, cfg.max_n, cfg.iters,
                                     outs=outs_l, gamma_max=cfg.gamma_max, mlp=mlp, feature_scale=cfg.feature_scale)
        run_s = lambda: vdi.generate(dbr, cam, tf_d, step, step, vdi.BISECT_SEQ, 0.0, cfg.max_n, cfg.iters,
                                     outs=outs_p, gamma_max=cfg.gamma_max)
        run_s()
        run_p()
        run_l()
        torch.cuda.synchronize()
        vdi.learned_stats()
        t_seq += timed(run_s, reps)
        t_plain += timed(run_p, reps)
        t_learned += timed(run_l, reps)
        st = vdi.learned_stats()
        for k in agg:
            agg[k] += st[k] // reps
        y_exact = torch.log2(torch.stack([o.gamma for o in outs_p]).double() * (1.0 - 1e-4)).float().contiguous()
        run_e = lambda: vdi.generate(dbr, cam, tf_d, step, step, vdi.LEARNED, 0.0, cfg.max_n, cfg.iters,
                                     outs=outs_l, gamma_max=cfg.gamma_max, y=y_exact,
                                     feature_scale=cfg.feature_scale)
        run_e()
        t_exact += timed(run_e, reps)
        vdi.learned_stats()
        for a, b in zip(outs_p, outs_l):
            identical &= bool(torch.equal(a.count, b.count) and torch.equal(a.gamma, b.gamma)
                              and torch.equal(a.color, b.color) and torch.equal(a.depth, b.depth))
        comp_p = vdi.composite(outs_p, vdi.BISECT, 0.0, cfg.max_n, cfg.iters)
        comp_l = vdi.composite(outs_l, vdi.BISECT, 0.0, cfg.max_n, cfg.iters)
        mae_learned += float((vdi.render_original_view(comp_l) - vdi.render_original_view(comp_p)).abs().mean())
        frames += 1
        rays += len(bricks) * P
    served = agg["kept"] + agg["refined"]
    return {
        "frames": frames,
        "brick_rays": rays,
        "plain_ms": t_plain / frames,
        "learned_ms": t_learned / frames,
        "speedup": t_plain / t_learned,
        "plain_seq_ms": t_seq / frames,
        "speedup_vs_seq": t_seq / t_learned,
        "exact_threshold_ms": t_exact / frames,
        "speedup_exact_threshold": t_plain / t_exact,
        "kept_rate": agg["kept"] / max(served, 1),
        **agg,
        "identical_to_plain": identical,
        "rgba_mae_vs_plain_render": mae_learned / frames,
    }


# ---------------------------------------------------------------- compositing

def composite_training_pairs(seeds: Sequence[int], k: int = 16, n: int = 20, out_n: int = 20,
                             width: int = 512, height: int = 256
                             ) -> Tuple[torch.Tensor, torch.Tensor, Dict[str, int]]:
    """(features, gamma*) pairs of the compositing bisection: for maximally
    interleaved inputs of k lists of n supersegments per pixel (the dense
    stress generator, seeded), the general merge's prediction features and
    the plain bisection's threshold of every pixel it re-segmented."""
    xs, ys = [], []
    P = width * height
    for seed in seeds:
        c, d, cnt = synth.dense_interleaved_lists(k, n, P, seed=seed, device="cuda")
        ins = [vdi.VDI(width, height, n, 0.01, vdi.REGULAR, c[r].contiguous(), d[r].contiguous(),
                       cnt[r].contiguous()) for r in range(k)]
        feat = torch.zeros((P, 64), dtype=torch.int16, device="cuda")
        out = vdi.composite(ins, vdi.BISECT, 0.0, out_n, 10, features=feat)
        keep = cnt.sum(dim=0) > out_n
        xs.append(feat[keep])
        ys.append(out.gamma[keep])
        del ins, c, d, out
    X, Y = torch.cat(xs).contiguous(), torch.cat(ys).contiguous()
    return X, Y, {"pairs": int(X.shape[0])}


def evaluate_composite(mlp: vdi.MLP, ins: Sequence[vdi.VDI], out_n: int, reps: int = 5) -> Dict[str, float]:
    """The composite of `ins` with the bisection's first scan steered by the
    out_n-th-largest-distance rule (BISECT) and by the regressor (LEARNED):
    median time of each and whether the outputs are identical (they must be)."""
    a = vdi.composite(ins, vdi.BISECT, 0.0, out_n, 10)
    b = vdi.composite(ins, vdi.LEARNED, 0.0, out_n, 10, mlp=mlp)
    torch.cuda.synchronize()
    same = all(torch.equal(getattr(a, f), getattr(b, f)) for f in ("color", "depth", "count", "gamma"))
    t_p = timed(lambda: vdi.composite(ins, vdi.BISECT, 0.0, out_n, 10, out=a), reps)
    t_l = timed(lambda: vdi.composite(ins, vdi.LEARNED, 0.0, out_n, 10, out=b, mlp=mlp), reps)
    return {"bisect_ms": t_p, "learned_ms": t_l, "speedup": t_p / t_l, "identical": bool(same)}
