"""Scene fitting with the libgs kernels: the anchor (neural-Gaussian) form of
Sec. 2.3 against plain explicit Gaussians, on views rendered from a seeded
ground-truth scene, with held-out PSNR over cumulative GPU time.

Every training step is libgs entry points only (decode, preprocess, binning,
compositing, L1, backward, decoder backward, grouped Adam); PyTorch holds
the buffers. The pair count is read back after each binning pass (the pair
buffers grow as the Gaussians do), for both methods alike. PSNR is
evaluation, computed on the host from the rendered held-out images.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np
import torch

from . import _lib, scenes
from .anchors import ANCHOR_NAMES, MLP_NAMES, AnchorDecoder, to_device
from .rasterizer import PARAM_NAMES, Rasterizer, l1_loss, params_to_device


@dataclasses.dataclass
class FitConfig:
    gt_gaussians: int = 20_000
    anchors: int = 2_000
    train_views: int = 16
    test_views: int = 4
    width: int = 192
    height: int = 192
    steps: int = 300
    eval_every: int = 50
    seed: int = 4
    gt_sh_degree: int = 0
    gt_large_frac: float = 0.05
    anchor_max_steps: int = 0      # > 0: the anchor form may run past `steps` to reach the target
    lr_feat: float = 5e-3
    lr_mlp: float = 2e-3
    lr_offsets: float = 1e-2
    lr_scaling: float = 1e-4
    lrs_plain: dict = dataclasses.field(default_factory=lambda: dict(
        means=1.6e-4, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, sh=2.5e-3))


def _cams(n, seed, w, h):
    res = ((w, h),)
    return scenes.orbit_cameras(n, seed=seed, radius=3.2, jitter=0.35, resolutions=res)


def psnr(img, gt):
    """PSNR of an image in [0, 1] against its reference (evaluation only; the
    mean squared error is summed on the device in FP64)."""
    d = torch.as_tensor(img).to(torch.float64) - torch.as_tensor(gt).to(
        device=torch.as_tensor(img).device, dtype=torch.float64)
    mse = float((d * d).mean().item())
    return -10.0 * math.log10(max(mse, 1e-20))


class _Views:
    """One Rasterizer serving every camera of a fit (all of one resolution):
    the steps render one view at a time, so the per-view buffers are shared
    and only the camera changes."""

    def __init__(self, n, cams, deg):
        self.cams = [_lib.camera(c) for c in cams]
        self.rast = Rasterizer(n, cams[0], deg, headroom=2.0)

    def view(self, v):
        self.rast.cam = self.cams[v]
        return self.rast

    def size(self, p):
        """Pair capacity for the largest view (host reads)."""
        for v in range(len(self.cams)):
            r = self.view(v)
            r.preprocess(p)
            P = r.bin_sort(check_overflow=True)
            if r.capacity < 2 * P + 4096:
                r._alloc_pairs(2 * P + 4096)


def ground_truth(cfg: FitConfig):
    gt = scenes.surface_cloud(cfg.gt_gaussians, seed=cfg.seed, sh_degree=cfg.gt_sh_degree,
                              width=cfg.width, height=cfg.height, large_frac=cfg.gt_large_frac)
    cams = _cams(cfg.train_views + cfg.test_views, cfg.seed + 7, cfg.width, cfg.height)
    p = params_to_device(gt)
    views = _Views(cfg.gt_gaussians, cams, cfg.gt_sh_degree)
    views.size(p)
    imgs = []
    for v in range(len(cams)):
        r = views.view(v)
        r.forward(p, check_overflow=True)
        imgs.append(r.image.clone())
    return gt, cams, imgs


class AnchorModel:
    """Anchors + shared MLP; children decoded per view and rendered directly."""

    def __init__(self, cfg: FitConfig, gt_means, cams):
        a = scenes.anchor_cloud(cfg.anchors, seed=cfg.seed + 1, source_means=gt_means)
        self.a = to_device(a, ANCHOR_NAMES)
        self.m = to_device(scenes.decoder_mlp(seed=cfg.seed + 2), MLP_NAMES)
        # the view-direction inputs start with zero weights: the decoded
        # children are the same for every view at step 0, so the plain model
        # can start from exactly the anchor form's scene (they are learned
        # from there on)
        self.m['w1'][:, _lib.ANCHOR_FEAT:] = 0.0
        self.A = cfg.anchors
        self.dec = AnchorDecoder(self.A)
        self.cams = cams
        self.gcams = [_lib.camera(c) for c in cams]
        self.views = _Views(self.A * _lib.ANCHOR_CHILDREN, cams, _lib.GS_DIRECT)
        # trained: features and the shared MLP (Sec. 2.3), and the child offsets
        # and scaling factors of each anchor; anchor positions stay fixed
        self.train = dict(feat=self.a['feat'], offsets=self.a['offsets'],
                          scaling=self.a['scaling'], **self.m)
        self.lr = dict(feat=cfg.lr_feat, offsets=cfg.lr_offsets, scaling=cfg.lr_scaling,
                       **{k: cfg.lr_mlp for k in MLP_NAMES})
        self.mom = {k: (torch.zeros_like(v), torch.zeros_like(v)) for k, v in self.train.items()}
        self.grads = {k: torch.empty_like(v) for k, v in self.train.items()}
        self.step_count = torch.zeros(1, dtype=torch.int32, device='cuda')
        self.dchild_buf = None
        ch = self.dec.decode(self.a, self.m, self.gcams[0])
        self.views.size(ch)

    def _children(self, v):
        return self.dec.decode(self.a, self.m, self.gcams[v])

    def render(self, v):
        ch = self._children(v)
        r = self.views.view(v)
        r.forward(ch, check_overflow=True)
        return r.image

    def step(self, v, target, loss):
        ch = self._children(v)
        r = self.views.view(v)
        r.forward(ch, check_overflow=True)
        _, dI = l1_loss(r.image, target, None, loss)
        dchild = r.backward(ch, dI, None, self.dchild_buf)
        self.dchild_buf = dchild
        da = {k: self.grads[k] for k in ('feat', 'offsets', 'scaling')}
        dm = {k: self.grads[k] for k in MLP_NAMES}
        self.dec.backward(self.a, self.m, self.gcams[v], dchild, da, dm)
        groups = [(self.train[k], self.grads[k], self.mom[k][0], self.mom[k][1], self.lr[k])
                  for k in self.train]
        _lib.gs_adam_step_grouped(groups, 0.9, 0.999, 1e-15, self.step_count)

    def plain_init(self):
        """The decoded children of view 0 as explicit Gaussians (SH degree 0):
        the plain baseline starts from the same rendered scene."""
        ch = {k: v.clone() for k, v in self._children(0).items()}
        op = ch['opacity_logits'].clamp(1e-4, 1 - 1e-4)
        c0 = 0.5 / math.sqrt(math.pi)
        return dict(means=ch['means'], log_scales=torch.log(ch['log_scales']),
                    quats=ch['quats'], opacity_logits=torch.log(op / (1 - op)),
                    sh=((ch['sh'] - 0.5) / c0).reshape(1, 3, -1).contiguous())


class PlainModel:
    def __init__(self, cfg: FitConfig, init, cams):
        self.p = {k: v.contiguous() for k, v in init.items()}
        self.n = self.p['means'].shape[1]
        self.views = _Views(self.n, cams, 0)
        self.views.size(self.p)
        self.lr = dict(cfg.lrs_plain)
        self.mom = {k: (torch.zeros_like(v), torch.zeros_like(v)) for k, v in self.p.items()}
        self.grads = {k: torch.empty_like(v) for k, v in self.p.items()}
        self.step_count = torch.zeros(1, dtype=torch.int32, device='cuda')

    def render(self, v):
        r = self.views.view(v)
        r.forward(self.p, check_overflow=True)
        return r.image

    def step(self, v, target, loss):
        r = self.views.view(v)
        r.forward(self.p, check_overflow=True)
        _, dI = l1_loss(r.image, target, None, loss)
        r.backward(self.p, dI, None, self.grads)
        groups = [(self.p[k], self.grads[k], self.mom[k][0], self.mom[k][1], self.lr[k])
                  for k in PARAM_NAMES]
        _lib.gs_adam_step_grouped(groups, 0.9, 0.999, 1e-15, self.step_count)


def _evaluate(model, cfg, imgs):
    vals = []
    for t in range(cfg.train_views, cfg.train_views + cfg.test_views):
        vals.append(psnr(model.render(t), imgs[t]))
    return float(np.mean(vals))


def train(model, cfg: FitConfig, imgs, log=None, steps=None, stop_at=None):
    """Returns a list of (step, cumulative GPU ms of training steps, held-out
    PSNR). stop_at: end at the first evaluation that reaches this PSNR."""
    steps = cfg.steps if steps is None else steps
    curve = [(0, 0.0, _evaluate(model, cfg, imgs))]
    loss = torch.zeros(1, device='cuda')
    gpu_ms = 0.0
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rng = np.random.default_rng(cfg.seed + 11)
    order = rng.permutation(cfg.train_views)
    for s in range(1, steps + 1):
        v = int(order[(s - 1) % cfg.train_views])
        a.record()
        model.step(v, imgs[v], loss)
        b.record()
        b.synchronize()
        gpu_ms += a.elapsed_time(b)
        if s % cfg.eval_every == 0 or s == steps:
            curve.append((s, gpu_ms, _evaluate(model, cfg, imgs)))
            if log:
                log(f'[fit] {type(model).__name__} step {s}: {gpu_ms:.1f} ms, '
                    f'PSNR {curve[-1][2]:.2f} dB')
            if stop_at is not None and curve[-1][2] >= stop_at:
                break
    return curve


def time_to(curve, target):
    """First (step, GPU ms) at which the held-out PSNR reaches `target`."""
    for s, ms, p in curve:
        if p >= target:
            return s, ms
    return None


def compare(cfg: FitConfig, log=None):
    """Fit the anchor form and plain Gaussians from the same start; returns
    both curves and the time each needs to come within 0.1 dB of the plain
    model's final held-out PSNR. The plain model runs cfg.steps; the anchor
    form runs cfg.steps, or with cfg.anchor_max_steps > 0 until it reaches
    that PSNR or runs out of steps."""
    gt, cams, imgs = ground_truth(cfg)
    am = AnchorModel(cfg, gt['means'], cams)
    pm = PlainModel(cfg, am.plain_init(), cams)
    cp = train(pm, cfg, imgs, log)
    target = cp[-1][2] - 0.1
    if cfg.anchor_max_steps > 0:
        ca = train(am, cfg, imgs, log, steps=cfg.anchor_max_steps, stop_at=target)
    else:
        ca = train(am, cfg, imgs, log)
    return dict(anchor=ca, plain=cp, target_psnr=target, anchor_time_to_target=time_to(ca, target),
                plain_time_to_target=time_to(cp, target))
