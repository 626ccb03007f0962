"""Densifying fit (the final round's training, Sec. 3.1-3.2): explicit Gaussians trained from a
sparse start on views of a seeded ground-truth scene, with

  * the photometric loss of Eq. 5, (1 - lambda) L1 + lambda (1 - SSIM)
    (plain L1 with ssim_lambda = 0), plus a depth L1 term whose weight starts at 0.1
    and falls linearly to 0 over the run (depth regularisation), against a
    noisy copy of the ground-truth blended depth, or of the blended inverse
    depth (disparity, which the paper supervises) with depth_mode 1;
  * multi-view score-guided growth and pruning (Eq. 3-4, 6) at fixed
    intervals: K sampled training views are rendered, their Eq. 3 error
    masks built, the Eq. 4 counts summed (and, weighted by each view's
    Eq. 5 loss, the Eq. 6 pruning score), the Gaussians whose count reaches
    the threshold are cloned or split, and those whose normalised pruning
    score exceeds prune_threshold are removed.

Every training step and every densification event is libgs entry points
(preprocess, binning, compositing, photometric and depth losses, backward,
grouped Adam; photometric loss, error mask, split score, score accumulation,
threshold, plan, apply). PyTorch holds the buffers
and draws the split children's standard-normal offsets. The host reads the
pair count after each binning pass (the pair buffers grow with the scene)
and the threshold and output count of each densification event.

The threshold of an event is the paper's predefined lower bound on the mean
count per view (min_score, times K) raised, when needed, to keep the event
within its growth budget: the target count follows a geometric schedule from
the initial count to `growth_to` over the events.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Optional

import numpy as np
import torch

from . import _lib, scenes
from .rasterizer import PARAM_NAMES, Adam, Rasterizer, l1_loss, params_to_device


@dataclasses.dataclass
class DensifyConfig:
    gt_gaussians: int = 1_000_000
    init_gaussians: int = 300_000
    growth_to: int = 3_000_000
    views: int = 200
    holdout_every: int = 8
    width: int = 1600
    height: int = 1066
    sh_degree: int = 3
    steps: int = 6000
    densify_from: int = 500
    densify_until: int = 4000
    densify_every: int = 500
    k_views: int = 10
    tau: float = 0.1
    min_score: float = 2.0       # lower bound on s+ (masked pixels per view)
    split_scale: float = 0.02    # clone at or below this largest scale, else split
    depth_weight: float = 0.1
    depth_noise: float = 0.01
    depth_mode: int = 0          # 0: depth channel p_z; 1: inverse depth (disparity)
    ssim_lambda: float = 0.2     # Eq. 5 weight of the SSIM term (0: plain L1)
    prune_threshold: Optional[float] = 0.9   # Eq. 6 (None: no pruning)
    orbit_radius: float = 4.0
    seed: int = 5
    lrs: dict = dataclasses.field(default_factory=lambda: dict(
        means=1.6e-4, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, sh=2.5e-3))


def psnr(img, gt):
    mse = float(np.mean((np.asarray(img, np.float64) - np.asarray(gt, np.float64)) ** 2))
    return -10.0 * math.log10(max(mse, 1e-20))


def _alloc_like(p, n):
    return {k: torch.empty(tuple(v.shape[:-1]) + (n,), dtype=v.dtype, device=v.device)
            for k, v in p.items()}


class DensifyFit:
    """State of one densifying fit: ground truth, the trained Gaussians, one
    rasterizer (all views share a resolution; the camera is switched per
    step), optimiser moments and the densification scratch."""

    def __init__(self, cfg: DensifyConfig, log: Optional[Callable[[str], None]] = None):
        self.cfg = cfg
        self.log = log or (lambda s: None)
        dev = torch.device('cuda')
        t0 = time.perf_counter()
        gt = scenes.surface_cloud(cfg.gt_gaussians, seed=cfg.seed, sh_degree=cfg.sh_degree,
                                  width=16, height=16)
        cams = scenes.orbit_cameras(cfg.views, seed=cfg.seed + 1, radius=cfg.orbit_radius,
                                    resolutions=((cfg.width, cfg.height),))
        for c in cams:
            c.depth_mode = cfg.depth_mode
        self.cams = cams
        self.gcams = [_lib.camera(c) for c in cams]
        self.test = [v for v in range(cfg.views) if v % cfg.holdout_every == 0]
        self.train = [v for v in range(cfg.views) if v % cfg.holdout_every != 0]
        self.HW = cfg.width * cfg.height
        # ground-truth images and depths, and the noisy depth targets
        gp = params_to_device(gt)
        R = Rasterizer(cfg.gt_gaussians, cams[0], cfg.sh_degree, headroom=1.5)
        gen = torch.Generator(device=dev)
        gen.manual_seed(cfg.seed + 2)
        self.gt_img, self.gt_depth = [], []
        for v in range(cfg.views):
            R.cam = self.gcams[v]
            R.forward(gp, check_overflow=True)
            self.gt_img.append(R.image.clone())
            noise = torch.randn(R.depth.shape, generator=gen, device=dev)
            self.gt_depth.append((R.depth * (1.0 + cfg.depth_noise * noise)).contiguous())
        del R, gp
        torch.cuda.synchronize()
        self.gt_seconds = time.perf_counter() - t0
        init = scenes.sparse_init(gt['means'], cfg.init_gaussians, seed=cfg.seed + 3,
                                  sh_degree=cfg.sh_degree)
        self.p = params_to_device(init)
        self.n = cfg.init_gaussians
        self.adam = Adam(self.p, cfg.lrs)
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(cfg.seed + 4)
        self.rng = np.random.default_rng(cfg.seed + 5)
        self.loss = torch.zeros(1, device=dev)
        self.loss_d = torch.zeros(1, device=dev)
        self.dI = torch.empty((3, cfg.height, cfg.width), device=dev)
        self.dD = torch.empty((cfg.height, cfg.width), device=dev)
        self.mask = torch.empty(self.HW, dtype=torch.uint8, device=dev)
        self.minmax = torch.empty(2, dtype=torch.int32, device=dev)
        self.hist = torch.empty(_lib.SCORE_BINS, dtype=torch.int32, device=dev)
        self.thr = torch.zeros(1, dtype=torch.int32, device=dev)
        self.photo = torch.zeros(3, device=dev)
        self.photo_ws = torch.empty(_lib.gs_photo_loss_workspace(3, cfg.height, cfg.width),
                                    dtype=torch.uint8, device=dev)
        self.n_out = torch.zeros(1, dtype=torch.int32, device=dev)
        self.R = None
        self._setup(self.n, capacity=0)
        self.events = []
        self.on_event = None   # optional hook(dict: score, prune, t_min, cap, threshold)

    # -- buffers sized to the Gaussian count --------------------------------
    def _setup(self, n, capacity):
        self.R = Rasterizer(n, self.cams[0], self.cfg.sh_degree, capacity=capacity, headroom=1.5)
        self.grads = {k: torch.empty_like(v) for k, v in self.p.items()}
        self.score = torch.empty(n, dtype=torch.int32, device='cuda')
        self.count = torch.empty(n, dtype=torch.int32, device='cuda')
        self.prune = torch.empty(n, dtype=torch.float64, device='cuda')
        self.ws = torch.empty(_lib.gs_densify_workspace(n), dtype=torch.uint8, device='cuda')

    def n_events(self):
        c = self.cfg
        return len(range(c.densify_from, c.densify_until + 1, c.densify_every))

    # -- one training step ----------------------------------------------------
    def step(self, s, v):
        c, R = self.cfg, self.R
        R.cam = self.gcams[v]
        R.forward(self.p, check_overflow=True)
        if c.ssim_lambda > 0:
            _lib.gs_photo_loss(R.image, self.gt_img[v], 3, c.height, c.width, c.ssim_lambda,
                               self.photo_ws, self.photo, self.dI)
        else:
            l1_loss(R.image, self.gt_img[v], self.dI, self.loss)
        w = c.depth_weight * max(0.0, 1.0 - s / c.steps)
        self.loss_d.zero_()
        _lib.gs_depth_l1_loss(R.depth, self.gt_depth[v], self.HW, w, self.dD, self.loss_d)
        R.backward(self.p, self.dI, self.dD, self.grads)
        self.adam.step(self.grads)

    # -- one densification event --------------------------------------------
    def densify(self, event):
        c, R, n = self.cfg, self.R, self.n
        self.score.zero_()
        self.prune.zero_()
        for v in self.rng.choice(self.train, c.k_views, replace=False):
            R.cam = self.gcams[int(v)]
            R.forward(self.p, check_overflow=True)
            gt = self.gt_img[int(v)]
            _lib.gs_error_mask(R.image, gt, self.HW, c.tau, self.mask, self.minmax)
            # this view's Eq. 4 counts, added to the split score and, times
            # its Eq. 5 loss, to the pruning score
            _lib.gs_photo_loss(R.image, gt, 3, c.height, c.width, max(c.ssim_lambda, 0.0),
                               self.photo_ws, self.photo, None)
            self.count.zero_()
            _lib.gs_split_score(R.splats, n, R.vals, R.ranges, R.cam, self.mask, self.count)
            _lib.gs_prune_accumulate(self.count, n, self.photo, self.prune, self.score)
        E = self.n_events()
        target = round(c.init_gaussians * (c.growth_to / c.init_gaussians) ** (event / E))
        cap = max(0, target - n)
        t_min = max(1, math.ceil(c.k_views * c.min_score))
        _lib.gs_densify_threshold(self.score, n, t_min, cap, self.hist, self.thr)
        thr = int(self.thr.item()) & 0xFFFFFFFF
        if self.on_event:
            self.on_event(dict(score=self.score, prune=self.prune, t_min=t_min, cap=cap,
                               threshold=thr))
        rec = dict(event=event, n_in=n, cap=cap, threshold=thr, n_out=n)
        self.events.append(rec)
        if c.prune_threshold is not None:
            if cap == 0:
                thr = 0xFFFFFFFF
            _lib.gs_densify_prune_plan(self.score, self.p['log_scales'], n, thr, c.split_scale,
                                       self.prune, c.prune_threshold, self.ws, self.n_out)
        elif thr == 0xFFFFFFFF or cap == 0:
            return
        else:
            _lib.gs_densify_plan(self.score, self.p['log_scales'], n, thr, c.split_scale,
                                 self.ws, self.n_out)
        n_out = int(self.n_out.item()) & 0xFFFFFFFF
        if n_out == 0:      # everything pruned: keep the current set
            return
        rec['n_out'] = n_out
        if n_out == n and c.prune_threshold is None:
            return
        eps = torch.randn((2, 3, n), generator=self.gen, device='cuda')
        deg = c.sh_degree
        new_p = _alloc_like(self.p, n_out)
        _lib.gs_densify_apply(_lib.gaussians(*[self.p[k] for k in PARAM_NAMES]), n, deg, eps,
                              self.ws, n_out, False,
                              _lib.gaussians(*[new_p[k] for k in PARAM_NAMES]))
        new_m, new_v = _alloc_like(self.p, n_out), _alloc_like(self.p, n_out)
        for old, new in ((self.adam.m, new_m), (self.adam.v, new_v)):
            _lib.gs_densify_apply(_lib.gaussians(*[old[k] for k in PARAM_NAMES]), n, deg, None,
                                  self.ws, n_out, True,
                                  _lib.gaussians(*[new[k] for k in PARAM_NAMES]))
        self.p = new_p
        self.adam.params, self.adam.m, self.adam.v = new_p, new_m, new_v
        cap_pairs = int(R.capacity * n_out / n) + 4096
        self.n = n_out
        self._setup(n_out, capacity=cap_pairs)

    # -- evaluation -----------------------------------------------------------
    def evaluate(self):
        vals = []
        for v in self.test:
            self.R.cam = self.gcams[v]
            self.R.forward(self.p, check_overflow=True)
            vals.append(psnr(self.R.image.cpu().numpy(), self.gt_img[v].cpu().numpy()))
        return float(np.mean(vals))

    def run(self):
        """Train for cfg.steps; returns the timing and quality summary."""
        c = self.cfg
        psnr0 = self.evaluate()
        order = []
        event = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dens_s = 0.0
        for s in range(1, c.steps + 1):
            if not order:
                order = list(self.rng.permutation(self.train))
            self.step(s, int(order.pop()))
            if c.densify_from <= s <= c.densify_until and \
                    (s - c.densify_from) % c.densify_every == 0:
                event += 1
                torch.cuda.synchronize()
                td = time.perf_counter()
                self.densify(event)
                torch.cuda.synchronize()
                dens_s += time.perf_counter() - td
                self.log(f'[densify] step {s}: event {event}, {self.events[-1]["n_in"]} -> '
                         f'{self.n} Gaussians (threshold {self.events[-1]["threshold"]})')
            if s % 500 == 0:
                self.log(f'[densify] step {s}: {time.perf_counter() - t0:.1f} s, {self.n} Gaussians')
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return dict(train_seconds=round(wall, 3), densify_seconds=round(dens_s, 3),
                    steps=c.steps, gaussians_init=c.init_gaussians, gaussians_final=self.n,
                    psnr_init=round(psnr0, 3), psnr_final=round(self.evaluate(), 3),
                    gt_render_seconds=round(self.gt_seconds, 3), events=self.events)
