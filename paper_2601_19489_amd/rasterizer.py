"""Rasterizer pipeline over the libgs C ABI, and its torch.autograd.Function.

PyTorch provides device memory and the stream; each step below is one or
more libgs entry points:
    preprocess -> bin_sort -> render_fwd      (forward, Sec. 2.1)
    render_bwd (image-space + per-Gaussian)   (backward, Sec. 2.2)
    adam_step                                  (optimiser)
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import torch

from . import _lib

PARAM_NAMES = ('means', 'log_scales', 'quats', 'opacity_logits', 'sh')


def params_to_device(d, device='cuda'):
    """Dict of contiguous float32 device tensors from a scene dict."""
    return {k: torch.as_tensor(d[k]).to(device=device, dtype=torch.float32).contiguous()
            for k in PARAM_NAMES}


def _gs(p) -> _lib.GsGaussians:
    return _lib.gaussians(p['means'], p['log_scales'], p['quats'], p['opacity_logits'], p['sh'])


@dataclasses.dataclass
class Frame:
    """Forward state of one view (what the backward needs)."""
    splats: torch.Tensor
    depth_keys: torch.Tensor
    tile_counts: torch.Tensor
    vals: torch.Tensor
    ranges: torch.Tensor
    pair_count: torch.Tensor
    image: torch.Tensor
    depth: torch.Tensor
    T_final: torch.Tensor
    n_contrib: torch.Tensor


class Rasterizer:
    """Buffers and calls for one camera and a fixed Gaussian count.

    The pair buffers are sized to a capacity with headroom; `forward`
    checks the device pair count and re-runs the binning with a larger
    capacity when it overflowed (one small device-to-host read per call
    unless check_overflow=False).

    With deferred=True the binning stops short of writing the tile lists
    (gs_bin_sort_deferred) and the forward writes each tile's list only as
    far as its compositing reaches (gs_render_fwd_deferred): the same
    images, and `vals` holds every position the backward reads, but not the
    rest of the lists (bin_sort with keys_out writes them all).

    The buffers hold the state of the last forward only. `generation`
    counts the forward steps run on them, so a caller can tell whether the
    state it wants to differentiate is still there; `frame()` copies it.
    """

    def __init__(self, n: int, cam, sh_degree: int, bg: Sequence[float] = (0.0, 0.0, 0.0),
                 tile: Optional[int] = None, capacity: int = 0, headroom: float = 1.25,
                 device='cuda', deferred: bool = False):
        self.n = int(n)
        self.deferred = bool(deferred)
        self.cam = _lib.camera(cam, tile)
        self.sh_degree = int(sh_degree)
        self.bg = tuple(float(x) for x in bg)
        self.headroom = headroom
        self.device = torch.device(device)
        W, H, T = self.cam.width, self.cam.height, self.cam.tile
        self.tiles_x = -(-W // T)
        self.tiles_y = -(-H // T)
        self.n_tiles = self.tiles_x * self.tiles_y
        dev = self.device
        self.splats = torch.empty((self.n, _lib.SPLAT_FLOATS), device=dev)
        self.depth_keys = torch.empty(self.n, dtype=torch.int32, device=dev)
        self.tile_counts = torch.empty(self.n, dtype=torch.int32, device=dev)
        self.ranges = torch.empty(self.n_tiles + 1, dtype=torch.int32, device=dev)
        self.pair_count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.image = torch.empty((3, H, W), device=dev)
        self.depth = torch.empty((H, W), device=dev)
        self.T_final = torch.empty((H, W), device=dev)
        self.n_contrib = torch.empty((H, W), dtype=torch.int32, device=dev)
        # one 10-double record per splat: grad2d[i] = dL/d(u, v, a, b, c, o, r, g, b, z)
        self.grad2d = torch.empty((self.n, _lib.GRAD2D_COMPONENTS), dtype=torch.float64, device=dev)
        # backward tile schedule (heaviest tiles first); None keeps tile-id order
        self.tile_order = torch.empty(2 * self.n_tiles, dtype=torch.int32, device=dev)
        self.capacity = 0
        self.vals = None
        self.workspace = None
        self.keys_out = None
        self.generation = 0
        self.pairs = None      # pair count of the last checked binning
        self._alloc_pairs(max(int(capacity), 1))

    def _alloc_pairs(self, capacity):
        self.capacity = int(capacity)
        self.vals = torch.empty(self.capacity, dtype=torch.int32, device=self.device)
        wb = _lib.gs_bin_sort_workspace(self.n, self.capacity, self.cam)
        self.workspace = torch.empty(wb, dtype=torch.uint8, device=self.device)

    # -- forward steps -------------------------------------------------
    def preprocess(self, p):
        self.generation += 1
        _lib.gs_preprocess(_gs(p), self.n, self.sh_degree, self.cam, self.splats, self.depth_keys,
                           self.tile_counts)

    def _bin(self, keys_out):
        if self.deferred and keys_out is None:
            _lib.gs_bin_sort_deferred(self.splats, self.depth_keys, self.tile_counts, self.n,
                                      self.cam, self.workspace, self.capacity, self.ranges,
                                      self.pair_count)
        else:
            _lib.gs_bin_sort(self.splats, self.depth_keys, self.tile_counts, self.n, self.cam,
                             self.workspace, self.capacity, self.vals, self.ranges, keys_out,
                             self.pair_count)

    def bin_sort(self, keys_out: Optional[torch.Tensor] = None, check_overflow: bool = True):
        self.generation += 1
        self.pairs = None
        self._bin(keys_out)
        if check_overflow:
            P = int(self.pair_count.item()) & 0xFFFFFFFF
            if P > self.capacity:
                self._alloc_pairs(int(P * self.headroom) + 1024)
                self._bin(keys_out)
            self.pairs = P
            return P
        return None

    def render_fwd(self):
        self.generation += 1
        if self.deferred:
            _lib.gs_render_fwd_deferred(self.splats, self.n, self.workspace, self.capacity,
                                        self.vals, self.ranges, self.cam, self.bg, self.image,
                                        self.depth, self.T_final, self.n_contrib)
        else:
            _lib.gs_render_fwd(self.splats, self.n, self.vals, self.ranges, self.cam, self.bg,
                               self.image, self.depth, self.T_final, self.n_contrib)

    def forward(self, p, check_overflow: bool = True):
        self.preprocess(p)
        self.bin_sort(check_overflow=check_overflow)
        self.render_fwd()
        return self.image, self.depth

    def frame(self) -> Frame:
        """Copy of the forward state the backward reads (device tensors)."""
        vals = self.vals if self.pairs is None else self.vals[:max(self.pairs, 1)]
        return Frame(*(t.clone() for t in (self.splats, self.depth_keys, self.tile_counts, vals,
                                           self.ranges, self.pair_count, self.image, self.depth,
                                           self.T_final, self.n_contrib)))

    # -- backward --------------------------------------------------------
    def backward(self, p, dL_dimage, dL_ddepth=None, grads=None, accumulate=False,
                 frame: Optional[Frame] = None):
        """Gradients of the last forward (or of `frame`, a copy from frame())."""
        if grads is None:
            grads = {k: torch.empty_like(v) for k, v in p.items()}
        f = self if frame is None else frame
        _lib.gs_render_bwd(_gs(p), self.n, self.sh_degree, self.cam, f.splats, f.vals,
                           f.ranges, self.bg, f.T_final, f.n_contrib,
                           dL_dimage.contiguous(),
                           None if dL_ddepth is None else dL_ddepth.contiguous(), self.grad2d,
                           _gs(grads), accumulate, tile_order=self.tile_order)
        return grads

    def backward_adam(self, p, dL_dimage, opt: 'Adam', dL_ddepth=None):
        """The backward of the last forward fused with one step of `opt`:
        the parameters in p and opt's moments are updated in place, as
        backward() followed by opt.step() would, without writing gradients."""
        _lib.gs_render_bwd_adam(_gs(p), self.n, self.sh_degree, self.cam, self.splats, self.vals,
                                self.ranges, self.bg, self.T_final, self.n_contrib,
                                dL_dimage.contiguous(),
                                None if dL_ddepth is None else dL_ddepth.contiguous(),
                                self.grad2d, opt.fused_params(), tile_order=self.tile_order)


def l1_loss(image, target, dL_dimage=None, loss=None):
    """Mean |image - target| (device scalar) and its gradient, in libgs."""
    if dL_dimage is None:
        dL_dimage = torch.empty_like(image)
    if loss is None:
        loss = torch.zeros(1, device=image.device)
    else:
        loss.zero_()
    _lib.gs_l1_loss(image, target, image.numel(), dL_dimage, loss)
    return loss, dL_dimage


class Adam:
    """Adam over the Gaussian parameter groups (one learning rate each) in one
    launch (gs_adam_step_grouped); the step count lives on the device."""

    def __init__(self, params, lrs, betas=(0.9, 0.999), eps=1e-15):
        self.params = params
        self.lrs = dict(lrs)
        self.b1, self.b2 = betas
        self.eps = eps
        self.m = {k: torch.zeros_like(v) for k, v in params.items()}
        self.v = {k: torch.zeros_like(v) for k, v in params.items()}
        dev = next(iter(params.values())).device
        self.step_count = torch.zeros(1, dtype=torch.int32, device=dev)

    def fused_params(self) -> _lib.GsAdamParams:
        """The state as gs_render_bwd_adam takes it (the parameter groups
        must be the five Gaussian arrays)."""
        if tuple(self.params) != PARAM_NAMES:
            raise ValueError(f'the fused step needs the groups {PARAM_NAMES}')
        return _lib.adam_params(_gs(self.m), _gs(self.v), [self.lrs[k] for k in PARAM_NAMES],
                                self.b1, self.b2, self.eps, self.step_count)

    def step(self, grads):
        _lib.gs_adam_step_grouped(
            [(p, grads[k], self.m[k], self.v[k], self.lrs[k]) for k, p in self.params.items()],
            self.b1, self.b2, self.eps, self.step_count)


class StaleFrameError(RuntimeError):
    """The rasterizer ran another forward step after the one being
    differentiated, so the state that backward needs is gone."""


class GaussianRasterizer(torch.autograd.Function):
    """Differentiable render of one view.

    forward(means, log_scales, quats, opacity_logits, sh, raster, keep_frame)
    -> (image [3,H,W], depth [H,W]). The backward recomputes per-pixel
    transmittance from the stored final transmittance (no per-splat state is
    saved) and returns gradients for the five parameter tensors.

    The forward state (splats, sorted lists, T_final, n_contrib) lives in the
    Rasterizer's buffers. With keep_frame=False the backward uses them in
    place and raises StaleFrameError if the Rasterizer has run any forward
    step since; with keep_frame=True the forward copies them (device memory
    of about 48 B per Gaussian, 4 B per pair and 8 B per pixel), so several
    forwards on one Rasterizer can be differentiated in any order.
    """

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, raster: Rasterizer,
                keep_frame: bool = False):
        p = dict(means=means.contiguous(), log_scales=log_scales.contiguous(),
                 quats=quats.contiguous(), opacity_logits=opacity_logits.contiguous(),
                 sh=sh.contiguous())
        image, depth = raster.forward(p)
        ctx.raster = raster
        ctx.save_for_backward(*[p[k] for k in PARAM_NAMES])
        ctx.generation = raster.generation
        ctx.frame = raster.frame() if keep_frame else None
        return image.clone(), depth.clone()

    @staticmethod
    def backward(ctx, dL_dimage, dL_ddepth):
        raster: Rasterizer = ctx.raster
        if ctx.frame is None and raster.generation != ctx.generation:
            raise StaleFrameError(
                'the rasterizer ran another forward after this one; differentiate before the '
                'next forward or pass keep_frame=True')
        p = dict(zip(PARAM_NAMES, ctx.saved_tensors))
        if dL_dimage is None:
            dL_dimage = torch.zeros_like(raster.image)
        grads = raster.backward(p, dL_dimage, dL_ddepth, frame=ctx.frame)
        return tuple(grads[k] for k in PARAM_NAMES) + (None, None)


def rasterize(means, log_scales, quats, opacity_logits, sh, raster: Rasterizer,
              keep_frame: bool = False):
    return GaussianRasterizer.apply(means, log_scales, quats, opacity_logits, sh, raster,
                                    keep_frame)
