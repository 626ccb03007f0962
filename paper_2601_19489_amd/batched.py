"""Batched multi-view training step over the libgs C ABI, its hipGraph
capture, and the autotuner of the launch knobs.

A minibatch of views (cameras of mixed resolutions, one set of Gaussians)
is rendered and differentiated with one launch per phase where the library
offers it: one preprocess launch for all views, the binning per view, one
persistent forward launch and one persistent backward launch over the
(view, tile) queue of all views, the per-view L1 losses, and one Adam launch
over all parameter groups with a device-side step count. The whole step has
no host synchronisation, so it can be captured once into a HIP graph
(torch.cuda.CUDAGraph) and replayed.
"""
from __future__ import annotations

import time
from typing import Dict, Optional, Sequence

import torch

from . import _lib
from .rasterizer import PARAM_NAMES


def _gs(p) -> _lib.GsGaussians:
    return _lib.gaussians(*(p[k] for k in PARAM_NAMES))


class BatchedRasterizer:
    """Per-view buffers and the batched calls for a fixed Gaussian count.

    deferred=True: the deferred binning (each view keeps its own workspace
    until the forward, which writes each tile's list only as far as it
    composites; the same results as the full lists)."""

    def __init__(self, n: int, cams: Sequence, sh_degree: int, tile: int = 16,
                 bg=(0.0, 0.0, 0.0), headroom: float = 1.25, device='cuda',
                 deferred: bool = False):
        if not 1 <= len(cams) <= _lib.MAX_VIEWS:
            raise ValueError(f'1..{_lib.MAX_VIEWS} views per batch')
        self.n = int(n)
        self.sh_degree = int(sh_degree)
        self.bg = tuple(float(x) for x in bg)
        self.headroom = headroom
        self.dev = torch.device(device)
        self.cams = [_lib.camera(c, tile) for c in cams]
        self.V = len(cams)
        dev = self.dev
        self.buf = []
        for c in self.cams:
            W, H, T = c.width, c.height, c.tile
            nt = (-(-W // T)) * (-(-H // T))
            self.buf.append(dict(
                splats=torch.empty((self.n, _lib.SPLAT_FLOATS), device=dev),
                depth_keys=torch.empty(self.n, dtype=torch.int32, device=dev),
                tile_counts=torch.empty(self.n, dtype=torch.int32, device=dev),
                vals=torch.empty(1, dtype=torch.int32, device=dev),
                ranges=torch.empty(nt + 1, dtype=torch.int32, device=dev),
                pair_count=torch.zeros(1, dtype=torch.int32, device=dev),
                image=torch.empty((3, H, W), device=dev),
                depth=torch.empty((H, W), device=dev),
                T_final=torch.empty((H, W), device=dev),
                n_contrib=torch.empty((H, W), dtype=torch.int32, device=dev),
                dL_dimage=torch.zeros((3, H, W), device=dev),
                grad2d=torch.empty((self.n, _lib.GRAD2D_COMPONENTS), dtype=torch.float64,
                                   device=dev),
                capacity=1))
        self.queue = torch.zeros(1, dtype=torch.int32, device=dev)
        # backward schedule over the (view, tile) items, heaviest first; None: queue order
        items = sum(b['ranges'].numel() - 1 for b in self.buf)
        self.tile_order = torch.empty(2 * items, dtype=torch.int32, device=dev)
        self.workspace = None
        self.workspaces = None  # deferred: one per view
        self.deferred = bool(deferred)
        self._views = None

    # -- buffers ---------------------------------------------------------
    def views(self):
        if self._views is None:
            vs = []
            for c, b in zip(self.cams, self.buf):
                v = _lib.GsView()
                v.cam = c
                for k in ('splats', 'depth_keys', 'tile_counts', 'vals', 'ranges', 'pair_count',
                          'image', 'depth', 'T_final', 'n_contrib', 'dL_dimage', 'grad2d'):
                    setattr(v, k, _lib._ptr(b[k]))
                v.keys_out = None
                v.dL_ddepth = None
                v.capacity = b['capacity']
                vs.append(v)
            self._views = vs
        return self._views

    def size_pairs(self, p):
        """Size every view's pair buffer from one binning pass (host read)."""
        _lib.gs_preprocess_batched(_gs(p), self.n, self.sh_degree, self.views())
        counts = [int(b['tile_counts'].to(torch.int64).sum().item()) for b in self.buf]
        for b, P in zip(self.buf, counts):
            b['capacity'] = int(P * self.headroom) + 4096
            b['vals'] = torch.empty(b['capacity'], dtype=torch.int32, device=self.dev)
        self._views = None
        if self.deferred:
            self.workspaces = [
                torch.empty(max(_lib.gs_bin_sort_workspace(self.n, b['capacity'], c), 16),
                            dtype=torch.uint8, device=self.dev)
                for c, b in zip(self.cams, self.buf)]
        else:
            wb = _lib.gs_bin_sort_batched_workspace(self.n, self.views())
            self.workspace = torch.empty(max(wb, 16), dtype=torch.uint8, device=self.dev)
        return counts

    # -- phases ----------------------------------------------------------
    def forward(self, p):
        vs = self.views()
        _lib.gs_preprocess_batched(_gs(p), self.n, self.sh_degree, vs)
        if self.deferred:
            _lib.gs_bin_sort_batched_deferred(self.n, vs, self.workspaces)
            _lib.gs_render_fwd_batched_deferred(self.n, vs, self.workspaces, self.bg, self.queue)
        else:
            _lib.gs_bin_sort_batched(self.n, vs, self.workspace)
            _lib.gs_render_fwd_batched(self.n, vs, self.bg, self.queue)

    def l1_losses(self, targets, loss):
        """Sum over views of each view's mean L1 (added to loss[0]); the
        image gradients land in the per-view dL_dimage buffers."""
        for b, t in zip(self.buf, targets):
            _lib.gs_l1_loss(b['image'], t, b['image'].numel(), b['dL_dimage'], loss)

    def backward(self, p, grads, accumulate=False):
        _lib.gs_render_bwd_batched(_gs(p), self.n, self.sh_degree, self.views(), self.bg,
                                   self.queue, _gs(grads), accumulate, tile_order=self.tile_order)

    def pair_counts(self):
        return [int(b['pair_count'].item()) & 0xFFFFFFFF for b in self.buf]


class TrainStep:
    """fwd + per-view L1 + bwd + grouped Adam over a view batch; eager or
    replayed from a captured HIP graph."""

    def __init__(self, raster: BatchedRasterizer, params: Dict[str, torch.Tensor], targets,
                 lrs: Dict[str, float], betas=(0.9, 0.999), eps=1e-15):
        self.r = raster
        self.p = params
        self.targets = [t.contiguous() for t in targets]
        self.lrs = dict(lrs)
        self.b1, self.b2 = betas
        self.eps = eps
        self.grads = {k: torch.empty_like(v) for k, v in params.items()}
        self.m = {k: torch.zeros_like(v) for k, v in params.items()}
        self.v = {k: torch.zeros_like(v) for k, v in params.items()}
        self.step_count = torch.zeros(1, dtype=torch.int32, device=raster.dev)
        self.loss = torch.zeros(1, device=raster.dev)
        self.max_pairs = torch.zeros(raster.V, dtype=torch.int64, device=raster.dev)
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    def _groups(self):
        return [(self.p[k], self.grads[k], self.m[k], self.v[k], self.lrs[k]) for k in PARAM_NAMES]

    def run(self):
        """One eager step (no host synchronisation)."""
        self.loss.zero_()
        self.r.forward(self.p)
        self.r.l1_losses(self.targets, self.loss)
        self.r.backward(self.p, self.grads)
        _lib.gs_adam_step_grouped(self._groups(), self.b1, self.b2, self.eps, self.step_count)
        for v, b in enumerate(self.r.buf):
            mp = self.max_pairs[v:v + 1]
            torch.maximum(mp, b['pair_count'].to(torch.int64), out=mp)

    def capture(self):
        """Record one step into a HIP graph (nothing executes while
        recording). Launch timing must be off."""
        _lib.gs_timer_enable(None)
        self.graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(self.graph):
            self.run()
        return self.graph

    def replay(self):
        self.graph.replay()

    def check_capacity(self):
        """Largest pair count seen per view against its capacity (host read)."""
        mps = self.max_pairs.tolist()
        for v, (mp, b) in enumerate(zip(mps, self.r.buf)):
            if mp > b['capacity']:
                raise RuntimeError(f'pair capacity overflow in view {v}: {mp} > {b["capacity"]}')
        return max(mps)


def autotune(make_step, tiles=(8, 16, 32), px=(1, 2, 4), persist=(8, 12, 16),
             fwd_batch=(64, 128, 256), bwd_batch=(32, 64, 128), warmup=2, iters=5, log=None):
    """Pick tile size, pixels per lane (forward, backward), persistent
    workgroups per CU and the splats per LDS batch (forward batch, backward
    bucket) by timing the batched step, one knob at a time.

    make_step(tile) returns a ready TrainStep for that tile size. Returns
    (best config dict, list of (config, ms per step)). The knobs do not
    change results, only speed (the tile size changes the binning, whose
    lists are checked against the oracle at every size).
    """
    table = []

    def measure(tile, cfg):
        _lib.gs_set_tuning(**cfg)
        st = make_step(tile)
        for _ in range(warmup):
            st.run()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(iters):
            st.run()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / iters
        st.check_capacity()
        table.append((dict(tile=tile, **cfg), ms))
        if log:
            log(f'[autotune] tile {tile} {cfg}: {ms:.3f} ms')
        del st
        return ms

    cfg = dict(fwd_px=1, bwd_px=4, persist_wgs=12, fwd_batch=0, bwd_batch=0)
    best_tile, best_ms = None, float('inf')
    for t in tiles:
        c = dict(cfg)
        if t == 8:
            c.update(fwd_px=1, bwd_px=1)
        elif t == 32:
            c.update(bwd_px=max(2, c['bwd_px']))
        ms = measure(t, c)
        if ms < best_ms:
            best_tile, best_ms, cfg = t, ms, c
    if best_tile != 8:
        for knob in ('fwd_px', 'bwd_px'):
            for v in px:
                if v == cfg[knob] or (knob == 'bwd_px' and best_tile == 32 and v < 2):
                    continue
                c = dict(cfg, **{knob: v})
                ms = measure(best_tile, c)
                if ms < best_ms:
                    best_ms, cfg = ms, c
    for v in persist:
        if v == cfg['persist_wgs']:
            continue
        c = dict(cfg, persist_wgs=v)
        ms = measure(best_tile, c)
        if ms < best_ms:
            best_ms, cfg = ms, c
    for knob, values in (('fwd_batch', fwd_batch), ('bwd_batch', bwd_batch)):
        for v in values:
            if v == cfg[knob]:
                continue
            c = dict(cfg, **{knob: v})
            ms = measure(best_tile, c)
            if ms < best_ms:
                best_ms, cfg = ms, c
    _lib.gs_set_tuning(**cfg)
    return dict(tile=best_tile, **cfg), table
