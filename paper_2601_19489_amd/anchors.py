"""Anchor (neural-Gaussian) decoder over the libgs C ABI (Sec. 2.3).

The anchors carry learnable features; one shared MLP (three heads) infers
the attributes of each anchor's 10 child Gaussians for the current camera,
and the children are rendered in direct mode (activated attributes). The
forward and backward are libgs entry points (BF16 matrix cores, FP32
accumulation); PyTorch only provides memory and the stream.
"""
from __future__ import annotations

import torch

from . import _lib

ANCHOR_NAMES = ('feat', 'pos', 'offsets', 'scaling')
MLP_NAMES = ('w1', 'b1', 'w2', 'b2')
CHILD_NAMES = ('means', 'log_scales', 'quats', 'opacity_logits', 'sh')  # direct-mode layout


def to_device(d, names, device='cuda'):
    return {k: torch.as_tensor(d[k]).to(device=device, dtype=torch.float32).contiguous()
            for k in names}


class AnchorDecoder:
    """Buffers and calls of the decoder for a fixed anchor count."""

    def __init__(self, n_anchors: int, device='cuda'):
        self.A = int(n_anchors)
        self.N = self.A * _lib.ANCHOR_CHILDREN
        self.device = torch.device(device)
        dev = self.device
        N = self.N
        self.children = dict(means=torch.empty((3, N), device=dev),
                             log_scales=torch.empty((3, N), device=dev),
                             quats=torch.empty((4, N), device=dev),
                             opacity_logits=torch.empty(N, device=dev),
                             sh=torch.empty((3, N), device=dev))
        self.workspace = torch.empty(max(_lib.gs_anchor_decode_workspace(self.A), 4),
                                     dtype=torch.uint8, device=dev)

    @staticmethod
    def _a(a):
        return _lib.anchors(a['feat'], a['pos'], a['offsets'], a['scaling'])

    @staticmethod
    def _m(m):
        return _lib.mlp(m['w1'], m['b1'], m['w2'], m['b2'])

    def decode(self, anchors, mlp, cam: _lib.GsCamera):
        c = self.children
        _lib.gs_anchor_decode_fwd(self._a(anchors), self.A, self._m(mlp), cam,
                                  _lib.gaussians(*(c[k] for k in CHILD_NAMES)))
        return c

    def backward(self, anchors, mlp, cam: _lib.GsCamera, dchild, danchors=None, dmlp=None,
                 accumulate=False):
        if danchors is None:
            danchors = {k: torch.empty_like(anchors[k]) for k in ('feat', 'offsets', 'scaling')}
        if dmlp is None:
            dmlp = {k: torch.empty_like(mlp[k]) for k in MLP_NAMES}
        da = _lib.GsAnchors()
        da.feat = _lib._ptr(danchors.get('feat'))
        da.offsets = _lib._ptr(danchors.get('offsets'))
        da.scaling = _lib._ptr(danchors.get('scaling'))
        dc = _lib.gaussians(*(dchild[k].contiguous() for k in CHILD_NAMES))
        _lib.gs_anchor_decode_bwd(self._a(anchors), self.A, self._m(mlp), cam, dc, da,
                                  self._m(dmlp), self.workspace, accumulate)
        return danchors, dmlp
