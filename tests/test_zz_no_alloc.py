"""The allocation-free decoder backward (gs_anchor_decode_bwd_noalloc)
against the workspace entry point (gs_anchor_decode_bwd), through the C ABI.

Both run the same kernels in the same order on the same inputs, so their
outputs are compared bit for bit. The allocation-free calls come two in a
row, the second with fewer anchors (a smaller grid, so the library's array
still holds more of the first call's partial sums than the second writes),
then once with no anchors.
"""
import numpy as np
import pytest
import torch

from paper_2601_19489_amd import _lib, scenes
from paper_2601_19489_amd.anchors import ANCHOR_NAMES, CHILD_NAMES, MLP_NAMES, AnchorDecoder, to_device

pytestmark = pytest.mark.gpu

CASES = ((100_000, 4, 0), (777, 5, 1), (0, 6, 0))   # (anchors, seed, accumulate)


def _prepare(A, seed):
    a = scenes.anchor_cloud(max(A, 1), seed=seed)
    if A == 0:
        a = {k: v[:, :0].copy() for k, v in a.items()}
    m = scenes.decoder_mlp(seed=seed + 10)
    cam = _lib.camera(scenes.look_at_camera((-0.4, 0.2, -3.5), (0, 0, 0), 320, 240))
    ad, md = to_device(a, ANCHOR_NAMES), to_device(m, MLP_NAMES)
    dec = AnchorDecoder(A)
    dec.decode(ad, md, cam)
    rng = np.random.default_rng(seed + 100)
    dchild = {k: torch.as_tensor(rng.standard_normal(v.shape).astype(np.float32), device='cuda')
              for k, v in dec.children.items()}
    return dec, ad, md, cam, dchild


def _outputs(ad, md):
    # non-zero starting values, so that accumulate = 1 is visible
    da = {k: torch.full_like(ad[k], 0.5) for k in ('feat', 'offsets', 'scaling')}
    dm = {k: torch.full_like(md[k], 0.25) for k in MLP_NAMES}
    return da, dm


def _structs(dec, ad, md, dchild, da, dm):
    g = _lib.GsAnchors()
    g.feat, g.offsets, g.scaling = (_lib._ptr(da[k]) for k in ('feat', 'offsets', 'scaling'))
    return (dec._a(ad), dec._m(md), _lib.gaussians(*(dchild[k] for k in CHILD_NAMES)), g,
            dec._m(dm))


def test_noalloc_backward_equals_workspace_backward():
    prepared = [_prepare(A, seed) for A, seed, _ in CASES]
    got = []
    for (A, _, acc), (dec, ad, md, cam, dchild) in zip(CASES, prepared):
        da, dm = _outputs(ad, md)
        a, m, dc, g, gm = _structs(dec, ad, md, dchild, da, dm)
        _lib.gs_anchor_decode_bwd_noalloc(a, A, m, cam, dc, g, gm, acc)
        got.append({**da, **dm})
    torch.cuda.synchronize()
    for (A, _, acc), (dec, ad, md, cam, dchild), res in zip(CASES, prepared, got):
        da, dm = _outputs(ad, md)
        a, m, dc, g, gm = _structs(dec, ad, md, dchild, da, dm)
        _lib.gs_anchor_decode_bwd(a, A, m, cam, dc, g, gm, dec.workspace, acc)
        torch.cuda.synchronize()
        for k, v in {**da, **dm}.items():
            assert torch.equal(res[k], v), (A, k)
        if A == 0:   # weight gradients written as zero, nothing else touched
            assert all(torch.count_nonzero(dm[k]) == 0 for k in MLP_NAMES)
        else:
            assert all(torch.count_nonzero(v - 0.25 * acc) > 0 for v in dm.values())


def test_noalloc_rejects_bad_arguments():
    dec, ad, md, cam, dchild = _prepare(10, 7)
    da, dm = _outputs(ad, md)
    a, m, dc, g, gm = _structs(dec, ad, md, dchild, da, dm)
    # checked on the host before anything is launched
    for A in (-1, (1 << 28) + 1):
        with pytest.raises(RuntimeError, match='invalid argument'):
            _lib.gs_anchor_decode_bwd_noalloc(a, A, m, cam, dc, g, gm)
    with pytest.raises(RuntimeError, match='invalid argument'):   # no weight-gradient outputs
        _lib.gs_anchor_decode_bwd_noalloc(a, 10, m, cam, dc, g, _lib.GsMlp())
    assert _lib.lib().gs_anchor_decode_bwd_noalloc(a, 10, m, cam, dc, g, gm, 2, None) == \
        _lib.GS_EINVAL                                             # accumulate must be 0 or 1
