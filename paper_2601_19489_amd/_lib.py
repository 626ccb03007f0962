"""ctypes binding of libgs (include/gs.h): argument marshalling only.

Every function here has the name of a C entry point and forwards torch
device tensors as raw pointers together with the current HIP stream; all
computation happens in the HIP kernels. 32-bit unsigned arrays travel as
torch.int32 tensors (same bits), 64-bit keys as torch.int64.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libgs.so')

SPLAT_FLOATS = 12
GRAD2D_COMPONENTS = 10

GS_OK, GS_EINVAL, GS_ECAPACITY, GS_EHIP = 0, 1, 2, 3
_STATUS = {GS_EINVAL: 'invalid argument', GS_ECAPACITY: 'workspace too small',
           GS_EHIP: 'HIP launch failure'}


class GsCamera(ctypes.Structure):
    _fields_ = [('width', ctypes.c_int32), ('height', ctypes.c_int32), ('tile', ctypes.c_int32),
                ('depth_mode', ctypes.c_int32), ('fx', ctypes.c_double), ('fy', ctypes.c_double),
                ('cx', ctypes.c_double), ('cy', ctypes.c_double), ('R', ctypes.c_double * 9),
                ('t', ctypes.c_double * 3), ('near_plane', ctypes.c_double)]


class GsTuning(ctypes.Structure):
    _fields_ = [('fwd_px', ctypes.c_int32), ('bwd_px', ctypes.c_int32),
                ('persist_wgs', ctypes.c_int32), ('seq_walk', ctypes.c_int32),
                ('fwd_batch', ctypes.c_int32), ('bwd_batch', ctypes.c_int32),
                ('reserved', ctypes.c_int32 * 2)]


class GsGaussians(ctypes.Structure):
    _fields_ = [('means', ctypes.c_void_p), ('log_scales', ctypes.c_void_p),
                ('quats', ctypes.c_void_p), ('opacity_logits', ctypes.c_void_p),
                ('sh', ctypes.c_void_p)]


class GsAnchors(ctypes.Structure):
    _fields_ = [('feat', ctypes.c_void_p), ('pos', ctypes.c_void_p),
                ('offsets', ctypes.c_void_p), ('scaling', ctypes.c_void_p)]


class GsMlp(ctypes.Structure):
    _fields_ = [('w1', ctypes.c_void_p), ('b1', ctypes.c_void_p), ('w2', ctypes.c_void_p),
                ('b2', ctypes.c_void_p)]


class GsView(ctypes.Structure):
    _fields_ = [('cam', GsCamera), ('splats', ctypes.c_void_p), ('depth_keys', ctypes.c_void_p),
                ('tile_counts', ctypes.c_void_p), ('vals', ctypes.c_void_p),
                ('ranges', ctypes.c_void_p), ('pair_count', ctypes.c_void_p),
                ('keys_out', ctypes.c_void_p), ('capacity', ctypes.c_int64),
                ('image', ctypes.c_void_p), ('depth', ctypes.c_void_p),
                ('T_final', ctypes.c_void_p), ('n_contrib', ctypes.c_void_p),
                ('dL_dimage', ctypes.c_void_p), ('dL_ddepth', ctypes.c_void_p),
                ('grad2d', ctypes.c_void_p)]


class GsAdamGroup(ctypes.Structure):
    _fields_ = [('p', ctypes.c_void_p), ('g', ctypes.c_void_p), ('m', ctypes.c_void_p),
                ('v', ctypes.c_void_p), ('n', ctypes.c_int64), ('lr', ctypes.c_float),
                ('reserved', ctypes.c_int32)]


class GsAdamParams(ctypes.Structure):
    _fields_ = [('m', GsGaussians), ('v', GsGaussians), ('lr', ctypes.c_float * 5),
                ('beta1', ctypes.c_float), ('beta2', ctypes.c_float), ('eps', ctypes.c_float),
                ('step', ctypes.c_void_p)]


MAX_VIEWS = 8
DEPTH_Z = 0
DEPTH_INVERSE = 1
SCORE_BINS = 65536
MAX_ADAM_GROUPS = 8
GS_DIRECT = -1
ANCHOR_CHILDREN = 10
ANCHOR_FEAT = 32

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_F = ctypes.c_float
_SIGS = {
    'gs_preprocess': [ctypes.POINTER(GsGaussians), _I64, _I32, ctypes.POINTER(GsCamera), _P, _P, _P, _P],
    'gs_bin_sort_workspace': [_I64, _I64, ctypes.POINTER(GsCamera), ctypes.POINTER(ctypes.c_size_t)],
    'gs_bin_sort': [_P, _P, _P, _I64, ctypes.POINTER(GsCamera), _P, ctypes.c_size_t, _I64, _P, _P,
                    _P, _P, _P],
    'gs_render_fwd': [_P, _I64, _P, _P, ctypes.POINTER(GsCamera), ctypes.POINTER(_F), _P, _P, _P, _P, _P],
    'gs_bin_sort_deferred': [_P, _P, _P, _I64, ctypes.POINTER(GsCamera), _P, ctypes.c_size_t, _I64,
                             _P, _P, _P],
    'gs_render_fwd_deferred': [_P, _I64, _P, ctypes.c_size_t, _I64, _P, _P,
                               ctypes.POINTER(GsCamera), ctypes.POINTER(_F), _P, _P, _P, _P, _P],
    'gs_render_bwd': [ctypes.POINTER(GsGaussians), _I64, _I32, ctypes.POINTER(GsCamera), _P, _P, _P,
                      ctypes.POINTER(_F), _P, _P, _P, _P, _P, ctypes.POINTER(GsGaussians), _I32, _P,
                      _P],
    'gs_render_bwd_adam': [ctypes.POINTER(GsGaussians), _I64, _I32, ctypes.POINTER(GsCamera), _P,
                           _P, _P, ctypes.POINTER(_F), _P, _P, _P, _P, _P,
                           ctypes.POINTER(GsAdamParams), _P, _P],
    'gs_l1_loss': [_P, _P, _I64, _P, _P, _P],
    'gs_adam_step': [_P, _P, _P, _P, _I64, _F, _F, _F, _F, _I32, _P],
    'gs_anchor_decode_fwd': [ctypes.POINTER(GsAnchors), _I64, ctypes.POINTER(GsMlp),
                             ctypes.POINTER(GsCamera), ctypes.POINTER(GsGaussians), _P],
    'gs_anchor_decode_workspace': [_I64, ctypes.POINTER(ctypes.c_size_t)],
    'gs_anchor_decode_bwd': [ctypes.POINTER(GsAnchors), _I64, ctypes.POINTER(GsMlp),
                             ctypes.POINTER(GsCamera), ctypes.POINTER(GsGaussians),
                             ctypes.POINTER(GsAnchors), ctypes.POINTER(GsMlp), _P, ctypes.c_size_t,
                             _I32, _P],
    'gs_anchor_decode_bwd_noalloc': [ctypes.POINTER(GsAnchors), _I64, ctypes.POINTER(GsMlp),
                                     ctypes.POINTER(GsCamera), ctypes.POINTER(GsGaussians),
                                     ctypes.POINTER(GsAnchors), ctypes.POINTER(GsMlp), _I32, _P],
    'gs_depth_l1_loss': [_P, _P, _I64, _F, _P, _P, _P],
    'gs_error_mask': [_P, _P, _I64, _F, _P, _P, _P],
    'gs_split_score': [_P, _I64, _P, _P, ctypes.POINTER(GsCamera), _P, _P, _P],
    'gs_densify_workspace': [_I64, ctypes.POINTER(ctypes.c_size_t)],
    'gs_densify_plan': [_P, _P, _I64, ctypes.c_uint32, _F, _P, ctypes.c_size_t, _P, _P],
    'gs_densify_apply': [ctypes.POINTER(GsGaussians), _I64, _I32, _P, _P, _I64, _I32,
                         ctypes.POINTER(GsGaussians), _P],
    'gs_densify_threshold': [_P, _I64, ctypes.c_uint32, _I64, _P, _P, _P],
    'gs_densify_prune_plan': [_P, _P, _I64, ctypes.c_uint32, _F, _P, ctypes.c_double, _P,
                              ctypes.c_size_t, _P, _P],
    'gs_photo_loss_workspace': [_I32, _I32, _I32, ctypes.POINTER(ctypes.c_size_t)],
    'gs_photo_loss': [_P, _P, _I32, _I32, _I32, _F, _P, ctypes.c_size_t, _P, _P, _P],
    'gs_prune_accumulate': [_P, _I64, _P, _P, _P, _P],
    'gs_render_fwd_ckpt': [_P, _I64, _P, _P, ctypes.POINTER(GsCamera), _P, _P, _P, _P, _P, _P,
                           _I32, _P, _P],
    'gs_render_bwd_ckpt': [ctypes.POINTER(GsGaussians), _I64, _I32, ctypes.POINTER(GsCamera), _P,
                           _P, _P, _P, _P, _P, _P, _I32, _P, _P, _P, ctypes.POINTER(GsGaussians),
                           _I32, _P],
    'gs_tile_count_variant': [_P, _I64, ctypes.POINTER(GsCamera), _I32, _P, _P],
    'gs_pose_grad': [ctypes.POINTER(GsGaussians), _I64, _I32, ctypes.POINTER(GsCamera), _P, _P,
                     _P],
    'gs_preprocess_batched': [ctypes.POINTER(GsGaussians), _I64, _I32, ctypes.POINTER(GsView),
                              _I32, _P],
    'gs_bin_sort_batched_workspace': [_I64, ctypes.POINTER(GsView), _I32,
                                      ctypes.POINTER(ctypes.c_size_t)],
    'gs_bin_sort_batched': [_I64, ctypes.POINTER(GsView), _I32, _P, ctypes.c_size_t, _P],
    'gs_bin_sort_batched_deferred': [_I64, ctypes.POINTER(GsView), _I32, ctypes.POINTER(_P),
                                     ctypes.POINTER(ctypes.c_size_t), _P],
    'gs_render_fwd_batched_deferred': [_I64, ctypes.POINTER(GsView), _I32, ctypes.POINTER(_P),
                                       ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_F), _P,
                                       _P],
    'gs_render_fwd_batched': [_I64, ctypes.POINTER(GsView), _I32, ctypes.POINTER(_F), _P, _P],
    'gs_render_bwd_batched': [ctypes.POINTER(GsGaussians), _I64, _I32, ctypes.POINTER(GsView),
                              _I32, ctypes.POINTER(_F), _P, ctypes.POINTER(GsGaussians), _I32, _P,
                              _P],
    'gs_adam_step_grouped': [ctypes.POINTER(GsAdamGroup), _I32, _F, _F, _F, _P, _P],
    'gs_timer_enable': [ctypes.c_char_p],
    'gs_set_tuning': [ctypes.POINTER(GsTuning)],
    'gs_get_tuning': [ctypes.POINTER(GsTuning)],
    'gs_timer_read': [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                      ctypes.POINTER(ctypes.c_int64)],
}
EXPORTS = tuple(_SIGS) + ('gs_version',)

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f'libgs.so not found at {LIB_PATH}; build it first with '
                               '`python -m paper_2601_19489_amd.build` (no CPU fallback exists)')
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.gs_version.restype = ctypes.c_char_p
        L.gs_version.argtypes = []
        _lib = L
    return _lib


def _check(name, status):
    if status != GS_OK:
        raise RuntimeError(f'{name} failed: {_STATUS.get(status, status)}')


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError('libgs takes device tensors only')
    if not t.is_contiguous():
        raise ValueError('libgs takes contiguous tensors only')
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def camera(cam, tile=None) -> GsCamera:
    """GsCamera from any object with width, height, fx, fy, cx, cy, R, t,
    near and tile attributes."""
    c = GsCamera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.tile = int(tile if tile is not None else getattr(cam, 'tile', 16))
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = [float(x) for x in list(getattr(cam.R, 'ravel', lambda: cam.R)())]
    t = [float(x) for x in list(getattr(cam.t, 'ravel', lambda: cam.t)())]
    c.R = (ctypes.c_double * 9)(*R)
    c.t = (ctypes.c_double * 3)(*t)
    c.near_plane = float(getattr(cam, 'near', 0.2))
    c.depth_mode = int(getattr(cam, 'depth_mode', DEPTH_Z))
    return c


def gaussians(means, log_scales, quats, opacity_logits, sh) -> GsGaussians:
    g = GsGaussians()
    g.means, g.log_scales, g.quats = (_ptr(x) for x in (means, log_scales, quats))
    g.opacity_logits, g.sh = _ptr(opacity_logits), _ptr(sh)
    return g


def anchors(feat, pos, offsets, scaling) -> GsAnchors:
    a = GsAnchors()
    a.feat, a.pos, a.offsets, a.scaling = (_ptr(x) for x in (feat, pos, offsets, scaling))
    return a


def mlp(w1, b1, w2, b2) -> GsMlp:
    m = GsMlp()
    m.w1, m.b1, m.w2, m.b2 = (_ptr(x) for x in (w1, b1, w2, b2))
    return m


def _bg(bg):
    return (ctypes.c_float * 3)(*[float(x) for x in bg])


def gs_version() -> str:
    return lib().gs_version().decode()


def gs_preprocess(g: GsGaussians, n, sh_degree, cam: GsCamera, splats, depth_keys, tile_counts,
                  stream=None):
    _check('gs_preprocess', lib().gs_preprocess(ctypes.byref(g), n, sh_degree, ctypes.byref(cam),
                                                _ptr(splats), _ptr(depth_keys), _ptr(tile_counts),
                                                _stream(stream)))


def gs_bin_sort_workspace(n, capacity, cam: GsCamera) -> int:
    out = ctypes.c_size_t(0)
    _check('gs_bin_sort_workspace', lib().gs_bin_sort_workspace(n, capacity, ctypes.byref(cam),
                                                                ctypes.byref(out)))
    return int(out.value)


def gs_bin_sort(splats, depth_keys, tile_counts, n, cam: GsCamera, workspace, capacity, vals,
                ranges, keys_out, pair_count, stream=None):
    nbytes = workspace.numel() * workspace.element_size()
    _check('gs_bin_sort', lib().gs_bin_sort(_ptr(splats), _ptr(depth_keys), _ptr(tile_counts), n,
                                            ctypes.byref(cam), _ptr(workspace), nbytes, capacity,
                                            _ptr(vals), _ptr(ranges), _ptr(keys_out),
                                            _ptr(pair_count), _stream(stream)))


def gs_bin_sort_deferred(splats, depth_keys, tile_counts, n, cam: GsCamera, workspace, capacity,
                         ranges, pair_count, stream=None):
    nbytes = workspace.numel() * workspace.element_size()
    _check('gs_bin_sort_deferred', lib().gs_bin_sort_deferred(
        _ptr(splats), _ptr(depth_keys), _ptr(tile_counts), n, ctypes.byref(cam), _ptr(workspace),
        nbytes, capacity, _ptr(ranges), _ptr(pair_count), _stream(stream)))


def gs_render_fwd_deferred(splats, n, workspace, capacity, vals, ranges, cam: GsCamera, bg, image,
                           depth, T_final, n_contrib, stream=None):
    nbytes = workspace.numel() * workspace.element_size()
    _check('gs_render_fwd_deferred', lib().gs_render_fwd_deferred(
        _ptr(splats), n, _ptr(workspace), nbytes, capacity, _ptr(vals), _ptr(ranges),
        ctypes.byref(cam), _bg(bg), _ptr(image), _ptr(depth), _ptr(T_final), _ptr(n_contrib),
        _stream(stream)))


def gs_render_fwd(splats, n, vals, ranges, cam: GsCamera, bg, image, depth, T_final, n_contrib,
                  stream=None):
    _check('gs_render_fwd', lib().gs_render_fwd(_ptr(splats), n, _ptr(vals), _ptr(ranges),
                                                ctypes.byref(cam), _bg(bg), _ptr(image),
                                                _ptr(depth), _ptr(T_final), _ptr(n_contrib),
                                                _stream(stream)))


def gs_render_bwd(g: GsGaussians, n, sh_degree, cam: GsCamera, splats, vals, ranges, bg, T_final,
                  n_contrib, dL_dimage, dL_ddepth, grad2d, grads: GsGaussians, accumulate=False,
                  tile_order=None, stream=None):
    """tile_order: optional int32 scratch of 2 x tiles words; when given the
    tiles are processed heaviest first."""
    _check('gs_render_bwd', lib().gs_render_bwd(ctypes.byref(g), n, sh_degree, ctypes.byref(cam),
                                                _ptr(splats), _ptr(vals), _ptr(ranges), _bg(bg),
                                                _ptr(T_final), _ptr(n_contrib), _ptr(dL_dimage),
                                                _ptr(dL_ddepth), _ptr(grad2d), ctypes.byref(grads),
                                                int(bool(accumulate)), _ptr(tile_order),
                                                _stream(stream)))


def adam_params(m: GsGaussians, v: GsGaussians, lrs, beta1, beta2, eps, step) -> GsAdamParams:
    """lrs: five learning rates (means, log_scales, quats, opacity_logits, sh);
    step: device int32 step count."""
    a = GsAdamParams()
    a.m, a.v = m, v
    for k in range(5):
        a.lr[k] = float(lrs[k])
    a.beta1, a.beta2, a.eps = float(beta1), float(beta2), float(eps)
    a.step = _ptr(step)
    return a


def gs_render_bwd_adam(g: GsGaussians, n, sh_degree, cam: GsCamera, splats, vals, ranges, bg,
                       T_final, n_contrib, dL_dimage, dL_ddepth, grad2d, adam: GsAdamParams,
                       tile_order=None, stream=None):
    """gs_render_bwd then one Adam step of the parameters in g, fused: the
    gradients are not written out."""
    _check('gs_render_bwd_adam', lib().gs_render_bwd_adam(
        ctypes.byref(g), n, sh_degree, ctypes.byref(cam), _ptr(splats), _ptr(vals), _ptr(ranges),
        _bg(bg), _ptr(T_final), _ptr(n_contrib), _ptr(dL_dimage), _ptr(dL_ddepth), _ptr(grad2d),
        ctypes.byref(adam), _ptr(tile_order), _stream(stream)))


def gs_l1_loss(image, target, n, dL_dimage, loss_sum, stream=None):
    _check('gs_l1_loss', lib().gs_l1_loss(_ptr(image), _ptr(target), n, _ptr(dL_dimage),
                                          _ptr(loss_sum), _stream(stream)))


def gs_adam_step(p, g, m, v, n, lr, beta1, beta2, eps, step, stream=None):
    _check('gs_adam_step', lib().gs_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), n, lr, beta1,
                                              beta2, eps, step, _stream(stream)))


def gs_anchor_decode_fwd(a: GsAnchors, n_anchors, m: GsMlp, cam: GsCamera, out: GsGaussians,
                         stream=None):
    _check('gs_anchor_decode_fwd', lib().gs_anchor_decode_fwd(
        ctypes.byref(a), n_anchors, ctypes.byref(m), ctypes.byref(cam), ctypes.byref(out),
        _stream(stream)))


def gs_anchor_decode_workspace(n_anchors) -> int:
    out = ctypes.c_size_t(0)
    _check('gs_anchor_decode_workspace',
           lib().gs_anchor_decode_workspace(n_anchors, ctypes.byref(out)))
    return int(out.value)


def gs_anchor_decode_bwd(a: GsAnchors, n_anchors, m: GsMlp, cam: GsCamera, dchild: GsGaussians,
                         danchors: GsAnchors, dmlp: GsMlp, workspace, accumulate=False,
                         stream=None):
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check('gs_anchor_decode_bwd', lib().gs_anchor_decode_bwd(
        ctypes.byref(a), n_anchors, ctypes.byref(m), ctypes.byref(cam), ctypes.byref(dchild),
        ctypes.byref(danchors), ctypes.byref(dmlp), _ptr(workspace), nbytes,
        int(bool(accumulate)), _stream(stream)))


def gs_anchor_decode_bwd_noalloc(a: GsAnchors, n_anchors, m: GsMlp, cam: GsCamera,
                                 dchild: GsGaussians, danchors: GsAnchors, dmlp: GsMlp,
                                 accumulate=False, stream=None):
    _check('gs_anchor_decode_bwd_noalloc', lib().gs_anchor_decode_bwd_noalloc(
        ctypes.byref(a), n_anchors, ctypes.byref(m), ctypes.byref(cam), ctypes.byref(dchild),
        ctypes.byref(danchors), ctypes.byref(dmlp), int(bool(accumulate)), _stream(stream)))


def gs_depth_l1_loss(depth, target, n, weight, dL_ddepth, loss_sum, stream=None):
    _check('gs_depth_l1_loss', lib().gs_depth_l1_loss(_ptr(depth), _ptr(target), n, weight,
                                                      _ptr(dL_ddepth), _ptr(loss_sum),
                                                      _stream(stream)))


def gs_error_mask(image, target, n_pixels, tau, mask, minmax, stream=None):
    _check('gs_error_mask', lib().gs_error_mask(_ptr(image), _ptr(target), n_pixels, tau,
                                                _ptr(mask), _ptr(minmax), _stream(stream)))


def gs_split_score(splats, n, vals, ranges, cam: GsCamera, mask, score, stream=None):
    _check('gs_split_score', lib().gs_split_score(_ptr(splats), n, _ptr(vals), _ptr(ranges),
                                                  ctypes.byref(cam), _ptr(mask), _ptr(score),
                                                  _stream(stream)))


def gs_densify_workspace(n) -> int:
    out = ctypes.c_size_t(0)
    _check('gs_densify_workspace', lib().gs_densify_workspace(n, ctypes.byref(out)))
    return int(out.value)


def gs_densify_plan(score, log_scales, n, threshold, split_scale, workspace, n_out, stream=None):
    nbytes = workspace.numel() * workspace.element_size()
    _check('gs_densify_plan', lib().gs_densify_plan(_ptr(score), _ptr(log_scales), n, threshold,
                                                    split_scale, _ptr(workspace), nbytes,
                                                    _ptr(n_out), _stream(stream)))


def gs_densify_apply(g: GsGaussians, n, sh_degree, eps, workspace, n_out, moments,
                     out: GsGaussians, stream=None):
    _check('gs_densify_apply', lib().gs_densify_apply(
        ctypes.byref(g), n, sh_degree, _ptr(eps), _ptr(workspace), n_out, int(bool(moments)),
        ctypes.byref(out), _stream(stream)))


def gs_densify_threshold(score, n, min_threshold, max_selected, scratch, threshold,
                         stream=None):
    _check('gs_densify_threshold', lib().gs_densify_threshold(
        _ptr(score), n, min_threshold, max_selected, _ptr(scratch), _ptr(threshold),
        _stream(stream)))


def gs_densify_prune_plan(score, log_scales, n, threshold, split_scale, prune_score,
                          prune_threshold, workspace, n_out, stream=None):
    nbytes = workspace.numel() * workspace.element_size()
    _check('gs_densify_prune_plan', lib().gs_densify_prune_plan(
        _ptr(score), _ptr(log_scales), n, threshold, split_scale, _ptr(prune_score),
        prune_threshold, _ptr(workspace), nbytes, _ptr(n_out), _stream(stream)))


def gs_photo_loss_workspace(channels, height, width) -> int:
    out = ctypes.c_size_t(0)
    _check('gs_photo_loss_workspace',
           lib().gs_photo_loss_workspace(channels, height, width, ctypes.byref(out)))
    return out.value


def gs_photo_loss(image, target, channels, height, width, lam, workspace, loss, dL_dimage=None,
                  stream=None):
    nbytes = workspace.numel() * workspace.element_size()
    _check('gs_photo_loss', lib().gs_photo_loss(
        _ptr(image), _ptr(target), channels, height, width, lam, _ptr(workspace), nbytes,
        _ptr(loss), _ptr(dL_dimage), _stream(stream)))


def gs_prune_accumulate(count, n, photo, prune_score, split_score=None, stream=None):
    _check('gs_prune_accumulate', lib().gs_prune_accumulate(
        _ptr(count), n, _ptr(photo), _ptr(prune_score), _ptr(split_score), _stream(stream)))


def gs_pose_grad(g: GsGaussians, n, sh_degree, cam: GsCamera, grad2d, pose_grad, stream=None):
    _check('gs_pose_grad', lib().gs_pose_grad(ctypes.byref(g), n, sh_degree, ctypes.byref(cam),
                                              _ptr(grad2d), _ptr(pose_grad), _stream(stream)))


TILES_COMPACT, TILES_SNUGBOX, TILES_3SIGMA = 0, 1, 2


def gs_tile_count_variant(splats, n, cam: GsCamera, variant, counts, stream=None):
    _check('gs_tile_count_variant', lib().gs_tile_count_variant(
        _ptr(splats), n, ctypes.byref(cam), variant, _ptr(counts), _stream(stream)))


CKPT_INTERVAL = 32


def gs_render_fwd_ckpt(splats, n, vals, ranges, cam: GsCamera, bg, image, depth, T_final,
                       n_contrib, ckpt, ckpt_buckets, ckpt_overflow, stream=None):
    _check('gs_render_fwd_ckpt', lib().gs_render_fwd_ckpt(
        _ptr(splats), n, _ptr(vals), _ptr(ranges), ctypes.byref(cam), _bg(bg),
        _ptr(image), _ptr(depth), _ptr(T_final), _ptr(n_contrib), _ptr(ckpt), ckpt_buckets,
        _ptr(ckpt_overflow), _stream(stream)))


def gs_render_bwd_ckpt(g: GsGaussians, n, sh_degree, cam: GsCamera, splats, vals, ranges, image,
                       depth, n_contrib, ckpt, ckpt_buckets, dL_dimage, dL_ddepth, grad2d,
                       grads: GsGaussians, accumulate=False, stream=None):
    _check('gs_render_bwd_ckpt', lib().gs_render_bwd_ckpt(
        ctypes.byref(g), n, sh_degree, ctypes.byref(cam), _ptr(splats), _ptr(vals), _ptr(ranges),
        _ptr(image), _ptr(depth), _ptr(n_contrib), _ptr(ckpt), ckpt_buckets, _ptr(dL_dimage),
        _ptr(dL_ddepth), _ptr(grad2d), ctypes.byref(grads), int(bool(accumulate)),
        _stream(stream)))


def views_array(views):
    """ctypes array of GsView from a sequence of GsView."""
    arr = (GsView * len(views))(*views)
    return arr


def gs_preprocess_batched(g: GsGaussians, n, sh_degree, views, stream=None):
    arr = views_array(views)
    _check('gs_preprocess_batched', lib().gs_preprocess_batched(
        ctypes.byref(g), n, sh_degree, arr, len(views), _stream(stream)))


def gs_bin_sort_batched_workspace(n, views) -> int:
    out = ctypes.c_size_t(0)
    arr = views_array(views)
    _check('gs_bin_sort_batched_workspace', lib().gs_bin_sort_batched_workspace(
        n, arr, len(views), ctypes.byref(out)))
    return int(out.value)


def gs_bin_sort_batched(n, views, workspace, stream=None):
    arr = views_array(views)
    nbytes = workspace.numel() * workspace.element_size()
    _check('gs_bin_sort_batched', lib().gs_bin_sort_batched(n, arr, len(views), _ptr(workspace),
                                                            nbytes, _stream(stream)))


def _workspace_arrays(workspaces):
    ptrs = (ctypes.c_void_p * len(workspaces))(*(w.data_ptr() for w in workspaces))
    sizes = (ctypes.c_size_t * len(workspaces))(*(w.numel() * w.element_size()
                                                   for w in workspaces))
    return ptrs, sizes


def gs_bin_sort_batched_deferred(n, views, workspaces, stream=None):
    """workspaces: one device tensor per view (gs_bin_sort_workspace bytes each)."""
    arr = views_array(views)
    ptrs, sizes = _workspace_arrays(workspaces)
    _check('gs_bin_sort_batched_deferred', lib().gs_bin_sort_batched_deferred(
        n, arr, len(views), ptrs, sizes, _stream(stream)))


def gs_render_fwd_batched_deferred(n, views, workspaces, bg, queue, stream=None):
    arr = views_array(views)
    ptrs, sizes = _workspace_arrays(workspaces)
    _check('gs_render_fwd_batched_deferred', lib().gs_render_fwd_batched_deferred(
        n, arr, len(views), ptrs, sizes, _bg(bg), _ptr(queue), _stream(stream)))


def gs_render_fwd_batched(n, views, bg, queue, stream=None):
    arr = views_array(views)
    _check('gs_render_fwd_batched', lib().gs_render_fwd_batched(n, arr, len(views), _bg(bg),
                                                                _ptr(queue), _stream(stream)))


def gs_render_bwd_batched(g: GsGaussians, n, sh_degree, views, bg, queue, grads: GsGaussians,
                          accumulate=False, tile_order=None, stream=None):
    arr = views_array(views)
    _check('gs_render_bwd_batched', lib().gs_render_bwd_batched(
        ctypes.byref(g), n, sh_degree, arr, len(views), _bg(bg), _ptr(queue), ctypes.byref(grads),
        int(bool(accumulate)), _ptr(tile_order), _stream(stream)))


def gs_adam_step_grouped(groups, beta1, beta2, eps, step, stream=None):
    """groups: sequence of (p, g, m, v, lr) device tensors and learning rate."""
    arr = (GsAdamGroup * len(groups))()
    for k, (p, g, m, v, lr) in enumerate(groups):
        arr[k].p, arr[k].g, arr[k].m, arr[k].v = _ptr(p), _ptr(g), _ptr(m), _ptr(v)
        arr[k].n = p.numel()
        arr[k].lr = float(lr)
    _check('gs_adam_step_grouped', lib().gs_adam_step_grouped(arr, len(groups), beta1, beta2, eps,
                                                              _ptr(step), _stream(stream)))


def gs_timer_enable(kernel_name):
    name = None if kernel_name is None else kernel_name.encode()
    _check('gs_timer_enable', lib().gs_timer_enable(name))


KERNELS = ('preprocess', 'radix_hist', 'radix_scatter', 'bin_runs', 'bin_hist', 'bin_scatter',
           'render_fwd', 'render_bwd', 'preprocess_bwd', 'preprocess_bwd_adam', 'l1_loss', 'adam',
           'decode_fwd',
           'decode_bwd', 'decode_reduce', 'error_mask', 'split_score', 'densify', 'photo_loss', 'pose_grad',
           'tile_order')


def gs_timer_read(kernel_name=None):
    """(summed device milliseconds, launches) of the timed launches of one
    kernel (None: all) since they were last read."""
    ms = ctypes.c_double(0.0)
    k = ctypes.c_int64(0)
    name = None if kernel_name is None else kernel_name.encode()
    _check('gs_timer_read', lib().gs_timer_read(name, ctypes.byref(ms), ctypes.byref(k)))
    return ms.value, k.value


def gs_get_tuning() -> dict:
    t = GsTuning()
    _check('gs_get_tuning', lib().gs_get_tuning(ctypes.byref(t)))
    return dict(fwd_px=t.fwd_px, bwd_px=t.bwd_px, persist_wgs=t.persist_wgs,
                seq_walk=t.seq_walk, fwd_batch=t.fwd_batch, bwd_batch=t.bwd_batch)


def gs_set_tuning(**kw):
    cur = gs_get_tuning()
    cur.update(kw)
    t = GsTuning()
    t.fwd_px, t.bwd_px = int(cur['fwd_px']), int(cur['bwd_px'])
    t.persist_wgs = int(cur['persist_wgs'])
    t.seq_walk = int(cur['seq_walk'])
    t.fwd_batch, t.bwd_batch = int(cur['fwd_batch']), int(cur['bwd_batch'])
    _check('gs_set_tuning', lib().gs_set_tuning(ctypes.byref(t)))
