"""The C ABI library loads and exports every entry point include/gs.h
declares; host-side argument checks reject bad calls without launching."""
import ctypes
import os
import re

import pytest

from paper_2601_19489_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, 'include')):
        if fn.endswith('.h'):
            text = open(os.path.join(ROOT, 'include', fn)).read()
            names.update(re.findall(r'^\s*(?:const\s+)?[\w\s\*]+?\b(gs_\w+)\s*\(', text, re.M))
    return names


def test_header_declares_the_bound_entry_points():
    assert set(_lib.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert _lib.gs_version().startswith('libgs')


def test_host_argument_checks():
    lib = _lib.lib()
    cam = _lib.GsCamera()
    cam.width, cam.height, cam.tile = 64, 64, 16
    cam.fx = cam.fy = 50.0
    cam.near_plane = 0.2
    g = _lib.GsGaussians()
    # negative size, bad SH degree, bad tile size -> GS_EINVAL, nothing launched
    assert lib.gs_preprocess(ctypes.byref(g), -1, 0, ctypes.byref(cam), None, None, None, None) == 1
    assert lib.gs_preprocess(ctypes.byref(g), 10, 4, ctypes.byref(cam), None, None, None, None) == 1
    cam.tile = 12
    assert lib.gs_preprocess(ctypes.byref(g), 10, 0, ctypes.byref(cam), None, None, None, None) == 1
    assert lib.gs_adam_step(None, None, None, None, 10, 0.1, 0.9, 0.999, 1e-8, 0, None) == 1
    out = ctypes.c_size_t(0)
    cam.tile = 16
    assert lib.gs_bin_sort_workspace(1000, 5000, ctypes.byref(cam), ctypes.byref(out)) == 0
    assert out.value > 5000 * 8  # the column runs: Gaussian id and row span per run
    assert lib.gs_bin_sort_workspace(10, 1 << 33, ctypes.byref(cam), ctypes.byref(out)) == 1
    # decoder: workspace query, bad sizes, missing outputs, missing workspace
    assert lib.gs_anchor_decode_workspace(100_000, ctypes.byref(out)) == 0
    assert out.value >= 256 * 9984 * 4
    assert lib.gs_anchor_decode_workspace(-1, ctypes.byref(out)) == 1
    a, m, dm = _lib.GsAnchors(), _lib.GsMlp(), _lib.GsMlp()
    assert lib.gs_anchor_decode_fwd(ctypes.byref(a), -5, ctypes.byref(m), ctypes.byref(cam),
                                    ctypes.byref(g), None) == 1
    assert lib.gs_anchor_decode_fwd(ctypes.byref(a), 10, ctypes.byref(m), ctypes.byref(cam),
                                    ctypes.byref(g), None) == 1
    assert lib.gs_anchor_decode_bwd(ctypes.byref(a), 10, ctypes.byref(m), ctypes.byref(cam),
                                    ctypes.byref(g), ctypes.byref(a), ctypes.byref(dm), None, 0,
                                    0, None) == 1
    # direct mode (-1) is a valid degree; -2 is not
    assert lib.gs_preprocess(ctypes.byref(g), 10, -2, ctypes.byref(cam), None, None, None, None) == 1
    # densification: workspace query and threshold arguments
    assert lib.gs_densify_workspace(1000, ctypes.byref(out)) == 0 and out.value >= 2000 * 4
    assert lib.gs_densify_workspace(-1, ctypes.byref(out)) == 1
    fake = ctypes.c_void_p(16)  # never dereferenced: each call below fails its host checks
    assert lib.gs_densify_threshold(fake, 10, 0, 5, fake, fake, None) == 1         # t_min 0
    assert lib.gs_densify_threshold(fake, 10, 65536, 5, fake, fake, None) == 1     # t_min too big
    assert lib.gs_densify_threshold(fake, 10, 1, -1, fake, fake, None) == 1        # cap < 0
    assert lib.gs_densify_threshold(fake, 10, 1, 5, None, fake, None) == 1         # no scratch
    assert lib.gs_densify_plan(fake, fake, 10, 0, 0.1, fake, 1 << 20, fake, None) == 1  # thr 0
