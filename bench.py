#!/usr/bin/env python3
"""Benchmark one training step of the tile rasterizer on one MI355X.

A step is the whole hot path over one view with inputs resident in HBM:
preprocess (EWA, SH, compact tile counts) -> binning and sort -> tile
compositing -> L1 loss -> backward (image space, then per Gaussian) ->
fused Adam over all parameters. Prints one JSON line.

Default workload: 1,000,000 Gaussians, SH degree 3, sampled on 3 noisy
planes and 4 spheres with a heavy-tailed scale mix (10% large), one
1600x1066 view with 16x16 tiles, a uniform random target image. Synthetic
inputs (seeded); the paper's own scenes are not used.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = 'fwd+bwd ms/iter @1M Gaussians 1600×1066, HBM GB/s; anchor vs plain time-to-PSNR'
HBM_PEAK_GBS = 8000.0
# Adam learning rates per parameter group (the values 3DGS-style training uses)
LRS = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, sh=2.5e-3)

WORKLOADS = {
    'headline': dict(n=1_000_000, width=1600, height=1066, sh_degree=3, seed=2),
    'surface500k': dict(n=500_000, width=1600, height=1066, sh_degree=3, seed=2),
    # 8 orbit views at mixed resolutions, one graph-captured batched step
    'batch8': dict(n=1_000_000, sh_degree=3, seed=3, views=8),
    # anchor form vs plain Gaussians: time to the plain model's held-out PSNR
    'anchor': dict(gt=200_000, anchors=20_000, train_views=24, test_views=6, width=800,
                   height=534, steps=2000, eval_every=100, seed=4),
    # anchor form vs plain Gaussians at full size: 100k anchors x 10 children
    # against a 500k-Gaussian SH3 ground truth, 100 + 20 views at 1600x1066;
    # plain runs 6000 steps, the anchor form until it reaches the plain
    # model's final held-out PSNR - 0.1 dB (at most 6000 steps)
    'c4': dict(gt=500_000, anchors=100_000, train_views=100, test_views=20, width=1600,
               height=1066, steps=6000, eval_every=100, seed=4),
    # densifying fit: 1M-Gaussian ground truth, 200 views (every 8th held out),
    # 300k sparse start grown to about 3M by Eq. 3-4, depth L1 0.1 -> 0
    'densify': dict(gt=1_000_000, init=300_000, growth_to=3_000_000, views=200, width=1600,
                    height=1066, steps=6000, seed=5, depth_mode=0),
    # the same fit supervising disparity (blended inverse depth) instead of depth
    'densify_disparity': dict(gt=1_000_000, init=300_000, growth_to=3_000_000, views=200,
                              width=1600, height=1066, steps=6000, seed=5, depth_mode=1),
}
BF16_PEAK_TFLOPS = 2500.0
DECODER_ANCHORS = 100_000
# decoder flops per anchor: 2 (35 x 96 + 32 x 110) multiply-adds forward,
# twice that in the backward (input and weight gradients)
DEC_FLOP_FWD = 2 * (35 * 96 + 32 * 110)
DEC_FLOP_BWD = 2 * DEC_FLOP_FWD
# decoder HBM bytes per anchor: forward reads feat, pos, offsets, scaling
# (32 + 3 + 30 + 6 floats) and writes 10 children x 14 floats; backward
# reads the anchor inputs and the 10 x 14 child gradients and writes dfeat,
# doffsets, dscaling (32 + 30 + 6 floats)
DEC_BYTES_FWD = 4 * (71 + 140)
DEC_BYTES_BWD = 4 * (71 + 140 + 68)


# FP32 vector issue ceiling: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane operations
# per second (an FMA is one operation; packed FP32 is not used by this build)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# VALU lane operations of one (pixel, splat) evaluation of the compositing
# formula (an FMA counts once, a transcendental four times: quarter rate)
OPS_FWD = 23          # dx, dy, Q, skip test, exp, alpha, T', stop test, blend C and D
OPS_BWD = 49          # as forward, plus 1/(1-a), dL/dalpha, the 9 gradient sums, S update
OPS_BWD_DEPTH = 53    # with the depth term


def kernel_bytes(name, n, K, P, Pr, pixels, waves_pairs):
    """Algorithmic HBM bytes of one launch of each kernel.

    n Gaussians, K SH coefficients, P pairs, Pr processed (tile, splat)
    pairs, pixels, waves_pairs (wavefront, splat) reductions in the backward.
    """
    params = 4 * (3 + 3 + 4 + 1 + 3 * K)
    if name == 'preprocess':
        return n * (params + 48 + 4 + 4)
    if name == 'render_fwd':
        return Pr * (4 + 48) + pixels * (12 + 4 + 4 + 4) + 0
    if name == 'render_bwd':
        return Pr * (4 + 48) + pixels * (4 + 4 + 12) + waves_pairs * 40
    if name == 'preprocess_bwd':
        return n * (params + 40 + params)
    if name == 'preprocess_bwd_adam':  # p, m, v read and written, the 2D gradient read
        return n * (6 * params + 40)
    return None


def view_stats(n_contrib, ranges, tiles_x, tiles_y, T):
    """Work of one rendered view: pairs P, (tile, splat) pairs the forward
    and backward visit, pixels, and (pixel, splat) evaluations. n_contrib is
    the [H, W] uint32 image, ranges the column-major tile ranges."""
    import numpy as np

    nc = n_contrib.astype(np.int64)
    H, W = nc.shape
    pad = np.zeros((tiles_y * T, tiles_x * T), np.int64)
    pad[:H, :W] = nc
    tmax = pad.reshape(tiles_y, T, tiles_x, T).max(axis=(1, 3))
    r = ranges.astype(np.int64)
    lens = np.diff(r).reshape(tiles_x, tiles_y).T       # column-major tile ids
    lens_px = np.repeat(np.repeat(lens, T, axis=0), T, axis=1)[:H, :W]
    return dict(P=int(r[-1]), Pr_fwd=int(np.minimum(tmax + 1, lens).sum()),
                Pr_bwd=int(tmax.sum()), pixels=H * W, tiles=tiles_x * tiles_y,
                evals_fwd=int(np.minimum(nc + 1, lens_px).sum()), evals_bwd=int(nc.sum()))


def column_runs(splats, tiles_x):
    """Column runs of the binning: per Gaussian, the columns from the first
    to the last holding tiles (splat record word 11: first column | count
    << 16), clamped to the grid."""
    import numpy as np

    w = np.ascontiguousarray(splats[:, 11]).view(np.uint32).astype(np.int64)
    f, ln = w & 0xFFFF, w >> 16
    ln = np.where(f >= tiles_x, 0, np.minimum(ln, tiles_x - f))
    return int(ln.sum())


def step_model(n, K, views, fused=False, deferred=False):
    """Algorithmic HBM bytes and FP32 VALU lane operations of one training
    step over `views` (view_stats dicts), per kernel: what the method itself
    has to move or compute, not what this build's kernels happen to move.

    preprocess      parameters (11 + 3K floats) read; 48-byte splat record,
                    depth key and tile count written, per Gaussian and view
    binning         per Gaussian and view the depth key, tile count and the
                    six record fields of the tile-set walk read (32 B); per
                    pair one 4-byte Gaussian id written; tile ranges
    render_fwd      per visited (tile, splat): id and record (52 B); per pixel
                    image, depth, T_final, n_contrib written (24 B); VALU:
                    OPS_FWD per evaluation
    l1_loss         per pixel image and target read, dL/dimage written (36 B)
    tile_order      n_contrib read per pixel (the launch also clears the
                    backward's 2D gradient accumulators, not counted)
    render_bwd      per visited (tile, splat): id, record, one 40-byte
                    gradient read and written; per pixel image gradient,
                    T_final, n_contrib read (20 B); VALU: OPS_BWD per evaluation
    preprocess_bwd  parameters read, one 40-byte 2D gradient per Gaussian and
                    view read, parameter gradients written
    adam            per parameter p, g, m, v read and p, m, v written (28 B)
    bwd_adam        (fused=True, one view: in place of the last two) per
                    parameter p, m, v read and written (24 B), one 40-byte 2D
                    gradient per Gaussian read
    deferred=True (the lists written by the forward as far as it reaches;
    views carry 'runs'): the binning writes one 8-byte run per column run
    instead of the pairs, and the forward reads a run (8 B) in place of an
    id and writes the id (4 B) per visited (tile, splat)
    """
    params = 4 * (11 + 3 * K)
    V = len(views)
    S = lambda k: sum(v[k] for v in views)  # noqa: E731
    m = {
        'preprocess': (V * n * (params + 48 + 4 + 4), 0),
        'binning': (V * n * 32 + (8 * S('runs') if deferred else 4 * S('P'))
                    + 4 * (S('tiles') + V), 0),
        'render_fwd': ((60 if deferred else 52) * S('Pr_fwd') + 24 * S('pixels'),
                       OPS_FWD * S('evals_fwd')),
        'l1_loss': (36 * S('pixels'), 0),
        'tile_order': (4 * S('pixels'), 0),
        'render_bwd': ((52 + 80) * S('Pr_bwd') + 20 * S('pixels'), OPS_BWD * S('evals_bwd')),
        'preprocess_bwd': (n * (2 * params + 40 * V), 0),
        'adam': (n * params // 4 * 28, 0),
    }
    if fused:
        del m['preprocess_bwd'], m['adam']
        m['bwd_adam'] = (n * (params // 4 * 24 + 40 * V), 0)
    return m


# which timed launches of the library belong to which row of step_model
STEP_ROWS = {'preprocess': ('preprocess',), 'binning': ('radix_hist', 'radix_scatter', 'bin_runs',
                                                         'bin_hist', 'bin_scatter'),
             'render_fwd': ('render_fwd',), 'l1_loss': ('l1_loss',), 'tile_order': ('tile_order',),
             'render_bwd': ('render_bwd',), 'preprocess_bwd': ('preprocess_bwd',),
             'adam': ('adam',), 'bwd_adam': ('preprocess_bwd_adam',)}


def step_roofline(model, ms_per_step, kernel_ms=None):
    """Step roofline: t_roof = sum over kernels of max(bytes / HBM peak,
    ops / VALU issue peak); frac = t_roof / measured step time; the step's
    algorithmic HBM GB/s. kernel_ms (event-timed ms per step by library
    kernel name) adds each row's measured time (launches the library does not
    time, such as its scans, count only in the step total)."""
    rows = {}
    t_roof = 0.0
    tot_bytes = 0
    for k, (b, ops) in model.items():
        tb, to = b / (HBM_PEAK_GBS * 1e9), ops / (ALU_PEAK_TOPS * 1e12)
        t = max(tb, to)
        t_roof += t
        tot_bytes += b
        row = {'bytes': int(b), 'ops': int(ops), 'bound': 'alu' if to > tb else 'hbm',
               't_roof_ms': round(t * 1e3, 4)}
        if kernel_ms is not None:
            ms = sum(kernel_ms.get(x, 0.0) for x in STEP_ROWS[k])
            row['ms'] = round(ms, 4)
            row['frac'] = round(t * 1e3 / ms, 4) if ms > 0 else None
        rows[k] = row
    return {'t_roof_ms': round(t_roof * 1e3, 4), 'ms_per_step': round(ms_per_step, 4),
            'frac': round(t_roof * 1e3 / ms_per_step, 4),
            'algorithmic_gb': round(tot_bytes / 1e9, 4),
            'hbm_gbs': round(tot_bytes / (ms_per_step * 1e-3) / 1e9, 1),
            'hbm_frac': round(tot_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            'peaks': {'hbm_gbs': HBM_PEAK_GBS, 'valu_tops': round(ALU_PEAK_TOPS, 2)},
            'kernels': rows}


# state the forked oracle workers of cpu_baseline read (set before the fork)
_CPU = {}


def _cpu_worker_init():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _cpu_share(job):
    """One worker's share of one phase of the oracle step; returns its
    seconds. Runs in a forked worker process (numpy, one thread)."""
    import numpy as np

    from oracle import adam as oadam
    from oracle import backward as obwd
    from oracle import binning as obin
    from oracle import preprocess as opre
    from oracle import render as oren

    kind, idx = job
    d, pre, cam = _CPU['d'], _CPU['pre'], _CPU['cam']
    N = d['means'].shape[1]
    t = time.perf_counter()
    if kind == 'preprocess':
        opre.preprocess(d['means'][:, idx], d['log_scales'][:, idx], d['quats'][:, idx],
                        d['opacity_logits'][idx], d['sh'][..., idx], d['sh_degree'], cam)
    elif kind == 'binning':
        sub = {k: (v[..., idx] if isinstance(v, np.ndarray) and v.shape[-1:] == (N,) else v)
               for k, v in pre.items() if not k.startswith('_')}
        obin.tile_counts(sub, cam)
        obin.sorted_pairs(sub, cam)
    elif kind == 'tiles':
        tiles = [tuple(x) for x in idx]
        n_all = cam.tiles_x * cam.tiles_y
        lists = {tt: obin.tile_members(pre, cam, *tt) for tt in tiles}
        ranges = np.zeros(n_all + 1, np.int64)
        order = []
        for tid in range(n_all):
            m = lists.get(divmod(tid, cam.tiles_y))
            if m is not None:
                order.append(m)
            ranges[tid + 1] = ranges[tid] + (0 if m is None else len(m))
        vals = np.concatenate(order) if order else np.zeros(0, np.int64)
        dI = np.random.default_rng(len(tiles)).standard_normal((3, cam.height, cam.width)) * 1e-3
        oren.render(pre, cam, vals, ranges, tiles=tiles)
        g2d, _ = oren.render_backward(pre, cam, vals, ranges, dI, tiles=tiles)
        _CPU['g2d_shape'] = g2d.shape
    elif kind == 'backward':
        sub_pre = opre.preprocess(d['means'][:, idx], d['log_scales'][:, idx], d['quats'][:, idx],
                                  d['opacity_logits'][idx], d['sh'][..., idx], d['sh_degree'], cam)
        g2d = np.random.default_rng(len(idx)).standard_normal((10, len(idx))) * 1e-6
        obwd.preprocess_backward(sub_pre, g2d, d['sh_degree'], cam)
        for k in ('means', 'log_scales', 'quats', 'opacity_logits', 'sh'):
            x = d[k][..., idx]
            oadam.adam_step(x, x, np.zeros_like(x), np.zeros_like(x), 1e-3, 0.9, 0.999, 1e-15, 1)
    return time.perf_counter() - t


def cpu_workers():
    """The host cores this process may use, at most 16 (one GPU's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(d, per_worker_g=12000, per_worker_tiles=4, seed=0):
    """Time the FP64 oracle on a bounded sample of one training step, on a
    pool of forked worker processes (one thread each), and scale each phase
    to the full step. Must run before the process initialises the GPU (the
    workers are forked). Returns the JSON object."""
    import multiprocessing

    import numpy as np

    from oracle import preprocess as opre

    cam = d['camera']
    N = d['means'].shape[1]
    W = cpu_workers()
    rng = np.random.default_rng(seed)
    t_all = time.perf_counter()
    # the full preprocess, which the tile lists of the sampled tiles need (the
    # workers time their own share of it below)
    _CPU.update(d=d, cam=cam, pre=opre.preprocess(d['means'], d['log_scales'], d['quats'],
                                                  d['opacity_logits'], d['sh'], d['sh_degree'],
                                                  cam))
    n_g = min(N, per_worker_g * W)
    sample = np.sort(rng.choice(N, n_g, replace=False))
    n_all = cam.tiles_x * cam.tiles_y
    n_t = per_worker_tiles * W
    tiles = np.stack([rng.integers(cam.tiles_x // 4, 3 * cam.tiles_x // 4, n_t),
                      rng.integers(cam.tiles_y // 4, 3 * cam.tiles_y // 4, n_t)], axis=1)
    phases = {'preprocess': (np.array_split(np.arange(N), W), 1.0),
              'binning': (np.array_split(sample, W), N / n_g),
              'tiles': (np.array_split(tiles, W), n_all / n_t),
              'backward': (np.array_split(sample, W), N / n_g)}
    wall, cpu = {}, {}
    ctx = multiprocessing.get_context('fork')
    with ctx.Pool(W, initializer=_cpu_worker_init) as pool:
        for name, (jobs, scale) in phases.items():
            t = time.perf_counter()
            secs = pool.map(_cpu_share, [(name, j) for j in jobs])
            wall[name] = (time.perf_counter() - t) * scale
            cpu[name] = sum(secs) * scale
        pool.close()
        pool.join()
    _CPU.clear()
    total = sum(wall.values())
    return {'value': round(total * 1e3, 1), 'unit': 'ms/iter', 'cores': W, 'kind': 'oracle',
            'sample': (f'FP64 numpy oracle on {W} forked worker processes (one thread each): '
                       f'preprocess of all {N} Gaussians; tile sets + sort of {n_g} sampled '
                       f'Gaussians (x{N / n_g:.1f}); per-tile lists + render fwd/bwd of {n_t} '
                       f'sampled tiles (x{n_all / n_t:.1f}); per-Gaussian backward + Adam of the '
                       f'Gaussian sample (x{N / n_g:.1f}); '
                       f'{time.perf_counter() - t_all:.1f} s wall'),
            'phase_ms': {k: round(v * 1e3, 1) for k, v in wall.items()},
            'single_thread_equiv_ms': round(sum(cpu.values()) * 1e3, 1),
            'host_cpu': f'{_cpu_model()}, {os.cpu_count()} logical CPUs, {W} used'}


TRAFFIC_SUMMARY = os.path.join(ROOT, 'profiles', 'step_1M_1600x1066_hbm_traffic.md')


def measured_traffic(kernel):
    """Calibrated HBM bytes per launch of `kernel` from the committed counter
    summary, or None when the kernel's source changed since it was measured
    (or the summary has no row for it)."""
    import hashlib
    try:
        lines = open(TRAFFIC_SUMMARY).read().splitlines()
    except OSError:
        return None
    for line in lines:
        cells = [c.strip() for c in line.strip().strip('|').split('|')]
        if len(cells) == 5 and cells[0] == kernel:
            src, digest = cells[1].split()
            path = os.path.join(ROOT, 'paper_2601_19489_amd', 'csrc', src)
            now = hashlib.sha256(open(path, 'rb').read()).hexdigest()[:16]
            return int(float(cells[4])) if now == digest else None
    return None


TRACE_SUMMARY = os.path.join(ROOT, 'profiles', 'step_1M_1600x1066_kernel_trace.md')


def profile_avg_ms(kernel):
    """Average duration (ms) of one launch of `kernel` over the timed steps of
    the committed rocprofv3 kernel-trace summary of this workload, or None
    when the kernel's source changed since (or the summary has no row)."""
    import hashlib
    try:
        lines = open(TRACE_SUMMARY).read().splitlines()
    except OSError:
        return None
    for line in lines:
        cells = [c.strip() for c in line.strip().strip('|').split('|')]
        if len(cells) == 4 and cells[0] == kernel:
            src, digest = cells[1].split()
            path = os.path.join(ROOT, 'paper_2601_19489_amd', 'csrc', src)
            now = hashlib.sha256(open(path, 'rb').read()).hexdigest()[:16]
            try:
                return round(float(cells[3]) / 1e3, 4) if now == digest else None
            except ValueError:
                return None
    return None


COUNTER_SUMMARY = os.path.join(ROOT, 'profiles', 'render_valu_decoder_mfma_counters_1M_1600x1066.md')


def valu_counters(kernel):
    """VALU issue utilisation and lane instructions per evaluation of a render
    kernel from the committed SQ_INSTS_VALU counter summary, or None when
    the kernel's source changed since (or the summary has no row)."""
    import hashlib
    try:
        lines = open(COUNTER_SUMMARY).read().splitlines()
    except OSError:
        return None
    for line in lines:
        cells = [c.strip() for c in line.strip().strip('|').split('|')]
        if len(cells) == 8 and cells[0] == kernel:
            src, digest = cells[1].split()
            path = os.path.join(ROOT, 'paper_2601_19489_amd', 'csrc', src)
            if hashlib.sha256(open(path, 'rb').read()).hexdigest()[:16] != digest:
                return None
            return {'valu_issue_utilisation': float(cells[5]),
                    'lane_instructions_per_eval': float(cells[6]),
                    'source': 'SQ_INSTS_VALU, rocprofv3 --pmc (profiles/)'}
    return None


def decoder_measure(iters=20):
    """Time the anchor decoder forward and backward at 100,000 anchors with
    HIP events on the current stream. Returns the JSON object."""
    import torch

    from paper_2601_19489_amd import _lib, scenes
    from paper_2601_19489_amd.anchors import ANCHOR_NAMES, MLP_NAMES, AnchorDecoder, to_device

    A = DECODER_ANCHORS
    a = to_device(scenes.anchor_cloud(A, seed=4), ANCHOR_NAMES)
    m = to_device(scenes.decoder_mlp(seed=5), MLP_NAMES)
    cam = _lib.camera(scenes.look_at_camera((0.0, 0.0, -4.0), (0, 0, 0), 1600, 1066))
    dec = AnchorDecoder(A)
    ch = dec.decode(a, m, cam)
    dchild = {k: torch.randn_like(v) * 1e-3 for k, v in ch.items()}
    da = {k: torch.empty_like(a[k]) for k in ('feat', 'offsets', 'scaling')}
    dm = {k: torch.empty_like(v) for k, v in m.items()}
    for _ in range(3):
        dec.decode(a, m, cam)
        dec.backward(a, m, cam, dchild, da, dm)
    torch.cuda.synchronize()
    _lib.gs_timer_read(None)
    _lib.gs_timer_enable('*')
    for _ in range(iters):
        dec.decode(a, m, cam)
        dec.backward(a, m, cam, dchild, da, dm)
    torch.cuda.synchronize()
    t = {k: _lib.gs_timer_read(k) for k in ('decode_fwd', 'decode_bwd', 'decode_reduce')}
    _lib.gs_timer_enable(None)
    _lib.gs_timer_read(None)
    fwd = t['decode_fwd'][0] / max(t['decode_fwd'][1], 1)
    bwd = t['decode_bwd'][0] / max(t['decode_bwd'][1], 1)
    red = t['decode_reduce'][0] / max(t['decode_reduce'][1], 1)
    out = {'anchors': A, 'children': A * 10, 'fwd_ms': round(fwd, 4), 'bwd_ms': round(bwd, 4),
           'reduce_ms': round(red, 4)}
    for ph, ms, fl, by in (('fwd', fwd, DEC_FLOP_FWD, DEC_BYTES_FWD),
                           ('bwd', bwd, DEC_FLOP_BWD, DEC_BYTES_BWD)):
        tf = A * fl / (ms * 1e-3) / 1e12
        gb = A * by / (ms * 1e-3) / 1e9
        out[ph] = {'mfma_tflops': round(tf, 2), 'mfma_frac_bf16': round(tf / BF16_PEAK_TFLOPS, 5),
                   'hbm_gbs': round(gb, 1), 'hbm_frac': round(gb / HBM_PEAK_GBS, 4)}
    return out


def ablation_measure(R, p, iters=5):
    """Binning ablation on the benchmark view (Sec. 2.1): pair counts of the
    compact tile set, the SnugBox and the 3-sigma box, and the tile-set walks
    (preprocess count + run count/emit) load-balanced against sequential."""
    import torch

    from paper_2601_19489_amd import _lib

    n = R.n
    counts = torch.empty(n, dtype=torch.int32, device='cuda')
    pairs = {}
    for name, v in (('compact', _lib.TILES_COMPACT), ('snugbox', _lib.TILES_SNUGBOX),
                    ('box_3sigma', _lib.TILES_3SIGMA)):
        _lib.gs_tile_count_variant(R.splats, n, R.cam, v, counts)
        pairs[name] = int(counts.to(torch.int64).sum().item())
    res = {'pairs': pairs}
    for label, seq in (('load_balanced', 0), ('sequential', 1)):
        _lib.gs_set_tuning(seq_walk=seq)
        R.forward(p, check_overflow=False)
        torch.cuda.synchronize()
        _lib.gs_timer_read(None)  # no events left from earlier measurements
        _lib.gs_timer_enable('*')
        for _ in range(iters):
            R.forward(p, check_overflow=False)
        torch.cuda.synchronize()
        t = {k: _lib.gs_timer_read(k) for k in ('preprocess', 'bin_runs')}
        _lib.gs_timer_enable(None)
        _lib.gs_timer_read(None)
        res[label + '_walk_ms'] = {k: round(ms / max(c, 1), 4) for k, (ms, c) in t.items()}
    _lib.gs_set_tuning(seq_walk=0)
    # backward designs: this build's pixel-parallel recompute backward against
    # the checkpointed per-splat backward (checkpointing forward + backward)
    import math
    names = ('means', 'log_scales', 'quats', 'opacity_logits', 'sh')
    R.forward(p, check_overflow=False)
    torch.cuda.synchronize()
    nbk = max(1, math.ceil(int(R.n_contrib.max().item()) / _lib.CKPT_INTERVAL))
    ck = torch.empty(R.n_tiles * nbk * 5 * 256, device='cuda')
    ovf = torch.zeros(1, dtype=torch.int32, device='cuda')
    img, dep = torch.empty_like(R.image), torch.empty_like(R.depth)
    Tf, nc = torch.empty_like(R.T_final), torch.empty_like(R.n_contrib)
    dI = torch.full_like(R.image, 1e-7)
    grads = {k: torch.empty_like(v) for k, v in p.items()}
    g2 = torch.empty_like(R.grad2d)
    G = _lib.gaussians(*(p[k] for k in names))
    GG = _lib.gaussians(*(grads[k] for k in names))
    t = {}
    for label, fn in (('pixel_parallel', lambda: (R.render_fwd(), R.backward(p, dI, None, grads))),
                      ('checkpointed_per_splat', lambda: (
                          _lib.gs_render_fwd_ckpt(R.splats, n, R.vals, R.ranges, R.cam, R.bg, img,
                                                  dep, Tf, nc, ck, nbk, ovf),
                          _lib.gs_render_bwd_ckpt(G, n, R.sh_degree, R.cam, R.splats, R.vals,
                                                  R.ranges, img, dep, nc, ck, nbk, dI, None, g2,
                                                  GG)))):
        fn()
        torch.cuda.synchronize()
        _lib.gs_timer_read(None)
        _lib.gs_timer_enable('*')
        for _ in range(iters):
            fn()
        torch.cuda.synchronize()
        t[label] = {k: round(_lib.gs_timer_read(k)[0] / iters, 4)
                    for k in ('render_fwd', 'render_bwd', 'preprocess_bwd')}
        _lib.gs_timer_enable(None)
        _lib.gs_timer_read(None)
    res['backward_ms'] = t
    res['checkpoint_buckets'] = nbk
    res['checkpoint_overflow'] = int(ovf.item())
    return res


def densify_measure(R, p, target, iters=10):
    """Time the densification pieces on the benchmark view: the Eq. 3 error
    mask, the Eq. 4 split score, and the clone/split plan and apply over all
    Gaussians (the apply into fresh arrays). Returns the JSON object."""
    import torch

    from paper_2601_19489_amd import _lib, scenes

    n = R.n
    HW = R.image.shape[1] * R.image.shape[2]
    mask = torch.empty(R.image.shape[1:], dtype=torch.uint8, device='cuda')
    mm = torch.empty(2, dtype=torch.int32, device='cuda')
    score = torch.zeros(n, dtype=torch.int32, device='cuda')
    ws = torch.empty(_lib.gs_densify_workspace(n), dtype=torch.uint8, device='cuda')
    n_out_d = torch.zeros(1, dtype=torch.int32, device='cuda')
    eps = torch.randn((2, 3, n), device='cuda')
    names = ('means', 'log_scales', 'quats', 'opacity_logits', 'sh')
    R.forward(p, check_overflow=False)
    _lib.gs_error_mask(R.image, target, HW, 0.1, mask, mm)
    _lib.gs_split_score(R.splats, n, R.vals, R.ranges, R.cam, mask, score)
    thr = max(1, int(score.float().quantile(0.9).item()))
    _lib.gs_densify_plan(score, p['log_scales'], n, thr, 0.05, ws, n_out_d)
    n_out = int(n_out_d.item())
    out = {k: torch.empty(tuple(v.shape[:-1]) + (n_out,), device='cuda') for k, v in p.items()}
    g = _lib.gaussians(*(p[k] for k in names))
    o = _lib.gaussians(*(out[k] for k in names))
    torch.cuda.synchronize()
    _lib.gs_timer_read(None)
    _lib.gs_timer_enable('*')
    for _ in range(iters):
        _lib.gs_error_mask(R.image, target, HW, 0.1, mask, mm)
        _lib.gs_split_score(R.splats, n, R.vals, R.ranges, R.cam, mask, score)
        _lib.gs_densify_plan(score, p['log_scales'], n, thr, 0.05, ws, n_out_d)
        _lib.gs_densify_apply(g, n, 3, eps, ws, n_out, False, o)
    torch.cuda.synchronize()
    t = {k: _lib.gs_timer_read(k) for k in ('error_mask', 'split_score', 'densify')}
    _lib.gs_timer_enable(None)
    _lib.gs_timer_read(None)
    res = {k: round(v[0] / max(v[1], 1), 4) for k, v in t.items()}
    res.update(gaussians_in=n, gaussians_out=n_out, score_threshold=thr,
               masked_pixels=int(mask.sum().item()))
    # apply: reads 236 B and writes 236 B per output Gaussian (SH3)
    res['densify_apply_gbs'] = round((n + n_out) * 236 / (res['densify'] * 1e-3) / 1e9, 1)
    return res


def batch8_measure(steps, warmup, tune=False):
    """8 orbit views at mixed resolutions, 1M Gaussians: the graph-captured
    batched step against the eager per-view loop, with the step roofline of
    the batch. Returns the JSON object."""
    import numpy as np
    import torch

    from paper_2601_19489_amd import _lib, scenes
    from paper_2601_19489_amd.batched import BatchedRasterizer, TrainStep, autotune
    from paper_2601_19489_amd.rasterizer import Adam, Rasterizer, l1_loss, params_to_device

    wl = WORKLOADS['batch8']
    d = scenes.surface_cloud(wl['n'], seed=wl['seed'], sh_degree=wl['sh_degree'], width=64,
                             height=64)
    cams = scenes.orbit_cameras(wl['views'], seed=wl['seed'])
    p = params_to_device(d)
    n = wl['n']
    K = (wl['sh_degree'] + 1) ** 2
    targets = [torch.as_tensor(scenes.random_image((3, c.height, c.width), 200 + i),
                               device='cuda') for i, c in enumerate(cams)]

    def make(tile):
        q = {k: v.clone() for k, v in p.items()}
        B = BatchedRasterizer(n, cams, wl['sh_degree'], tile=tile, deferred=True)
        B.size_pairs(q)
        return TrainStep(B, q, targets, LRS)

    tuned = None
    if tune:
        tuned, _table = autotune(make, log=lambda m: print(m, file=sys.stderr, flush=True))
        tile = tuned['tile']
    else:
        tile = 16
    st = make(tile)
    st.run()
    torch.cuda.synchronize()
    st.capture()
    for _ in range(max(warmup, 1)):
        st.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.replay()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / steps
    st.check_capacity()
    views = []
    for c, b in zip(st.r.cams, st.r.buf):
        T = c.tile
        views.append(view_stats(b['n_contrib'].cpu().numpy().view(np.uint32),
                                b['ranges'].cpu().numpy().view(np.uint32),
                                -(-c.width // T), -(-c.height // T), T))
        views[-1]['runs'] = column_runs(b['splats'].cpu().numpy(), -(-c.width // T))
    # eager per-view loop over the same views (single-view entry points)
    q = {k: v.clone() for k, v in p.items()}
    rs = [Rasterizer(n, c, wl['sh_degree'], tile=tile) for c in cams]
    for r in rs:
        r.preprocess(q)
        P = r.bin_sort(check_overflow=True)
        r._alloc_pairs(int(P * 1.25) + 4096)
    opt = Adam(q, LRS)
    grads = {k: torch.empty_like(v) for k, v in q.items()}
    loss = torch.zeros(1, device='cuda')

    def eager_step():
        for i, r in enumerate(rs):
            r.preprocess(q)
            r.bin_sort(check_overflow=False)
            r.render_fwd()
            _, dI = l1_loss(r.image, targets[i], None, loss)
            r.backward(q, dI, None, grads, accumulate=i > 0)
        opt.step(grads)

    for _ in range(max(warmup, 1)):
        eager_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        eager_step()
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / steps
    res = {'workload': f'{n} Gaussians SH{wl["sh_degree"]}, 8 orbit views '
                       f'({", ".join(f"{c.width}x{c.height}" for c in cams)}), tile {tile}, one '
                       f'persistent launch per render phase, HIP-graph replay',
           'graph_ms_per_step': round(ms_graph, 3), 'eager_per_view_ms_per_step': round(ms_eager, 3),
           'speedup_vs_eager': round(ms_eager / ms_graph, 3),
           'pixels': sum(v['pixels'] for v in views), 'pairs': [v['P'] for v in views],
           'tuning': tuned or _lib.gs_get_tuning(),
           'step_roofline': step_roofline(step_model(n, K, views, deferred=st.r.deferred),
                                          ms_graph)}
    del st, rs, q, grads, opt
    torch.cuda.empty_cache()
    if tune:  # back to the default knobs for whatever runs next
        _lib.gs_set_tuning(fwd_px=1, bwd_px=4, persist_wgs=12, fwd_batch=0, bwd_batch=0)
    return res


def run_batch8(args):
    """The batched 8-view workload on its own line."""
    from paper_2601_19489_amd import _lib

    _lib.lib()
    b = batch8_measure(args.steps, args.warmup, args.autotune)
    out = {'metric': 'batched fwd+bwd+Adam ms/step, 8 views at mixed resolutions, 1M Gaussians',
           'value': b['graph_ms_per_step'], 'unit': 'ms/step', 'n_gpus': 1, 'steps': args.steps,
           'warmup': args.warmup, 'ms_per_step': b['graph_ms_per_step'],
           'higher_is_better': False, 'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f32',
           'data': 'synthetic', 'config': {'workload': 'batch8: ' + b['workload']}, 'batch8': b}
    print(json.dumps(out), flush=True)


def c4_measure(log=None):
    """The anchor form against plain Gaussians at the full anchor workload:
    cumulative GPU ms of training steps to come within 0.1 dB of the plain
    model's final held-out PSNR. Returns the JSON object."""
    from paper_2601_19489_amd.fit import FitConfig, compare

    wl = WORKLOADS['c4']
    cfg = FitConfig(gt_gaussians=wl['gt'], anchors=wl['anchors'], train_views=wl['train_views'],
                    test_views=wl['test_views'], width=wl['width'], height=wl['height'],
                    steps=wl['steps'], eval_every=wl['eval_every'], seed=wl['seed'],
                    gt_sh_degree=3, gt_large_frac=0.1, anchor_max_steps=wl['steps'])
    t0 = time.perf_counter()
    res = compare(cfg, log=log)
    wall = time.perf_counter() - t0
    ta, tp = res['anchor_time_to_target'], res['plain_time_to_target']
    ca, cp = res['anchor'], res['plain']
    if ta is None:
        sign = 'the anchor form does not reach the target within the step budget'
    elif ta[1] < tp[1]:
        sign = 'the anchor form reaches the target in less GPU time'
    else:
        sign = 'the plain model reaches the target in less GPU time'
    return {'workload': f'GT {wl["gt"]} Gaussians SH3 (surface cloud, 10% large), '
                        f'{wl["anchors"]} anchors x 10 children (1M Gaussians), '
                        f'{wl["train_views"]} train + {wl["test_views"]} held-out orbit views '
                        f'{wl["width"]}x{wl["height"]}; plain: {wl["steps"]} steps; anchor: until '
                        f'the target, at most {wl["steps"]} steps; held-out PSNR every '
                        f'{wl["eval_every"]} steps',
            'target_psnr': round(res['target_psnr'], 3),
            'plain_final_psnr': round(cp[-1][2], 3), 'anchor_best_psnr': round(max(p for _s, _m, p in ca), 3),
            'start_psnr': {'plain': round(cp[0][2], 3), 'anchor': round(ca[0][2], 3)},
            'plain_time_to_target_ms': None if tp is None else round(tp[1], 1),
            'anchor_time_to_target_ms': None if ta is None else round(ta[1], 1),
            'plain_steps_to_target': None if tp is None else tp[0],
            'anchor_steps_to_target': None if ta is None else ta[0],
            'sign': sign,
            'plain_ms_per_step': round(cp[-1][1] / max(cp[-1][0], 1), 4),
            'anchor_ms_per_step': round(ca[-1][1] / max(ca[-1][0], 1), 4),
            'anchor_curve': [(st, round(ms, 1), round(p, 3)) for st, ms, p in ca[::5]],
            'plain_curve': [(st, round(ms, 1), round(p, 3)) for st, ms, p in cp[::5]],
            'wall_s': round(wall, 1)}


def run_anchor(args):
    """Anchor form vs plain Gaussians fitted to views of a seeded scene:
    cumulative GPU ms of training steps to reach within 0.1 dB of the plain
    model's final held-out PSNR. One JSON line."""
    from paper_2601_19489_amd import _lib
    from paper_2601_19489_amd.fit import FitConfig, compare

    _lib.lib()
    wl = WORKLOADS['anchor']
    cfg = FitConfig(gt_gaussians=wl['gt'], anchors=wl['anchors'], train_views=wl['train_views'],
                    test_views=wl['test_views'], width=wl['width'], height=wl['height'],
                    steps=wl['steps'], eval_every=wl['eval_every'], seed=wl['seed'])
    res = compare(cfg, log=lambda m: print(m, file=sys.stderr, flush=True))
    ta, tp = res['anchor_time_to_target'], res['plain_time_to_target']
    out = {'metric': 'anchor vs plain time-to-PSNR (GPU ms to within 0.1 dB of the plain '
                     'model\'s final held-out PSNR)',
           'value': None if ta is None else round(ta[1], 1), 'unit': 'ms', 'n_gpus': 1,
           'higher_is_better': False, 'data': 'synthetic', 'dtype': 'f32+bf16',
           'config': {'workload': f'anchor: GT {wl["gt"]} Gaussians, {wl["anchors"]} anchors x 10 '
                                  f'children, {wl["train_views"]} train + {wl["test_views"]} '
                                  f'held-out views {wl["width"]}x{wl["height"]}, '
                                  f'{wl["steps"]} steps each'},
           'target_psnr': round(res['target_psnr'], 3),
           'anchor_time_to_target': ta, 'plain_time_to_target': tp,
           'anchor_curve': [(s, round(ms, 1), round(p, 3)) for s, ms, p in res['anchor']],
           'plain_curve': [(s, round(ms, 1), round(p, 3)) for s, ms, p in res['plain']]}
    print(json.dumps(out), flush=True)


def c5_measure(log=None, workload='densify'):
    """The densifying fit (1M-Gaussian ground truth, 200 views, 300k start,
    Eq. 3-6, depth L1 0.1 -> 0, 6000 steps): wall seconds of the training
    run (steps and densification events) and held-out PSNR. Returns the JSON
    object."""
    from paper_2601_19489_amd.densify_fit import DensifyConfig, DensifyFit

    wl = WORKLOADS[workload]
    cfg = DensifyConfig(gt_gaussians=wl['gt'], init_gaussians=wl['init'],
                        growth_to=wl['growth_to'], views=wl['views'], width=wl['width'],
                        height=wl['height'], steps=wl['steps'], seed=wl['seed'],
                        depth_mode=wl['depth_mode'])
    res = DensifyFit(cfg, log=log).run()
    return {'workload': f'GT {wl["gt"]} Gaussians SH3, {wl["views"]} orbit views '
                        f'{wl["width"]}x{wl["height"]} (every 8th held out), {wl["init"]} sparse '
                        f'start, growth budget towards {wl["growth_to"]} every 500 steps over '
                        f'500-4000 (K = 10 views; Eq. 4 growth, Eq. 6 pruning above 0.9), Eq. 5 '
                        f'loss (lambda 0.2), {"disparity" if wl["depth_mode"] else "depth"} L1 '
                        f'0.1 -> 0, {wl["steps"]} steps', **res}


def run_densify(args):
    """Densifying fit from a sparse start: wall seconds of the training run
    (steps and densification events, evaluation and ground-truth rendering
    excluded) and the held-out PSNR. One JSON line."""
    from paper_2601_19489_amd import _lib
    from paper_2601_19489_amd.densify_fit import DensifyConfig, DensifyFit

    _lib.lib()
    wl = WORKLOADS[args.workload]
    cfg = DensifyConfig(gt_gaussians=wl['gt'], init_gaussians=wl['init'],
                        growth_to=wl['growth_to'], views=wl['views'], width=wl['width'],
                        height=wl['height'], steps=wl['steps'], seed=wl['seed'],
                        depth_mode=wl['depth_mode'])
    fit = DensifyFit(cfg, log=lambda m: print(m, file=sys.stderr, flush=True))
    res = fit.run()
    out = {'metric': 'densifying fit wall time (s) and held-out PSNR',
           'value': res['train_seconds'], 'unit': 's', 'n_gpus': 1, 'steps': cfg.steps,
           'higher_is_better': False, 'data': 'synthetic', 'dtype': 'f32',
           'config': {'workload': f'densify: GT {wl["gt"]} Gaussians SH3, {wl["views"]} orbit '
                                  f'views {wl["width"]}x{wl["height"]} (every 8th held out), '
                                  f'{wl["init"]} sparse start grown towards {wl["growth_to"]} '
                                  f'every 500 steps over 500-4000 (K = 10 views; Eq. 4 growth, '
                                  f'Eq. 6 pruning above 0.9), Eq. 5 loss (lambda 0.2), '
                                  f'{"disparity" if wl["depth_mode"] else "depth"} L1 '
                                  f'0.1 -> 0, {wl["steps"]} steps'},
           **res}
    print(json.dumps(out), flush=True)


def _cpu_model():
    try:
        for line in open('/proc/cpuinfo'):
            if line.startswith('model name'):
                return line.split(':', 1)[1].strip()
    except OSError:
        pass
    return 'unknown'


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=20)
    ap.add_argument('--workload', default='headline', choices=sorted(WORKLOADS))
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-extras', action='store_true',
                    help='headline workload: skip the batched 8-view and anchor-vs-plain objects')
    ap.add_argument('--breakdown', action='store_true', help='print per-kernel times to stderr')
    ap.add_argument('--two-launch-step', action='store_true',
                    help='headline: time the step with the backward and Adam as two launches '
                         '(the fused form, gs_render_bwd_adam, is then timed for comparison)')
    ap.add_argument('--full-lists', action='store_true',
                    help='headline: write every tile list in the binning (gs_bin_sort + '
                         'gs_render_fwd) instead of the deferred form')
    ap.add_argument('--autotune', action='store_true', help='batch8: autotune the launch knobs')
    ap.add_argument('--copy-probe', type=int, default=0, metavar='BYTES',
                    help='only copy BYTES between two device buffers 5 times (calibrates the HBM '
                         'byte counters against a plain copy of known size) and exit')
    args = ap.parse_args()
    if args.gpus != 1:
        print(f'bench.py runs on exactly one GPU: the rasterizer step is a single-GPU kernel '
              f'pipeline and this build has no multi-GPU path (asked for --gpus {args.gpus}).',
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe:
        a = torch.ones(args.copy_probe // 4, device='cuda')
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({'copy_probe_bytes': args.copy_probe}))
        return

    from paper_2601_19489_amd import _lib, scenes
    from paper_2601_19489_amd.rasterizer import Adam, Rasterizer, l1_loss, params_to_device

    # headline workloads: the scene and the CPU baseline come first, before
    # anything loads the HIP library or touches the GPU (the oracle workers
    # are forked)
    d = cpu_base = None
    if args.workload in ('headline', 'surface500k'):
        wl = WORKLOADS[args.workload]
        t0 = time.perf_counter()
        d = scenes.surface_cloud(wl['n'], seed=wl['seed'], sh_degree=wl['sh_degree'],
                                 width=wl['width'], height=wl['height'])
        print(f'[bench] scene generated in {time.perf_counter() - t0:.1f}s', file=sys.stderr, flush=True)
        cpu_base = None
        if not args.no_cpu_baseline:
            # the oracle workers are forked, so this runs before the GPU is touched
            t = time.perf_counter()
            cpu_base = cpu_baseline(d)
            print(f'[bench] cpu baseline took {time.perf_counter() - t:.1f}s', file=sys.stderr,
                  flush=True)

    _lib.lib()  # fails loudly if the HIP library is missing
    # kernel knobs from the environment (every workload; the defaults otherwise)
    tune = {k: int(os.environ[v]) for k, v in (('fwd_px', 'GS_FWD_PX'), ('bwd_px', 'GS_BWD_PX'),
                                                ('persist_wgs', 'GS_PERSIST_WGS'))
            if v in os.environ}
    if tune:
        _lib.gs_set_tuning(**tune)

    if args.workload == 'batch8':
        run_batch8(args)
        return
    if args.workload in ('densify', 'densify_disparity'):
        run_densify(args)
        return
    if args.workload == 'anchor':
        run_anchor(args)
        return
    if args.workload == 'c4':
        c = c4_measure(log=lambda m: print(m, file=sys.stderr, flush=True))
        print(json.dumps({'metric': 'anchor vs plain time-to-PSNR (GPU ms)',
                          'value': c['anchor_time_to_target_ms'], 'unit': 'ms', 'n_gpus': 1,
                          'higher_is_better': False, 'data': 'synthetic', 'dtype': 'f32+bf16',
                          'config': {'workload': 'c4: ' + c['workload']}, 'c4': c}), flush=True)
        return

    torch.cuda.set_device(0)
    p = params_to_device(d)
    target = torch.as_tensor(d['target'], device='cuda').contiguous()
    n = wl['n']
    K = (wl['sh_degree'] + 1) ** 2
    R = Rasterizer(n, d['camera'], wl['sh_degree'], deferred=not args.full_lists)
    opt = Adam(p, LRS)
    grads = {k: torch.empty_like(v) for k, v in p.items()}
    dI = torch.empty_like(R.image)
    loss = torch.zeros(1, device='cuda')
    maxP = torch.zeros(1, dtype=torch.int64, device='cuda')

    # size the pair buffers once (one host read), with headroom for growth
    R.preprocess(p)
    P0 = R.bin_sort(check_overflow=True)
    R._alloc_pairs(int(P0 * 1.25) + 4096)

    fused = not args.two_launch_step

    def step(fused=fused):
        R.preprocess(p)
        R.bin_sort(check_overflow=False)
        R.render_fwd()
        l1_loss(R.image, target, dI, loss)
        if fused:  # backward and Adam in one pass over the parameters
            R.backward_adam(p, dI, opt)
        else:
            R.backward(p, dI, None, grads)
            opt.step(grads)
        torch.maximum(maxP, R.pair_count, out=maxP)  # one kernel (int32 promoted)

    # untimed steps of both forms of the step (first launches, clocks up),
    # then warm-up with every kernel timed to find the dominant one
    step()
    for _ in range(max(args.warmup, 1)):
        step(not fused)
    torch.cuda.synchronize()
    _lib.gs_timer_enable('*')
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    breakdown = {}
    for k in _lib.KERNELS:
        ms, cnt = _lib.gs_timer_read(k)
        if cnt:
            breakdown[k] = (ms / max(args.warmup, 1), cnt / max(args.warmup, 1))
    _lib.gs_timer_read(None)
    dominant = max(breakdown, key=lambda k: breakdown[k][0])
    print(f'[bench] warm-up done; dominant kernel {dominant}', file=sys.stderr, flush=True)

    def time_other():
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(args.steps):
            step(not fused)
        torch.cuda.synchronize()
        return (time.perf_counter() - ta) * 1e3 / args.steps

    # the other form of the step, timed just before and just after the timed
    # region (its mean is reported for comparison)
    other_before = time_other()
    # timed region: only the dominant kernel is bracketed by events
    _lib.gs_timer_enable(dominant)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_ms, dom_launches = _lib.gs_timer_read(dominant)
    _lib.gs_timer_enable(None)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    other_ms = 0.5 * (other_before + time_other())
    Pmax = int(maxP.item())
    if Pmax > R.capacity:
        raise RuntimeError(f'pair capacity overflow during timing: {Pmax} > {R.capacity}')

    # workload statistics (outside the timed region)
    P = int(R.pair_count.item())
    T = R.cam.tile
    nc = R.n_contrib.cpu().numpy().view(np.uint32)
    ranges = R.ranges.cpu().numpy().view(np.uint32)
    vs = view_stats(nc, ranges, R.tiles_x, R.tiles_y, T)
    vs['runs'] = column_runs(R.splats.cpu().numpy(), R.tiles_x)
    Pr_fwd, Pr_bwd, pixels = vs['Pr_fwd'], vs['Pr_bwd'], vs['pixels']
    evals_fwd, evals_bwd = vs['evals_fwd'], vs['evals_bwd']
    waves_pairs = Pr_bwd * (T * T // 64)

    avg = dom_ms / max(dom_launches, 1)
    if dominant in ('render_fwd', 'render_bwd'):
        units, per = ((evals_fwd, OPS_FWD) if dominant == 'render_fwd' else (evals_bwd, OPS_BWD))
        achieved = units * per / (avg * 1e-3) / 1e12
        roof = {'bound': 'alu', 'achieved': round(achieved, 2), 'peak': round(ALU_PEAK_TOPS, 1),
                'unit': 'Tops/s', 'frac': round(achieved / ALU_PEAK_TOPS, 4),
                'traffic': measured_traffic(dominant),
                'kernel': dominant, 'avg_launch_ms': round(avg, 4),
                'units_per_launch': units, 'ops_per_unit': per,
                'unit_of_work': '(pixel, splat) evaluation; op = FP32 VALU lane operation'}
        cnt = valu_counters(dominant)
        if cnt is not None:
            roof['counters'] = cnt
        prof = profile_avg_ms(dominant)
        if prof is not None:
            roof['profile_avg_ms'] = prof
            roof['frac_at_profile_avg'] = round(units * per / (prof * 1e-3) / 1e12
                                                / ALU_PEAK_TOPS, 4)
    else:
        nbytes = kernel_bytes(dominant, n, K, P, Pr_fwd, pixels, waves_pairs)
        roof = None
        if nbytes is not None:
            achieved = nbytes / (avg * 1e-3) / 1e9
            roof = {'bound': 'hbm', 'achieved': round(achieved, 1), 'peak': HBM_PEAK_GBS,
                    'unit': 'GB/s', 'frac': round(achieved / HBM_PEAK_GBS, 4),
                    'traffic': measured_traffic(dominant),
                    'kernel': dominant, 'avg_launch_ms': round(avg, 4),
                    'bytes_per_launch': int(nbytes)}
    kernel_ms = {k: v[0] for k, v in breakdown.items()}
    if roof is not None:
        roof['step'] = step_roofline(step_model(n, K, [vs], fused=fused, deferred=R.deferred),
                                     ms_per_step, kernel_ms)
    out = {
        'metric': METRIC, 'value': round(ms_per_step, 3), 'unit': 'ms/iter', 'n_gpus': 1,
        'steps': args.steps, 'warmup': args.warmup, 'ms_per_step': round(ms_per_step, 3),
        'higher_is_better': False, 'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f32',
        'data': 'synthetic',
        'config': {'workload': f'{args.workload}: {n} Gaussians SH{wl["sh_degree"]}, '
                               f'{wl["width"]}x{wl["height"]}, tile {T}, surface-cloud scene '
                               f'seed {wl["seed"]}, step = fwd + L1 + bwd + Adam'
                               + (' (backward and Adam fused)' if fused else ''),
                   'gaussians': n, 'width': wl['width'], 'height': wl['height'],
                   'sh_degree': wl['sh_degree'], 'tile': T, 'pairs': P,
                   'column_runs': vs['runs'], 'lists': 'deferred' if R.deferred else 'full',
                   'processed_pairs_fwd': Pr_fwd, 'processed_pairs_bwd': Pr_bwd,
                   'pixel_evals_fwd': evals_fwd, 'pixel_evals_bwd': evals_bwd},
        'roofline': roof,
        'kernel_ms': {k: round(v[0], 4) for k, v in sorted(breakdown.items(), key=lambda x: -x[1][0])},
        ('unfused_step_ms' if fused else 'fused_step_ms'): round(other_ms, 3),
    }
    if args.breakdown:
        for k, (ms, cnt) in sorted(breakdown.items(), key=lambda x: -x[1][0]):
            print(f'[bench] {k:16s} {ms:8.3f} ms/step  {cnt:5.1f} launches', file=sys.stderr)
    out['decoder'] = decoder_measure()
    out['densify'] = densify_measure(R, p, target)
    out['ablation'] = ablation_measure(R, p)
    del R, opt, grads, p
    torch.cuda.empty_cache()
    if not args.no_extras:
        print('[bench] batch8 (autotuned launch knobs)', file=sys.stderr, flush=True)
        out['batch8'] = batch8_measure(args.steps, args.warmup, tune=True)
        print('[bench] c4', file=sys.stderr, flush=True)
        out['c4'] = c4_measure(log=lambda m: print(m, file=sys.stderr, flush=True))
        print('[bench] c5 (densifying fit)', file=sys.stderr, flush=True)
        out['c5'] = c5_measure(log=lambda m: print(m, file=sys.stderr, flush=True))
    if cpu_base is not None:
        out['cpu_baseline'] = cpu_base
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
