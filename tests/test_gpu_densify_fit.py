"""End-to-end densifying fit at a small size (Eq. 5 loss, depth or disparity
term, Eq. 3-4 growth, Eq. 6 pruning): every event's device threshold equals
the oracle's growth threshold on the same counts, each event's output count
equals the growth it selected minus the Gaussians the oracle's pruning rule
removes (on the same scores), growth stays within the event's budget, and
the held-out PSNR improves from the sparse grey start."""
import numpy as np
import pytest

from oracle import densify as oden
from oracle import ssim as ossim
from paper_2601_19489_amd.densify_fit import DensifyConfig, DensifyFit

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize('depth_mode,ssim_lambda,prune', [(0, 0.0, None), (1, 0.2, None),
                                                          (0, 0.2, 0.6)])
def test_small_densifying_fit(depth_mode, ssim_lambda, prune):
    # depth_mode 1 supervises the blended inverse depth (disparity)
    cfg = DensifyConfig(gt_gaussians=20_000, init_gaussians=3_000, growth_to=12_000, views=24,
                        holdout_every=8, width=160, height=120, sh_degree=1, steps=300,
                        densify_from=50, densify_until=200, densify_every=50, k_views=4,
                        min_score=1.0, depth_mode=depth_mode, ssim_lambda=ssim_lambda,
                        prune_threshold=prune)
    fit = DensifyFit(cfg, log=print)
    seen = []

    def check(ev):
        counts = ev['score'].cpu().numpy().view(np.uint32).astype(np.int64)
        thr = ev['threshold']
        want = oden.growth_threshold(counts, ev['t_min'], ev['cap'])
        assert thr == want, (ev['t_min'], ev['cap'], thr, want)
        grow = counts >= thr if (thr != oden.NO_THRESHOLD and ev['cap'] > 0) else \
            np.zeros(len(counts), bool)
        gone = np.zeros(len(counts), bool)
        if prune is not None:
            pscore = ev['prune'].cpu().numpy()
            assert np.all(pscore >= 0)
            gone = ossim.prune_mask(pscore, prune)
        seen.append((int(np.sum(grow & ~gone)), int(np.sum(gone)), ev['cap']))

    fit.on_event = check
    res = fit.run()
    print({k: v for k, v in res.items() if k != 'events'})
    assert len(res['events']) == 4 and len(seen) == 4
    for ev, (grown, removed, cap) in zip(res['events'], seen):
        assert grown <= cap
        assert ev['n_out'] == ev['n_in'] + grown - removed
    if prune is not None:
        assert sum(r for _, r, _ in seen) > 0
    assert cfg.init_gaussians < res['gaussians_final'] <= cfg.growth_to
    assert res['psnr_final'] > res['psnr_init'] + 3.0
