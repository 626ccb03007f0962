"""End-to-end densifying fit at a small size (depth term, Eq. 3-4 growth):
every event's device threshold equals the oracle's growth threshold on the
same counts, growth stays within each event's budget, and the held-out
PSNR improves from the sparse grey start."""
import numpy as np
import pytest

from oracle import densify as oden
from paper_2601_19489_amd.densify_fit import DensifyConfig, DensifyFit

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize('depth_mode', [0, 1])
def test_small_densifying_fit(depth_mode):
    # depth_mode 1 supervises the blended inverse depth (disparity)
    cfg = DensifyConfig(gt_gaussians=20_000, init_gaussians=3_000, growth_to=12_000, views=24,
                        holdout_every=8, width=160, height=120, sh_degree=1, steps=300,
                        densify_from=50, densify_until=200, densify_every=50, k_views=4,
                        min_score=1.0, depth_mode=depth_mode)
    fit = DensifyFit(cfg, log=print)
    seen = []

    def check(score, t_min, cap, thr):
        counts = score.cpu().numpy().view(np.uint32).astype(np.int64)
        want = oden.growth_threshold(counts, t_min, cap)
        assert thr == want, (t_min, cap, thr, want)
        seen.append((int(np.sum(counts >= thr)) if thr != oden.NO_THRESHOLD else 0, cap))

    fit.on_event = check
    res = fit.run()
    print(res)
    assert len(res['events']) == 4 and len(seen) == 4
    for ev, (selected, cap) in zip(res['events'], seen):
        assert selected <= cap
        assert ev['n_out'] == ev['n_in'] + selected
    assert cfg.init_gaussians < res['gaussians_final'] <= cfg.growth_to
    assert res['psnr_final'] > res['psnr_init'] + 3.0
