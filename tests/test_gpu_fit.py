"""Training with the kernels end to end (Sec. 2.3): the anchor form (decoder
forward/backward inside the loop) and plain Gaussians fit held-out views of
a seeded ground-truth scene from the same start. The plain model trains 600
steps; the anchor form trains until it comes within 0.1 dB of the plain
model's final held-out PSNR (at most 1200 steps).

The test asserts the measured sign of what the trained network gains: the
anchor form learns faster at first (it leads by about 1 dB after 120
steps), but plain Gaussians overtake it, and the anchor form needs more GPU
time to reach the plain model's final PSNR (about 1.5 s against 0.43 s on
this scene)."""
import json

import pytest

from paper_2601_19489_amd.fit import FitConfig, compare

pytestmark = pytest.mark.gpu


def _at(curve, step):
    return next(p for s, _ms, p in curve if s == step)


def test_anchor_form_leads_early_and_plain_gaussians_reach_the_target_sooner():
    cfg = FitConfig(gt_gaussians=20_000, anchors=2_000, train_views=16, test_views=4, width=160,
                    height=160, steps=600, eval_every=40, anchor_max_steps=1200)
    res = compare(cfg)
    a, p = res['anchor'], res['plain']
    print(json.dumps({k: v for k, v in res.items()}))
    # the same start: at step 0 the decoded children do not depend on the
    # view (zero view-direction weights) and the plain model holds exactly
    # them, up to the FP32 roundings of its parametrisation (log scale,
    # opacity logit, degree-0 SH)
    assert abs(a[0][2] - p[0][2]) < 0.05, (a[0], p[0])
    # both learn
    assert a[-1][2] > a[0][2] + 3.0, a
    assert p[-1][2] > p[0][2] + 3.0, p
    # the anchor form's early lead
    assert _at(a, 120) > _at(p, 120) + 0.5, (_at(a, 120), _at(p, 120))
    # the plain model's final PSNR - 0.1 dB: reached sooner by plain Gaussians
    ta, tp = res['anchor_time_to_target'], res['plain_time_to_target']
    assert tp is not None
    assert ta is None or ta[1] > tp[1], (ta, tp)
