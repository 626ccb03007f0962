"""GPU parity of the fused Adam step and the L1 loss kernel against the
oracle (textbook Adam in FP64; mean absolute error and its sign gradient)."""
import numpy as np
import pytest
import torch

from oracle import adam as oadam
from oracle import render as oren
from paper_2601_19489_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize('n', [1, 3, 4, 1001, 65536 + 7])
def test_adam_matches_oracle_over_steps(n):
    rng = np.random.default_rng(n)
    p0 = rng.standard_normal(n).astype(np.float32)
    gs = [rng.standard_normal(n).astype(np.float32) * 10 ** rng.uniform(-4, 1) for _ in range(5)]
    p = torch.as_tensor(p0.copy(), device='cuda')
    m = torch.zeros(n, device='cuda')
    v = torch.zeros(n, device='cuda')
    po, mo, vo = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    # the kernel receives FP32 hyper-parameters; the oracle gets the same values
    lr, b1, b2, eps = (float(np.float32(x)) for x in (1e-2, 0.9, 0.999, 1e-15))
    for k, g in enumerate(gs):
        _lib.gs_adam_step(p, torch.as_tensor(g, device='cuda'), m, v, n, lr, b1, b2, eps, k + 1)
        po, mo, vo = oadam.adam_step(po, g, mo, vo, lr, b1, b2, eps, k + 1)
    torch.cuda.synchronize()
    # FP32 moving averages: a few ulps of the largest term they average
    gmax = max(float(np.abs(g).max()) for g in gs)
    np.testing.assert_allclose(p.cpu().numpy(), po, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(m.cpu().numpy(), mo, rtol=1e-5, atol=1e-6 * gmax)
    np.testing.assert_allclose(v.cpu().numpy(), vo, rtol=1e-5, atol=1e-6 * gmax * gmax)


def test_adam_rejects_bad_arguments():
    x = torch.zeros(8, device='cuda')
    with pytest.raises(RuntimeError):
        _lib.gs_adam_step(x, x, x, x, 8, 1e-3, 0.9, 0.999, 1e-8, 0)  # step must be >= 1
    with pytest.raises(RuntimeError):
        _lib.gs_adam_step(x[1:], x[1:], x[1:], x[1:], 7, 1e-3, 0.9, 0.999, 1e-8, 1)  # unaligned


@pytest.mark.parametrize('shape', [(3, 64, 64), (3, 1066, 1600), (3, 7, 5)])
def test_l1_loss_matches_oracle(shape):
    rng = np.random.default_rng(sum(shape))
    img = rng.uniform(0, 1, shape).astype(np.float32)
    tgt = rng.uniform(0, 1, shape).astype(np.float32)
    tgt.ravel()[::17] = img.ravel()[::17]  # exact ties: gradient 0
    ti = torch.as_tensor(img, device='cuda')
    tt = torch.as_tensor(tgt, device='cuda')
    grad = torch.empty_like(ti)
    loss = torch.zeros(1, device='cuda')
    _lib.gs_l1_loss(ti, tt, img.size, grad, loss)
    torch.cuda.synchronize()
    lo, go = oren.l1_loss_grad(img, tgt)
    assert abs(loss.item() - lo) <= 1e-5 * lo
    np.testing.assert_array_equal(grad.cpu().numpy(), go.astype(np.float32))
