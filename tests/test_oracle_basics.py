"""Pins of the oracle's building blocks against libraries and closed forms:
SH basis (scipy), rotation matrices (scipy), Adam (torch), L1 gradient
(torch autograd)."""
import math

import numpy as np
import pytest
import scipy.special as ss
from scipy.spatial.transform import Rotation

from oracle import adam, preprocess, render, sh


def _sphere_dirs(n, seed=0):
    d = np.random.default_rng(seed).standard_normal((3, n))
    return d / np.linalg.norm(d, axis=0)


def test_sh_matches_scipy_complex_harmonics():
    # real form of scipy's complex Y_l^m (which carries the Condon-Shortley
    # phase): sqrt(2) Re Y_l^|m| for m > 0, sqrt(2) Im Y_l^|m| for m < 0
    dirs = _sphere_dirs(500)
    x, y, z = dirs
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    Y = sh.basis(dirs, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            Yc = ss.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                ref = math.sqrt(2) * Yc.real
            elif m < 0:
                ref = math.sqrt(2) * Yc.imag
            else:
                ref = Yc.real
            np.testing.assert_allclose(Y[l * l + l + m], ref, atol=1e-12, rtol=0)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi integrates degree <= 6
    # polynomials exactly
    nt, nphi = 12, 24
    ct, wt = np.polynomial.legendre.leggauss(nt)
    phi = 2 * np.pi * np.arange(nphi) / nphi
    CT, PHI = np.meshgrid(ct, phi, indexing='ij')
    ST = np.sqrt(1 - CT ** 2)
    dirs = np.stack([ST * np.cos(PHI), ST * np.sin(PHI), CT]).reshape(3, -1)
    w = (wt[:, None] * np.full(nphi, 2 * np.pi / nphi)[None]).ravel()
    Y = sh.basis(dirs, 3)
    G = (Y * w) @ Y.T
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_degree0_constant():
    Y = sh.basis(_sphere_dirs(10), 0)
    np.testing.assert_allclose(Y[0], 0.5 / math.sqrt(math.pi), rtol=0, atol=1e-15)


def test_sh_gradient_by_central_differences():
    dirs = _sphere_dirs(50, seed=3) * 1.3  # off-sphere points: polynomials only
    dY = sh.basis_grad(dirs, 3)
    h = 1e-6
    for a in range(3):
        e = np.zeros((3, 1)); e[a] = h
        fd = (sh.basis(dirs + e, 3) - sh.basis(dirs - e, 3)) / (2 * h)
        np.testing.assert_allclose(dY[:, a], fd, atol=1e-8)


def test_rotation_matches_scipy():
    q = np.random.default_rng(1).standard_normal((4, 200))
    q /= np.linalg.norm(q, axis=0)
    R = preprocess.quat_to_rotmat(q)
    ref = Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], axis=1)).as_matrix()
    np.testing.assert_allclose(R, ref, atol=1e-14)
    np.testing.assert_allclose(R @ np.transpose(R, (0, 2, 1)), np.broadcast_to(np.eye(3), R.shape),
                               atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)


def test_rotation_axis_angle_closed_form():
    # rotation by angle th about z: q = (cos th/2, 0, 0, sin th/2)
    th = 0.7
    q = np.array([[math.cos(th / 2)], [0.0], [0.0], [math.sin(th / 2)]])
    R = preprocess.quat_to_rotmat(q)[0]
    ref = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    np.testing.assert_allclose(R, ref, atol=1e-15)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(100)
    grads = [rng.standard_normal(100) for _ in range(4)]
    tp = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(100), np.zeros(100)
    for k, g in enumerate(grads):
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = adam.adam_step(p, g, m, v, 1e-2, 0.9, 0.999, 1e-8, k + 1)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    p, _, _ = adam.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 0.1, 0.9, 0.999, 1e-15, 1)
    np.testing.assert_allclose(p, -0.1 * g / (np.abs(g) + 1e-15), rtol=1e-12)


def test_l1_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    img = rng.uniform(0, 1, (3, 5, 6))
    tgt = rng.uniform(0, 1, (3, 5, 6))
    tgt[0, 0, 0] = img[0, 0, 0]  # sign(0) = 0
    loss, g = render.l1_loss_grad(img, tgt)
    ti = torch.tensor(img, requires_grad=True)
    tl = torch.nn.functional.l1_loss(ti, torch.tensor(tgt))
    tl.backward()
    assert abs(loss - tl.item()) < 1e-15
    np.testing.assert_allclose(g, ti.grad.numpy(), atol=0)
