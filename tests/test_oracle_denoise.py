"""Pins of the FP64 denoiser reference (oracle/denoise.py) against what
mathematics and independent library routines fix: torch's own conv3d and
autograd (FP64, CPU) as a second implementation of the convolution, central
finite differences of the whole loss, hand-expanded curl stencils, the
Fourier symbol of the binomial filter, the closed-form first Adam step and
the IEEE round-to-nearest-even definition of bfloat16."""
import numpy as np
import pytest
import torch
import torch.nn.functional as tF

import workloads
from oracle import denoise as dn


def _torch_conv(x, W, b):
    t = torch.from_numpy(x)[None]
    t = tF.pad(t, (1, 1, 1, 1, 0, 0), mode="circular")     # x, y periodic
    t = tF.pad(t, (0, 0, 0, 0, 1, 1))                       # zeta: zeros
    return tF.conv3d(t, torch.from_numpy(W), torch.from_numpy(b))[0].numpy()


def test_conv3d_matches_torch():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 5, 4, 6))
    W = rng.standard_normal((5, 3, 3, 3, 3))
    b = rng.standard_normal(5)
    assert np.allclose(dn.conv3d(x, W, b), _torch_conv(x, W, b), rtol=1e-13, atol=1e-13)


def test_conv3d_backward_matches_torch_autograd():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 3, 4, 5))
    W = rng.standard_normal((6, 4, 3, 3, 3))
    b = rng.standard_normal(6)
    gy = rng.standard_normal((6, 3, 4, 5))
    tx = torch.from_numpy(x).requires_grad_()
    tW = torch.from_numpy(W).requires_grad_()
    tb = torch.from_numpy(b).requires_grad_()
    t = tF.pad(tF.pad(tx[None], (1, 1, 1, 1, 0, 0), mode="circular"), (0, 0, 0, 0, 1, 1))
    (tF.conv3d(t, tW, tb)[0] * torch.from_numpy(gy)).sum().backward()
    gx, gW, gb = dn.conv3d_backward(x, W, gy)
    for mine, ref in ((gx, tx.grad), (gW, tW.grad), (gb, tb.grad)):
        assert np.allclose(mine, ref.numpy(), rtol=1e-12, atol=1e-12)


def test_identity_and_shift_kernels():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 4, 5, 6))
    W = np.zeros((1, 1, 3, 3, 3))
    W[0, 0, 1, 1, 1] = 1.0
    assert np.array_equal(dn.conv3d(x, W, np.array([0.5])), x + 0.5)
    # tap (kz, ky, kx) = (2, 0, 2) reads x[z + 1, y - 1, x + 1]
    W = np.zeros((1, 1, 3, 3, 3))
    W[0, 0, 2, 0, 2] = 1.0
    y = dn.conv3d(x, W, np.zeros(1))[0]
    for z, yy, xx in ((0, 0, 0), (2, 3, 5), (3, 1, 1)):
        want = x[0, z + 1, (yy - 1) % 5, (xx + 1) % 6] if z + 1 < 4 else 0.0
        assert y[z, yy, xx] == want


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(4)
    theta = workloads.denoiser_init(seed=5, last_scale=1.0, bias_scale=0.1).astype(np.float64)
    Z, Y, X = 6, 4, 4
    Jraw = rng.standard_normal((3, Z, Y, X)) * 0.01
    Jt = rng.standard_normal((3, Z, Y, X)) * 0.01
    args = dict(n_e=0.01, hx=0.4 * 2 * np.pi, hy=0.4 * 2 * np.pi, h=0.05 * 2 * np.pi,
                region=(1, 5))
    loss, g = dn.loss_and_grad(theta, Jraw, Jt, **args)
    offs = np.cumsum([0] + [co * ci * 27 + co for ci, co in dn.LAYERS])
    idx = np.concatenate([rng.choice(np.arange(offs[l], offs[l + 1]), 12, replace=False)
                          for l in range(4)])
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (dn.loss_and_grad(tp, Jraw, Jt, **args)[0]
              - dn.loss_and_grad(tm, Jraw, Jt, **args)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * np.abs(g).max()), (i, fd, g[i])


def test_curl_single_face_hand_expanded():
    Z, Y, X = 4, 3, 5
    hx, hy, h = 2.0, 3.0, 0.5
    A = np.zeros((3, Z, Y, X))
    A[1, 1, 1, 2] = 1.0                          # A_y on one face
    C = dn.curl(A, hx, hy, h)
    want = np.zeros_like(C)
    want[0, 1, 1, 2] = -1.0 / h                 # -(d/dz) A_y on J_x
    want[0, 2, 1, 2] = +1.0 / h
    want[2, 1, 1, 2] = +1.0 / hx                # (d/dx) A_y on J_z
    want[2, 1, 1, 3] = -1.0 / hx
    assert np.array_equal(C, want)
    A = np.zeros((3, Z, Y, X))
    A[2, 2, 0, 4] = 1.0                          # A_z, periodic neighbours
    C = dn.curl(A, hx, hy, h)
    want = np.zeros_like(C)
    want[0, 2, 0, 4] = 1.0 / hy
    want[0, 2, 1, 4] = -1.0 / hy
    want[1, 2, 0, 4] = -1.0 / hx
    want[1, 2, 0, 0] = 1.0 / hx
    assert np.array_equal(C, want)


def test_curl_is_divergence_free_and_adjoint():
    rng = np.random.default_rng(6)
    A = rng.standard_normal((3, 5, 4, 6))
    G = rng.standard_normal((3, 5, 4, 6))
    hx, hy, h = 2.5, 2.5, 0.3
    C = dn.curl(A, hx, hy, h)
    assert np.abs(dn.divergence(C, hx, hy, h)).max() < 1e-13 * np.abs(C).max() / h
    assert abs(np.sum(G * C) - np.sum(dn.curl_adjoint(G, hx, hy, h) * A)) < 1e-12 * np.sum(np.abs(G * C))


def test_binomial_symbol_and_zeta_ghosts():
    Z, Y, X = 5, 8, 16
    m = 3
    xs = np.arange(X)
    J = np.zeros((3, Z, Y, X))
    J[:, 2] = np.cos(2 * np.pi * m * xs / X)[None, None, :]
    F = dn.binomial(J)
    c2 = np.cos(np.pi * m / X) ** 2
    # x symbol cos^2(k h / 2), y constant, zeta 1-2-1 on a single plane
    assert np.allclose(F[:, 2], 0.5 * c2 * J[:, 2], atol=1e-15)
    assert np.allclose(F[:, 1], 0.25 * c2 * J[:, 2], atol=1e-15)
    assert np.allclose(F[:, 3], 0.25 * c2 * J[:, 2], atol=1e-15)
    assert not F[:, 0].any() and not F[:, 4].any()
    K = np.zeros((1, 3, 2, 4))
    K[0, 0] = 1.0                        # plane 0: the ghost below it is zero
    assert np.allclose(dn.binomial(K)[0, 0], 0.5)


def test_adam_first_step_closed_form():
    g = np.array([3.0, -1e-3, 0.0, 2.5e4])
    th = np.array([1.0, 2.0, 3.0, 4.0])
    new, m, v = dn.adam(th, np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    assert np.allclose(new, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # and it minimises a quadratic
    th = np.array([5.0, -3.0])
    m = v = np.zeros(2)
    for t in range(1, 3001):
        th, m, v = dn.adam(th, m, v, 2.0 * th, t, lr=0.05)
    assert np.abs(th).max() < 1e-3


def test_bf16_rounding():
    vals = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -7 + 2.0 ** -9), 3.0e-30])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, -(1 + 2.0 ** -7), None], dtype=object)
    got = dn.bf16(vals)
    for a, b in zip(got[:4], want[:4]):
        assert a == b
    rng = np.random.default_rng(7)
    r = rng.standard_normal(10000).astype(np.float32) * 10.0 ** rng.integers(-20, 20, 10000)
    ref = torch.from_numpy(r).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(dn.bf16(r), ref)


def test_apply_keeps_continuity_of_filtered_current():
    rng = np.random.default_rng(8)
    theta = workloads.denoiser_init(seed=1, last_scale=1.0, bias_scale=0.1).astype(np.float64)
    Jraw = rng.standard_normal((3, 6, 8, 8)) * 0.01
    J, A, Jf, _ = dn.apply(theta, Jraw, 0.01, 2.5, 2.5, 0.3)
    assert np.abs(A).max() > 0
    assert dn.continuity_rel(J, Jf, 2.5, 2.5, 0.3) < 1e-13
