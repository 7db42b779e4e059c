"""Pins of the oracle's gather + push against closed forms.

* Gyration in a uniform B: |u| is exact and the Higuera-Cary step is a
  rotation by 2 arctan(|beta| / gamma+) in the sense an electron gyrates.
* Crossed uniform E and B: the E x B drift state is an exact fixed point and a
  particle starting at rest drifts, on average, with v_d = E x B / B^2.
* Plane wave (the paper's single-electron example, Sec. 2, Fig. 1): for
  A_x = a0 cos(zeta) exp(-zeta^2 / 2 sigma^2), E_x = B_y = A_x'(zeta), an
  electron starting at rest has u_x = A_x, gamma - u_z = 1, and is at rest again
  after the pulse; the scheme's error is second order in (h, dtau).
* FP32 fused multiply-add: equal to the exact a b + c rounded once to the
  nearest FP32 number (exact rational arithmetic), including cases where a
  product rounded first, or a sum rounded first to FP64, gives another result.
"""
import math

import numpy as np
import pytest

from oracle import params
from oracle.plasma import Particles
from fractions import Fraction

from oracle.push import fma32, higuera_cary, madd, push_and_move, renormalise, velocities


def test_gyration_exact_rotation():
    dtau, B0, u0 = 0.3, 10.0, 0.5
    eps = -0.5 * dtau                      # electron: q/m = -1
    ux, uy, uz = np.array([u0]), np.array([0.0]), np.array([0.0])
    E = np.zeros((3, 1))
    B = np.array([[0.0], [0.0], [B0]])
    g = math.sqrt(1 + u0 * u0)
    beta = abs(eps * B0)
    sigma = g * g - beta * beta
    gplus = math.sqrt(0.5 * (sigma + math.sqrt(sigma * sigma + 4 * beta * beta)))
    theta = 2.0 * math.atan(beta / gplus)
    ang = 0.0
    for k in range(1, 201):
        ux, uy, uz = higuera_cary(ux, uy, uz, E, B, eps)
        ang += theta
        assert abs(math.hypot(ux[0], uy[0]) - u0) < 1e-15 * k * u0 + 1e-15
        assert uz[0] == 0.0
        if k == 1:
            # electron in +z field turns from +x towards +y
            assert uy[0] > 0
            assert abs(ux[0] - u0 * math.cos(theta)) < 1e-14
            assert abs(uy[0] - u0 * math.sin(theta)) < 1e-14
    # accumulated phase after 200 steps
    assert abs(math.atan2(uy[0], ux[0]) - math.atan2(math.sin(ang), math.cos(ang))) < 1e-11
    # Boris would rotate by 2 arctan(beta / gamma) instead: the HC angle differs
    assert abs(theta - 2.0 * math.atan(beta / g)) > 1e-3


def test_exb_drift_is_a_fixed_point():
    E0, B0 = 0.9, 1.0
    vd = -E0 / B0                          # E x B / B^2 = (E0 x) x (B0 z) / B0^2 = -E0/B0 y
    gd = 1.0 / math.sqrt(1.0 - vd * vd)
    u = [np.array([0.0]), np.array([gd * vd]), np.array([0.0])]
    E = np.array([[E0], [0.0], [0.0]])
    B = np.array([[0.0], [0.0], [B0]])
    for _ in range(200):
        u = list(higuera_cary(*u, E, B, -0.5 * 0.2))
    assert abs(u[0][0]) < 1e-13 and abs(u[2][0]) < 1e-13
    assert abs(u[1][0] - gd * vd) < 1e-13 * gd


def test_exb_from_rest_average_drift():
    E0, B0, dtau = 0.02, 1.0, 0.02
    vd = -E0 / B0
    u = [np.array([0.0]), np.array([0.0]), np.array([0.0])]
    E = np.array([[E0], [0.0], [0.0]])
    B = np.array([[0.0], [0.0], [B0]])
    # gyro-period in the drift frame ~ 2 pi gamma / B; average over 20 periods
    steps = int(round(20 * 2 * math.pi / dtau))
    vy = 0.0
    for _ in range(steps):
        u = list(higuera_cary(*u, E, B, -0.5 * dtau))
        g, _, v, _ = velocities(*u)
        vy += v[0]
    assert abs(vy / steps - vd) < 2e-3 * abs(vd)


def test_renormalise_cell_steps():
    d = np.array([0.2, 0.9, 0.1, 0.5, 0.0])
    s = np.array([0.3, 0.2, -0.3, -0.5, -1e-18])
    t, k = renormalise(d, s)
    assert list(k) == [0, 1, -1, 0, -1] or list(k) == [0, 1, -1, 0, 0]
    assert np.all((t >= 0) & (t < 1))
    # the value that rounds to 1.0 goes to the next cell with offset 0
    t, k = renormalise(np.array([0.0]), np.array([-1e-18]))
    assert k[0] == 0 and t[0] == 0.0


def _plane_wave_run(h, a0=1.0, sigma=3.0):
    Nz = int(round(48.0 / h))
    Nz = 1 << int(math.ceil(math.log2(Nz)))
    cfg = dict(dims=2, n=[8, 1, Nz], d=[1.0, 1.0, h], length_unit=1.0, n_e=0.0,
               tile=[8, 1, 8], filter_passes=1)
    p = params.from_config(cfg)
    zc = 24.0
    zeta = np.arange(Nz + p.ext + 1) * h - zc

    def A(z):
        return a0 * np.cos(z) * np.exp(-z * z / (2 * sigma * sigma))

    def dA(z):
        return a0 * np.exp(-z * z / (2 * sigma * sigma)) * (-np.sin(z) - z * np.cos(z) / sigma ** 2)

    F = np.zeros((6, Nz + p.ext + 1, 1, 8))
    F[0] = dA(zeta)[:, None, None]
    F[4] = dA(zeta)[:, None, None]
    F[:, Nz:] = 0.0
    z0 = zc + 7 * sigma
    P = Particles(ix=np.array([3]), iy=np.array([0]), iz=np.array([int(z0 / h)]),
                  dx=np.array([0.25]), dy=np.array([0.0]), dz=np.array([z0 / h - int(z0 / h)]),
                  ux=np.array([0.0]), uy=np.array([0.0]), uz=np.array([0.0]),
                  pid=np.array([0]))
    err_ux = err_inv = 0.0
    while True:
        zold = (P.iz[0] + P.dz[0]) * h
        push_and_move(p, P, F)
        znew = (P.iz[0] + P.dz[0]) * h
        zmid = 0.5 * (zold + znew) - zc
        g = math.sqrt(1 + P.ux[0] ** 2 + P.uy[0] ** 2 + P.uz[0] ** 2)
        err_ux = max(err_ux, abs(P.ux[0] - A(zmid)))
        err_inv = max(err_inv, abs(g - P.uz[0] - 1.0))
        if znew - zc < -7 * sigma:
            break
    return err_ux, err_inv, abs(P.ux[0]) + abs(P.uz[0])


def test_plane_wave_electron_closed_form_and_order():
    e1 = _plane_wave_run(0.1)
    e2 = _plane_wave_run(0.05)
    # closed-form orbit to second order
    assert e1[0] < 3e-3 and e1[1] < 3e-3
    # at rest after the pulse
    assert e2[2] < 1e-4
    # second order: halving (h, dtau) divides the error by ~4
    assert 3.0 < e1[0] / e2[0] < 5.0
    assert 3.0 < e1[1] / e2[1] < 5.0


def _round_binary32(x):
    """Exact rational -> nearest binary32 (ties to even), normal range."""
    if x == 0:
        return 0.0
    sign = -1 if x < 0 else 1
    x = abs(x)
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1
    elif Fraction(2) ** (e + 1) <= x:
        e += 1
    m = x / Fraction(2) ** (e - 23)          # in [2^23, 2^24)
    q = m.numerator // m.denominator
    r = m - q
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and q % 2 == 1):
        q += 1
    return sign * float(Fraction(q) * Fraction(2) ** (e - 23))


def test_fma32_is_the_exact_value_rounded_once():
    rng = np.random.default_rng(7)
    n = 4000
    a = (rng.standard_normal(n) * 2.0 ** rng.integers(-20, 20, n)).astype(np.float32)
    b = (rng.standard_normal(n) * 2.0 ** rng.integers(-20, 20, n)).astype(np.float32)
    c = (rng.standard_normal(n) * 2.0 ** rng.integers(-40, 40, n)).astype(np.float32)
    # heavy cancellation: c close to -a b
    k = n // 4
    c[:k] = -(a[:k] * b[:k]) * (1 + rng.integers(-4, 5, k) * 2.0 ** -23)
    one = np.float32(1 + 2.0 ** -12)
    hard_a = np.array([one, one, one], np.float32)
    hard_c = np.array([2.0 ** -30, 2.0 ** -60, -(2.0 ** -60)], np.float32)
    a = np.concatenate([a, hard_a])
    b = np.concatenate([b, hard_a])
    c = np.concatenate([c, hard_c])
    got = fma32(a, b, c)
    want = np.array([_round_binary32(Fraction(float(x)) * Fraction(float(y)) + Fraction(float(z)))
                     for x, y, z in zip(a, b, c)], np.float32)
    assert np.array_equal(got, want)
    # (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24: the product alone is a tie, so the
    # addend decides; rounding the product first, or the sum to FP64 first,
    # loses it
    assert got[-3] == np.float32(1 + 2.0 ** -11 + 2.0 ** -23)
    assert (a[-3] * b[-3]) + c[-3] == np.float32(1 + 2.0 ** -11)
    assert got[-2] == np.float32(1 + 2.0 ** -11 + 2.0 ** -23)
    assert np.float32(np.float64(a[-2]) * np.float64(b[-2]) + np.float64(c[-2])) == np.float32(1 + 2.0 ** -11)
    assert got[-1] == np.float32(1 + 2.0 ** -11)


def test_madd_fp64_is_product_then_sum():
    rng = np.random.default_rng(8)
    a, b, c = rng.standard_normal((3, 1000))
    assert np.array_equal(madd(a, b, c), a * b + c)
    assert madd(a.astype(np.float32), b.astype(np.float32), c.astype(np.float32)).dtype == np.float32
