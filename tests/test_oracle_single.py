"""Pins of the oracle's iterated box spline beta^{4,m}_a (eq. (iterated_spline)) and of
its single-pass filter, against what the paper and the mathematics fix:

* m = 1 is beta^4_a, evaluated by an independent routine (polygon clipping);
* the Fourier transform is prod_k sinc^m(a_k u_k.w / 2) (eq. (conv2));
* mass 1, central symmetry, and covariance m times that of beta^4_a (a sum of m
  independent copies; Sec. 3.3 uses the a / sqrt(m) rescaling that keeps it);
* the m-fold convolution of the ZP element is a partition of unity (its directions
  are lattice vectors);
* the fast single pass (m-fold running sums, (m+1)^4 differences, ZP^{*m}
  interpolation) equals the direct sum sum_k f[k] beta^{4,m}_{a(n)}(n - k).

Quadrature: the sum over a uniform grid of step h of a compactly supported function
times e^{-i w.x} is exact up to the aliases F(w + 2 pi k / h), k != 0; with h = 1/8
they are below 1e-6 of F(0) for the scales used (prod sinc^m decays like |w|^(-2m)
along the lattice axes).
"""
import math

import numpy as np
import pytest

SQ2 = math.sqrt(2.0)
U = np.array([[1.0, 0.0], [1 / SQ2, 1 / SQ2], [0.0, 1.0], [-1 / SQ2, 1 / SQ2]])


def grid(orc, a, m, h=0.125):
    rx = m * 0.5 * (a[0] + (a[1] + a[3]) / SQ2)
    ry = m * 0.5 * (a[2] + (a[1] + a[3]) / SQ2)
    xs = np.arange(-math.ceil(rx / h), math.ceil(rx / h) + 1) * h + 1e-9
    ys = np.arange(-math.ceil(ry / h), math.ceil(ry / h) + 1) * h + 2e-9
    B = np.array([[orc.boxspline_m(a, m, x, y) for x in xs] for y in ys])
    return xs[None, :], ys[:, None], B, h * h


def test_m1_is_beta4(orc):
    rng = np.random.default_rng(11)
    for a in [(1.3, 2.1, 1.7, 0.9), (0.6, 3.0, 2.2, 1.4), (1.0, SQ2, 1.0, SQ2)]:
        for x, y in rng.uniform(-3, 3, (150, 2)):
            assert orc.boxspline_m(a, 1, x, y) == pytest.approx(orc.boxspline(a, x, y), abs=2e-15)


@pytest.mark.parametrize("m,a", [(2, (1.3, 2.1, 1.7, 0.9)), (2, (2.0, 0.8, 1.1, 1.9)), (3, (1.1, 1.2, 0.9, 1.4))])
def test_fourier_mass_covariance(orc, m, a):
    X, Y, B, dA = grid(orc, a, m)
    assert B.min() >= -1e-15
    assert (B * dA).sum() == pytest.approx(1.0, abs=2e-6)
    for w in [(0.7, 0.0), (0.0, 1.1), (0.9, -0.6), (1.7, 0.4), (-0.5, 2.3)]:
        F = (B * np.exp(-1j * (w[0] * X + w[1] * Y))).sum() * dA
        ref = 1.0
        for k in range(4):
            t = 0.5 * a[k] * (U[k] @ np.array(w))
            ref *= (math.sin(t) / t if t != 0 else 1.0) ** m
        assert abs(F - ref) < 2e-6, (w, F, ref)
    cov = np.array([[(B * X * X).sum(), (B * X * Y).sum()], [(B * X * Y).sum(), (B * Y * Y).sum()]]) * dA
    ref = m * sum(a[k] ** 2 / 12.0 * np.outer(U[k], U[k]) for k in range(4))
    assert np.abs(cov - ref).max() < 2e-5


def test_central_symmetry(orc):
    rng = np.random.default_rng(12)
    a = (1.4, 0.9, 2.2, 1.6)
    for x, y in rng.uniform(-4, 4, (60, 2)):
        assert orc.boxspline_m(a, 2, x, y) == pytest.approx(orc.boxspline_m(a, 2, -x, -y), abs=1e-15)


@pytest.mark.parametrize("m", [2, 3])
def test_zp_power_partition_of_unity(orc, m):
    rng = np.random.default_rng(13)
    r = 2 * m
    for y in rng.random((8, 2)):
        s = sum(orc.zp_m(m, y[0] - i, y[1] - j) for i in range(-r, r + 2) for j in range(-r, r + 2))
        assert s == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("m,shape,lo,hi", [(2, (9, 11), 0.9, 2.4), (2, (6, 5), 1.6, 3.0), (3, (5, 6), 1.0, 1.8)])
def test_fast_equals_direct_sum(orc, m, shape, lo, hi):
    rng = np.random.default_rng(14 + m)
    img = rng.uniform(0, 1, shape)
    a = rng.uniform(lo, hi, shape + (4,))
    b = orc.pass_single(img, a, m, "brute")
    f = orc.pass_single(img, a, m, "fast")
    # the m-fold window sums lose about eps * (window / a)^(4m) of the output scale
    assert np.abs(f - b).max() < 1e-8


def test_direct_sum_of_delta_is_the_kernel(orc):
    img = np.zeros((15, 15))
    img[7, 7] = 1.0
    a = np.broadcast_to(np.array([1.2, 1.9, 0.8, 1.3]), (15, 15, 4)).copy()
    out = orc.pass_single(img, a, 2, "brute")
    for r, c in [(7, 7), (5, 8), (9, 4), (3, 7)]:
        assert out[r, c] == pytest.approx(orc.boxspline_m(a[0, 0], 2, c - 7, r - 7), abs=1e-15)
