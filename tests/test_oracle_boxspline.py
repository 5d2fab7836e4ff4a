"""Pins of the oracle's box spline (polygon clipping) against facts the paper and
the mathematics fix: ZP lattice values and partition of unity, the support
polygon, unit mass, the covariance closed form (eq. (covariance_ZP)), the
fourth moments of App. E, the kurtosis matrix (App. E, eq. (finalForm)) and the
Fourier transform prod_k sinc(a_k u_k.w / 2) (App. A, eq. (A1)).

Quadrature: midpoint rule on a uniform grid covering the support.  For a C^1
function with compact support the O(h^2) term of the midpoint rule integrates
a second derivative over the whole plane and vanishes, so the grid below is
accurate to far better than the tolerances used.
"""
import math

import numpy as np
import pytest

SQ2 = math.sqrt(2.0)
U = np.array([[1.0, 0.0], [1 / SQ2, 1 / SQ2], [0.0, 1.0], [-1 / SQ2, 1 / SQ2]])


def quad_grid(orc, a, h=0.004):
    rx = 0.5 * (a[0] + (a[1] + a[3]) / SQ2) + 0.01
    ry = 0.5 * (a[2] + (a[1] + a[3]) / SQ2) + 0.01
    nx, ny = int(2 * rx / h) + 1, int(2 * ry / h) + 1
    x0, y0 = -rx + 0.5 * h + 1e-7, -ry + 0.5 * h + 2e-7
    B = orc.boxspline_grid(a, x0, y0, h, nx, ny)
    X = x0 + h * np.arange(nx)[None, :]
    Y = y0 + h * np.arange(ny)[:, None]
    return X, Y, B, h * h


CASES = [(1.3, 2.1, 0.9, 1.7), (2.449, 2.449, 2.449, 2.449), (3.2, 0.7, 1.1, 2.6), (1.0, SQ2, 1.0, SQ2)]


# ----------------------------------------------------------------------------- ZP element

def test_zp_lattice_values(orc):
    # ZP(x) = 1/2 area([-1/2,1/2]^2 intersect (x + {|y1|+|y2| <= 1})) (density of T1(1,0)+T2(1,1)+T3(0,1)+T4(-1,1)).
    # At 0 the unit square lies in the diamond: 1/2.  At (1,0) the overlap is the triangle
    # {0 <= y1 <= 1/2, |y2| <= y1} of area 1/4: 1/8.  At (1,1) the overlap is a single point: 0.
    assert orc.zp(0, 0) == pytest.approx(0.5, abs=1e-15)
    for x, y in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
        assert orc.zp(x, y) == pytest.approx(0.125, abs=1e-15)
    for x, y in [(1, 1), (-1, 1), (2, 0), (0, -2), (2, 1)]:
        assert orc.zp(x, y) == pytest.approx(0.0, abs=1e-15)


def test_zp_partition_of_unity(orc):
    # b_k u_k are lattice vectors, so sum_m ZP(y - m) = 1 for every y.
    rng = np.random.default_rng(1)
    for y in rng.random((40, 2)) * 3 - 1.5:
        s = sum(orc.zp(y[0] - m1, y[1] - m2) for m1 in range(-4, 5) for m2 in range(-4, 5))
        assert s == pytest.approx(1.0, abs=1e-14)


def test_zp_support_octagon(orc):
    # support {sum t_k b_k u_k, |t_k| <= 1/2} = {|x| <= 3/2, |y| <= 3/2, |x|+|y| <= 2}; at most 7 lattice points
    rng = np.random.default_rng(2)
    for x, y in rng.random((400, 2)) * 5 - 2.5:
        inside = abs(x) < 1.5 and abs(y) < 1.5 and abs(x) + abs(y) < 2
        v = orc.zp(x, y)
        assert (v > 0) == inside, (x, y, v)
    for y in rng.random((100, 2)) * 2:
        npts = sum(orc.zp(y[0] - m1, y[1] - m2) > 0 for m1 in range(-3, 4) for m2 in range(-3, 4))
        assert npts <= 7


# ----------------------------------------------------------------------------- moments

@pytest.mark.parametrize("a", CASES)
def test_mass_and_covariance(orc, a):
    X, Y, B, dA = quad_grid(orc, a)
    mass = B.sum() * dA
    assert mass == pytest.approx(1.0, abs=2e-7)
    C = np.array([[(X * X * B).sum(), (X * Y * B).sum()], [(X * Y * B).sum(), (Y * Y * B).sum()]]) * dA
    a1, a2, a3, a4 = a
    ref = np.array([[2 * a1**2 + a2**2 + a4**2, a2**2 - a4**2], [a2**2 - a4**2, 2 * a3**2 + a2**2 + a4**2]]) / 24.0
    np.testing.assert_allclose(C, ref, atol=2e-6)
    # symmetry about the origin: odd moments vanish
    assert abs((X * B).sum() * dA) < 1e-7 and abs((Y * B).sum() * dA) < 1e-7


def _moments4_paper(a, mu4, mu2, typo=False):
    a1, a2, a3, a4 = a
    p = lambda v, k: v**k
    m40 = 0.25 * mu4 * (4 * p(a1, 4) + p(a2, 4) + p(a4, 4)) + 0.5 * mu2**2 * (6 * a1**2 * a2**2 + 6 * a1**2 * a4**2 + 3 * a2**2 * a4**2)
    m31 = 0.25 * mu4 * (p(a2, 4) - p(a4, 4)) + 1.5 * mu2**2 * a1**2 * (a2**2 - a4**2)
    a34 = a3**3 * a4**2 if typo else a3**2 * a4**2
    m22 = 0.25 * mu4 * (p(a2, 4) + p(a4, 4)) + 0.5 * mu2**2 * (a1**2 * a2**2 + a1**2 * a4**2 + a2**2 * a3**2 + a34 - a2**2 * a4**2 + 2 * a1**2 * a3**2)
    m13 = 0.25 * mu4 * (p(a2, 4) - p(a4, 4)) + 1.5 * mu2**2 * a3**2 * (a2**2 - a4**2)
    m04 = 0.25 * mu4 * (4 * p(a3, 4) + p(a2, 4) + p(a4, 4)) + 0.5 * mu2**2 * (6 * a2**2 * a3**2 + 6 * a3**2 * a4**2 + 3 * a2**2 * a4**2)
    return np.array([m40, m31, m22, m13, m04])


@pytest.mark.parametrize("a", CASES[:3])
def test_fourth_moments_appendix_e(orc, a, paper):
    X, Y, B, dA = quad_grid(orc, a)
    num = np.array([(X**4 * B).sum(), (X**3 * Y * B).sum(), (X**2 * Y**2 * B).sum(), (X * Y**3 * B).sum(),
                    (Y**4 * B).sum()]) * dA
    mu4, mu2 = paper["box_moments"]["mu4"], paper["box_moments"]["mu2"]
    np.testing.assert_allclose(num, _moments4_paper(a, mu4, mu2), rtol=2e-5, atol=1e-6)
    if abs(a[2] - 1.0) > 0.05:   # the printed a3^3 a4^2 term differs from a3^2 a4^2 unless a3 = 1
        assert abs(num[2] - _moments4_paper(a, mu4, mu2, typo=True)[2]) > 1e-5


@pytest.mark.parametrize("a", CASES[:3])
def test_kurtosis_matrix_final_form(orc, a, paper):
    X, Y, B, dA = quad_grid(orc, a)
    Cm = np.array([[(X * X * B).sum(), (X * Y * B).sum()], [(X * Y * B).sum(), (Y * Y * B).sum()]]) * dA
    # L = int (x x^T)^2 f ; (x x^T)^2 = |x|^2 x x^T
    R2 = X * X + Y * Y
    L = np.array([[(R2 * X * X * B).sum(), (R2 * X * Y * B).sum()], [(R2 * X * Y * B).sum(), (R2 * Y * Y * B).sum()]]) * dA
    K = L - np.trace(Cm) * Cm - 2 * Cm @ Cm
    mu4, mu2 = paper["box_moments"]["mu4"], paper["box_moments"]["mu2"]
    a1, a2, a3, a4 = a
    Kf = (mu4 - 3 * mu2**2) * np.array([[a1**4 + 0.5 * (a2**4 + a4**4), 0.5 * (a2**4 - a4**4)],
                                         [0.5 * (a2**4 - a4**4), a3**4 + 0.5 * (a2**4 + a4**4)]])
    np.testing.assert_allclose(K, Kf, rtol=1e-4, atol=2e-6)


@pytest.mark.parametrize("a", CASES[:2])
def test_fourier_transform_is_sinc_product(orc, a):
    X, Y, B, dA = quad_grid(orc, a, h=0.005)
    for w in [(0.7, -0.3), (1.9, 0.4), (-1.1, 2.2), (2.5, 2.5)]:
        num = (B * np.cos(w[0] * X + w[1] * Y)).sum() * dA
        ref = np.prod([np.sinc(a[k] * (U[k] @ np.array(w)) / 2 / np.pi) for k in range(4)])
        assert num == pytest.approx(ref, abs=2e-6)


def test_boxspline_symmetric_and_scales(orc):
    rng = np.random.default_rng(3)
    a = (1.7, 0.9, 2.3, 1.4)
    for x, y in rng.random((50, 2)) * 4 - 2:
        assert orc.boxspline(a, x, y) == pytest.approx(orc.boxspline(a, -x, -y), abs=1e-15)
        # dilation: beta_{c a}(c x) = beta_a(x) / c^2
        c = 1.7
        assert orc.boxspline([c * v for v in a], c * x, c * y) == pytest.approx(orc.boxspline(a, x, y) / c**2, rel=1e-12, abs=1e-15)
