"""Pins of the oracle's scale-vector solve (Sec. 3.2.2) against what the paper
and the mathematics fix:

* Thm. 2.2 with N = 4: covariance sigma^2 I gives a_k = sigma sqrt6;
* the covariance of the solved box spline equals the requested covariance,
  checked with quadrature of the oracle's own box spline (independent of the
  solver's matrix M) and, over many random cases, with eq. (covariance_ZP),
  itself pinned by quadrature in test_oracle_boxspline;
* optimality: no feasible t on a fine grid gives a smaller ||K_p||^2 (App. E);
* rotation by pi/4 permutes the scales, (a1,a2,a3,a4) -> (a4,a1,a2,a3)
  (a rotation moves box k onto direction k+1; ||K|| is rotation invariant,
  App. D), which pins every index of the solve;
* the elongation bound of Prop. 3.1 (eq. (bound)) and its value 3 + 2 sqrt2 at
  the mid-way orientations.
"""
import math

import numpy as np
import pytest

SQ2 = math.sqrt(2.0)


def cov_closed_form(a):
    a1, a2, a3, a4 = a
    return np.array([2 * a1**2 + a2**2 + a4**2, a2**2 - a4**2, 2 * a3**2 + a2**2 + a4**2]) / 24.0


def cov_request(sigma, rho, theta):
    s = 2 * sigma**2
    lmax, lmin = s * rho / (1 + rho), s / (1 + rho)
    c, sn = math.cos(theta), math.sin(theta)
    return np.array([lmax * c * c + lmin * sn * sn, 0.5 * (lmax - lmin) * math.sin(2 * theta), lmin * c * c + lmax * sn * sn])


def kurt_norm2(p):
    # App. E: ||K||^2 proportional to sum p_k^4 + (p1^2 + p3^2)(p2^2 + p4^2), p = a^2
    return np.sum(p**4, axis=-1) + (p[..., 0]**2 + p[..., 2]**2) * (p[..., 1]**2 + p[..., 3]**2)


def U_bound(phi):
    # Prop. 3.1, eq. (bound)
    nu = 0.5 * (math.tan(phi) - 1 / math.tan(phi)) * np.sign(math.pi / 2 - phi)
    r = math.sqrt(1 + nu * nu)
    return (1 + abs(nu) + r) / (1 + abs(nu) - r)


@pytest.mark.parametrize("sigma", [0.8, 1.0, 2.5, 7.0, 32.0])
def test_isotropic_is_sigma_sqrt6(orc, paper, sigma):
    a, cl, ea = orc.scales_from_srt(sigma, 1.0, 0.37, eps=1e-6)
    np.testing.assert_allclose(a, sigma * paper["isotropic_scale"]["factor"], rtol=1e-12)
    assert not cl and not ea


@pytest.mark.parametrize("srt", [(1.0, 2.5, 0.4), (3.0, 4.0, 2.0), (1.5, 1.8, 1.1)])
def test_solved_covariance_by_quadrature(orc, srt):
    a, cl, _ = orc.scales_from_srt(*srt, eps=1e-3)
    assert not cl
    h = 0.006
    rx = 0.5 * (a[0] + (a[1] + a[3]) / SQ2) + 0.01
    ry = 0.5 * (a[2] + (a[1] + a[3]) / SQ2) + 0.01
    nx, ny = int(2 * rx / h) + 1, int(2 * ry / h) + 1
    x0, y0 = -rx + h / 2 + 1e-7, -ry + h / 2 + 3e-7
    B = orc.boxspline_grid(a, x0, y0, h, nx, ny)
    X = x0 + h * np.arange(nx)[None, :]
    Y = y0 + h * np.arange(ny)[:, None]
    Cq = np.array([(X * X * B).sum(), (X * Y * B).sum(), (Y * Y * B).sum()]) * h * h
    np.testing.assert_allclose(Cq, cov_request(*srt), rtol=1e-5, atol=1e-6)


def test_solved_covariance_many(orc):
    rng = np.random.default_rng(11)
    worst = 0.0
    n = 0
    while n < 3000:
        sigma = 0.5 + 20 * rng.random()
        theta = math.pi * rng.random()
        rmax = orc.rho_max(2 * sigma**2, theta, 0.25)
        rho = 1 + (min(rmax, 8.0) - 1) * rng.random() * 0.999
        a, cl, _ = orc.scales_from_srt(sigma, rho, theta, eps=0.25)
        assert not cl
        assert np.all(a * a >= 0.25 * (1 - 1e-12))
        req = cov_request(sigma, rho, theta)
        worst = max(worst, np.max(np.abs(cov_closed_form(a) - req)) / np.max(np.abs(req)))
        n += 1
    assert worst < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_solution_minimises_kurtosis(orc, seed):
    rng = np.random.default_rng(100 + seed)
    sigma, theta = 1 + 5 * rng.random(), math.pi * rng.random()
    rho = 1 + 4 * rng.random()
    eps = 0.25
    rho = min(rho, orc.rho_max(2 * sigma**2, theta, eps) * 0.99)
    a, _, _ = orc.scales_from_srt(sigma, rho, theta, eps=eps)
    p0 = a * a
    # the whole feasible line p0 + t e, e = (1,-1,1,-1), p >= eps
    e = np.array([1.0, -1.0, 1.0, -1.0])
    tl = max(eps - p0[0], eps - p0[2])
    tr = min(p0[1] - eps, p0[3] - eps)
    assert tl <= 1e-9 and tr >= -1e-9
    ts = np.linspace(tl, tr, 20001)
    P = p0[None, :] + ts[:, None] * e[None, :]
    k = kurt_norm2(P)
    assert kurt_norm2(p0) <= k.min() * (1 + 1e-12) + 1e-12
    # every point of the line has the same covariance
    for t in (tl, tr):
        np.testing.assert_allclose(cov_closed_form(np.sqrt(np.maximum(p0 + t * e, 0))), cov_closed_form(a), rtol=1e-9, atol=1e-12)


def test_rotation_by_quarter_pi_permutes_scales(orc):
    rng = np.random.default_rng(21)
    done = 0
    while done < 300:
        sigma, theta = 0.7 + 10 * rng.random(), (math.pi - math.pi / 4) * rng.random()
        rho = 1 + 5 * rng.random()
        eps = 0.25
        lim = min(orc.rho_max(2 * sigma**2, theta, eps), orc.rho_max(2 * sigma**2, theta + math.pi / 4, eps))
        if rho >= lim * 0.999:
            continue
        a, _, _ = orc.scales_from_srt(sigma, rho, theta, eps=eps)
        b, _, _ = orc.scales_from_srt(sigma, rho, theta + math.pi / 4, eps=eps)
        np.testing.assert_allclose(b, [a[3], a[0], a[1], a[2]], rtol=1e-9, atol=1e-9)
        done += 1


def test_elongation_bound(orc, paper):
    # eps -> 0: the largest feasible elongation is the bound U(phi) of Prop. 3.1
    for phi in np.linspace(0.05, math.pi - 0.05, 57):
        if min(abs(phi - k * math.pi / 4) for k in range(5)) < 1e-3:
            continue
        assert orc.rho_max(2.0, phi, 0.0) == pytest.approx(U_bound(phi), rel=1e-9)
    for phi in paper["elongation_bound_midway"]["phis"]:
        assert orc.rho_max(2.0, phi, 0.0) == pytest.approx(paper["elongation_bound_midway"]["value"], rel=1e-12)
        assert U_bound(phi) == pytest.approx(3 + 2 * SQ2, rel=1e-12)
    # along the box directions the bound is infinite
    for k in range(4):
        assert math.isinf(orc.rho_max(2.0, k * math.pi / 4, 0.0)) or orc.rho_max(2.0, k * math.pi / 4, 0.0) > 1e12


def test_clamp_keeps_size_orientation(orc):
    # requested elongation beyond the bound: lowered to the feasible maximum at fixed (s, theta)
    for theta in [math.pi / 8, 0.5, 2.0, 3 * math.pi / 8]:
        sigma, rho, eps = 2.0, 9.0, 0.25
        a, cl, ea = orc.scales_from_srt(sigma, rho, theta, eps=eps)
        assert cl and ea
        C = cov_closed_form(a)
        rmax = orc.rho_max(2 * sigma**2, theta, eps)
        np.testing.assert_allclose(C, cov_request(sigma, rmax, theta), rtol=1e-9, atol=1e-12)
        assert np.min(a * a) == pytest.approx(eps, rel=1e-9)


def test_cov_entry_matches_srt_entry(orc):
    rng = np.random.default_rng(5)
    for _ in range(200):
        sigma, theta, rho = 0.8 + 6 * rng.random(), math.pi * rng.random(), 1 + 3 * rng.random()
        a, _, _ = orc.scales_from_srt(sigma, rho, theta)
        b, _, _ = orc.scales_from_cov(*cov_request(sigma, rho, theta))
        np.testing.assert_allclose(a, b, rtol=1e-9)


def test_printed_zeta_prime_coefficients(orc):
    """The argmin found with the printed cubic agrees with a direct minimisation of
    ||K||^2 along the line, so the printed coefficients (Sec. 3.2.2) are the derivative."""
    rng = np.random.default_rng(8)
    for _ in range(50):
        sigma, theta, rho = 1 + 3 * rng.random(), math.pi * rng.random(), 1 + 1.5 * rng.random()
        a, _, ea = orc.scales_from_srt(sigma, rho, theta, eps=1e-9)
        p = a * a
        if ea or p.min() < 1e-6 * p.max():   # optimum on the boundary of [t_l, t_r]
            continue
        e = np.array([1.0, -1.0, 1.0, -1.0])
        d = 1e-4 * np.max(p)
        # interior optimum: symmetric difference of ||K||^2 along e vanishes
        g = (kurt_norm2(p + d * e) - kurt_norm2(p - d * e)) / (2 * d)
        assert abs(g) < 1e-6 * kurt_norm2(p) / np.max(p)
