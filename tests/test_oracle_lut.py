"""Pins of the oracle's look-up-table scale map (Sec. 3.2.2, O1/O2).

* At the table's nodes, in every octant and at any size, the looked-up scales
  have exactly the requested covariance (eq. (covariance_ZP), itself pinned by
  quadrature) and equal the direct solve with the floor eps_rel * s: this pins
  the node layout, the octant reduction, the permutation and the sqrt(s)
  scaling.  The permutation as printed (second and fourth octant rows
  exchanged) fails the covariance check.
* Between nodes the covariance error is small and falls like the square of the
  node spacing (bilinear interpolation of a smooth function).
* Isotropic requests give all four scales sqrt(3 s) (Thm. 2.2); octant edges
  are continuous.
"""
import math

import numpy as np
import pytest

from test_oracle_scales import cov_closed_form, cov_request

N = 17          # small tables keep the pins fast
EPS = 0.125


@pytest.fixture(scope="module")
def table(orc):
    return orc.lut_table(N, EPS)


def lut_one(orc, table, sigma, rho, theta):
    f = np.array([[[sigma, rho, theta]]], dtype=np.float64)
    return orc.scales_lut(f, orc.FIELD_SRT3, 1, table=table)[0, 0]


def test_nodes_every_octant_any_size(orc, table):
    rng = np.random.default_rng(5)
    checked = 0
    for i in range(1, N):
        for j in range(N):
            rho = (N - 1) / i
            phi = j * (math.pi / 4) / (N - 1)
            k = rng.integers(0, 4)
            sigma = math.sqrt(0.5) * (0.5 + 20 * rng.random())
            th = phi + k * math.pi / 4
            if th >= math.pi:
                continue
            s = 2 * sigma * sigma
            if rho >= orc.rho_max(s, th, EPS * s) * 0.999:
                continue   # clamped node: covariance differs from the request by design
            a = lut_one(orc, table, sigma, rho, th)
            np.testing.assert_allclose(cov_closed_form(a), cov_request(sigma, rho, th), rtol=2e-6,
                                       atol=2e-6 * s)
            ref, _, _ = orc.scales_from_srt(sigma, rho, th, eps=EPS * s)
            np.testing.assert_allclose(a, ref, rtol=2e-6)
            checked += 1
    assert checked > 150


def test_printed_permutation_fails(orc, table):
    sigma, rho, phi = 1.3, (N - 1) / 6, 3 * (math.pi / 4) / (N - 1)   # a node
    th = phi + math.pi / 4                           # second octant
    base = lut_one(orc, table, math.sqrt(0.5), rho, phi) * math.sqrt(2 * sigma * sigma)
    printed = np.array([base[1], base[2], base[3], base[0]])
    assert np.max(np.abs(cov_closed_form(printed) - cov_request(sigma, rho, th))) > 1e-2
    used = lut_one(orc, table, sigma, rho, th)
    np.testing.assert_allclose(cov_closed_form(used), cov_request(sigma, rho, th), rtol=2e-6, atol=1e-6)


def test_interpolation_error_second_order(orc):
    rng = np.random.default_rng(6)
    cases = []
    while len(cases) < 200:
        sigma, rho, th = 0.5 + 5 * rng.random(), 1 + 4 * rng.random(), math.pi * rng.random()
        s = 2 * sigma * sigma
        if rho < 0.8 * orc.rho_max(s, th, EPS * s):
            cases.append((sigma, rho, th))
    f = np.array([cases], dtype=np.float64)
    errs = []
    for n in (17, 33, 65):
        a = orc.scales_lut(f, orc.FIELD_SRT3, 1, nodes=n, eps_rel=EPS)[0]
        e = [np.abs(cov_closed_form(ai) - cov_request(*c)).max() / (2 * c[0] ** 2) for ai, c in zip(a, cases)]
        errs.append(max(e))
    print("max relative covariance error for 17, 33, 65 nodes:", errs)
    assert errs[2] < 5e-3
    assert errs[1] < errs[0] / 2.5 and errs[2] < errs[1] / 2.5


def test_isotropic_and_octant_continuity(orc, table):
    for sigma in (0.7, 3.0):
        a = lut_one(orc, table, sigma, 1.0, 0.4)
        np.testing.assert_allclose(a, math.sqrt(3 * 2 * sigma * sigma), rtol=1e-6)
    for k in (1, 2, 3):
        lo = lut_one(orc, table, 2.0, 2.2, k * math.pi / 4 - 1e-9)
        hi = lut_one(orc, table, 2.0, 2.2, k * math.pi / 4 + 1e-9)
        np.testing.assert_allclose(lo, hi, rtol=1e-6)


def test_cov_field_matches_srt_field(orc, table):
    rng = np.random.default_rng(8)
    srt = np.stack([0.5 + 4 * rng.random(50), 1 + 3 * rng.random(50), math.pi * rng.random(50)], -1)
    cov = np.array([cov_request(*c) for c in srt])
    a1 = orc.scales_lut(srt[None], orc.FIELD_SRT3, 2, table=table)
    a2 = orc.scales_lut(cov[None], orc.FIELD_COV3, 2, table=table)
    np.testing.assert_allclose(a1, a2, rtol=1e-9)
