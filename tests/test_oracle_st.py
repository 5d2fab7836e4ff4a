"""Pins of the oracle's structure-tensor step (Sec. 4.2).

* Central differences: exact on a ramp, with the border values each boundary
  rule implies.
* A plane wave cos(w (x cos p + y sin p)) has g g^T proportional to v v^T with
  v = (sin(w cos p), sin(w sin p)) at every pixel, so J has rank one away from
  the borders and theta* is the direction of v rotated by a quarter turn,
  for any window (closed form).
* The printed rules on a full-rank J give the filter covariance
  tr(J) I - J (its eigenvalues swapped onto the other eigenvectors): checked
  against that closed form; rank-one and zero tensors take the special rules.
* A quarter turn of the image swaps J11 and J22, negates J12 and turns theta*
  by -pi/2 (the isotropic window is invariant under the quarter turn).
* The window is this oracle's filter: fast = direct sum.
"""
import math

import numpy as np
import pytest

from paper_1003_2022_amd import inputs as I


def test_gradient_ramp_and_border_rules(orc):
    H, W = 7, 9
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    f = 0.25 * x - 0.5 * y + 3.0
    for b in (orc.BOUNDARY_REPLICATE, orc.BOUNDARY_SYMMETRIC):
        g1, g2 = orc.gradient(f, b)
        np.testing.assert_allclose(g1[:, 1:-1, 0], 0.25, atol=1e-15)
        np.testing.assert_allclose(g2[1:-1, :, 0], -0.5, atol=1e-15)
        # both rules repeat the border sample: a one-sided difference halved
        np.testing.assert_allclose(g1[:, 0, 0], 0.125, atol=1e-15)
        np.testing.assert_allclose(g1[:, -1, 0], 0.125, atol=1e-15)
        np.testing.assert_allclose(g2[0, :, 0], -0.25, atol=1e-15)
    g1, g2 = orc.gradient(f, orc.BOUNDARY_ZERO)
    np.testing.assert_allclose(g1[:, 0, 0], 0.5 * f[:, 1], atol=1e-15)
    np.testing.assert_allclose(g2[-1, :, 0], -0.5 * f[-2, :], atol=1e-15)


@pytest.mark.parametrize("phi,w", [(0.3, 0.9), (1.2, 0.5), (2.0, 1.4), (2.9, 0.7)])
def test_plane_wave_rank_one_and_orientation(orc, phi, w):
    H = W = 48
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    f = np.cos(w * (x * math.cos(phi) + y * math.sin(phi)))
    J = orc.structure_tensor(f, 2.0, 1, orc.BOUNDARY_SYMMETRIC)
    v = np.array([math.sin(w * math.cos(phi)), math.sin(w * math.sin(phi))])
    th_ref = math.atan2(v[0], -v[1]) % math.pi
    s, rho, th = orc.st_triple(J[14:-14, 14:-14], lambda_zero=1e-10 * (J[..., 0] + J[..., 2]).max())
    det = J[..., 0] * J[..., 2] - J[..., 1] ** 2
    tr = J[..., 0] + J[..., 2]
    assert np.max(np.abs(det[14:-14, 14:-14]) / tr[14:-14, 14:-14] ** 2) < 1e-12
    d = np.abs(th - th_ref)
    assert np.max(np.minimum(d, math.pi - d)) < 1e-9
    # rank one: the rule rho = max(1, lambda_max), s = lambda_max
    lmax = tr[14:-14, 14:-14]
    np.testing.assert_allclose(rho, np.maximum(1.0, lmax), rtol=1e-9)
    np.testing.assert_allclose(s, lmax, rtol=1e-9)


def _cov_from_triple(s, rho, th):
    l1, l2 = s * rho / (1 + rho), s / (1 + rho)
    c, sn = np.cos(th), np.sin(th)
    return np.stack([l1 * c * c + l2 * sn * sn, (l1 - l2) * c * sn, l1 * sn * sn + l2 * c * c], -1)


def test_full_rank_rules_give_adjugate(orc):
    rng = np.random.default_rng(7)
    A = rng.normal(size=(500, 2, 2))
    M = A @ np.swapaxes(A, 1, 2) + 1e-3 * np.eye(2)
    J = np.stack([M[:, 0, 0], M[:, 0, 1], M[:, 1, 1]], -1)
    for gain in (1.0, 37.5):
        s, rho, th = orc.st_triple(J, gain=gain)
        C = _cov_from_triple(s, rho, th)
        tr = J[:, 0] + J[:, 2]
        adj = gain * np.stack([tr - J[:, 0], -J[:, 1], tr - J[:, 2]], -1)
        np.testing.assert_allclose(C, adj, rtol=0, atol=1e-12 * gain * tr.max())
        np.testing.assert_allclose(s, gain * tr, rtol=1e-12)


def test_special_rules(orc):
    J = np.array([[0.0, 0.0, 0.0],        # flat
                  [2.5, 0.0, 0.0],        # rank one along x: theta* = pi/2
                  [0.0, 0.0, 0.5],        # rank one along y, lambda < 1: rho = 1
                  [3.0, 0.0, 1e-9]])      # below lambda_zero: rank one
    s, rho, th = orc.st_triple(J, lambda_zero=1e-6, a_flat=1.5)
    np.testing.assert_allclose(s, [1.5 ** 2 / 3, 2.5, 0.5, 3.0], rtol=1e-15)
    np.testing.assert_allclose(rho, [1.0, 2.5, 1.0, 3.0], rtol=1e-15)
    np.testing.assert_allclose(th[1:], [math.pi / 2, 0.0, math.pi / 2], atol=1e-15)
    fld = np.stack([np.sqrt(s / 2), rho, th], -1)
    # the flat filter: all four scales a_flat (covariance a_flat^2 / 6 I)
    a, _, _ = orc.scales_from_srt(*fld[0])
    np.testing.assert_allclose(a, 1.5, rtol=1e-9)


@pytest.mark.parametrize("boundary", [1, 2])
def test_quarter_turn_equivariance(orc, boundary):
    f = I.uniform_image(23, 30, 61)
    J = orc.structure_tensor(f, 1.7, 2, boundary)
    Jr = orc.structure_tensor(np.rot90(f).copy(), 1.7, 2, boundary)
    # rot90: f'[y', x'] = f[x', W-1-y']  =>  g'1 = g2, g'2 = -g1 at the matching pixel
    back = np.rot90(Jr, -1)
    np.testing.assert_allclose(back[..., 0], J[..., 2], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(back[..., 2], J[..., 0], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(back[..., 1], -J[..., 1], rtol=1e-10, atol=1e-13)
    _, _, th = orc.st_triple(J)
    _, _, thr = orc.st_triple(np.ascontiguousarray(back))
    d = np.abs(np.mod(th - math.pi / 2, math.pi) - thr)
    assert np.max(np.minimum(d, math.pi - d)) < 1e-7


def test_window_fast_equals_direct_sum(orc):
    f = I.uniform_image(19, 21, 62, channels=2)
    Jf = orc.structure_tensor(f, 1.3, 1, orc.BOUNDARY_SYMMETRIC, method="fast", tile=6)
    Jb = orc.structure_tensor(f, 1.3, 1, orc.BOUNDARY_SYMMETRIC, method="brute")
    np.testing.assert_allclose(Jf, Jb, rtol=1e-10, atol=1e-13)
    assert (Jf[..., 0] >= 0).all() and (Jf[..., 2] >= 0).all()
    assert (Jf[..., 0] * Jf[..., 2] - Jf[..., 1] ** 2 >= -1e-12).all()   # positive semi-definite
