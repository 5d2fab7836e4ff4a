"""Pins of the oracle's running sums and filter.

* Running sums (Algorithm 1, step 2): the nested infinite sums RS1..RS4 of
  Sec. 3.1 evaluated by brute force on tiny windows; backward unit differences
  along v4, v3, v2, v1 undo them exactly (integer variant); FP64 = 2 x integer.
* Taps and shift: Table 1 and the printed tau.
* Filter: the fast algorithm equals the direct sum sum_k f[k] beta_{a(n)}(n-k)
  (the exactness of Prop. 2.1 (link2) with the Dirac-comb input); the direct sum with
  a constant field is an ordinary 2-D convolution (scipy.signal.convolve2d);
  a = b reduces to the ZP lattice stencil 1/2, 1/8; unit mass holds exactly
  when a1, a3 are integers and otherwise equals the Poisson sum of the Fourier
  form prod sinc(a_k u_k.w/2) over w in 2 pi Z^2; iterating m passes with a/sqrt m
  approaches the Gaussian of the same covariance (Sec. 3.3).
"""
import math

import numpy as np
import pytest
from scipy.signal import convolve2d

from paper_1003_2022_amd import inputs as I

SQ2 = math.sqrt(2.0)
V = [(1, 0), (1, 1), (0, 1), (-1, 1)]   # b_k u_k as (dx, dy) lattice steps


def brute_running_sums(f, scale=SQ2):
    """g_b = RS4 RS3 RS2 RS1 f on the window by direct nested sums (zero outside the window)."""
    h, w = f.shape
    inside = lambda r, c: 0 <= r < h and 0 <= c < w
    g = f.astype(object) if scale is None else f.astype(np.float64)
    factors = [1, scale, 1, scale] if scale is not None else [1, 1, 1, 1]
    for (dx, dy), fac in zip(V, factors):
        out = np.zeros_like(g)
        for r in range(h):
            for c in range(w):
                acc = 0
                k = 0
                while inside(r - k * dy, c - k * dx):
                    acc = acc + g[r - k * dy, c - k * dx]
                    k += 1
                out[r, c] = fac * acc
        g = out
    return g


def test_running_sums_brute_f64(orc):
    f = I.uniform_image(7, 9, 3).astype(np.float64)
    g = orc.preint_window_f64(f, 0, 0, 7, 9)
    np.testing.assert_allclose(g, brute_running_sums(f), rtol=1e-14)


def test_running_sums_brute_i64_and_window(orc):
    img = I.uniform_image(6, 8, 4, "u16")
    # window sticking out of the image on every side: samples outside are zero
    g = orc.preint_window_i64(img, -2, -3, 11, 13)
    f = np.zeros((11, 13), dtype=np.int64)
    f[2:8, 3:11] = img
    ref = brute_running_sums(f.astype(object), scale=None)
    assert np.array_equal(g, np.array(ref, dtype=np.int64))


def test_integer_scans_inverted_by_differences(orc):
    img = I.uniform_image(40, 37, 5, "u16")
    G = orc.preint_window_i64(img, -5, -4, 52, 50).astype(np.uint64)
    with np.errstate(over="ignore"):
        for dx, dy in reversed(V):   # undo RS4 first
            sh = np.zeros_like(G)
            h, w = G.shape
            r0, r1 = max(0, dy), h
            c0, c1 = max(0, dx), min(w, w + dx)
            sh[r0:r1, c0:c1] = G[r0 - dy:r1 - dy, c0 - dx:c1 - dx]
            G = G - sh
    f = np.zeros((52, 50), dtype=np.uint64)
    f[5:45, 4:41] = img
    assert np.array_equal(G, f)


def test_f64_scan_is_twice_integer_scan(orc):
    img = I.uniform_image(30, 33, 6, "u16")
    gi = orc.preint_window_i64(img, -3, -3, 40, 41)
    gf = orc.preint_window_f64(img, -3, -3, 40, 41)
    np.testing.assert_allclose(gf, 2.0 * gi.astype(np.float64), rtol=1e-14)


def test_table1_taps_and_tau(orc, paper):
    rng = np.random.default_rng(9)
    for _ in range(5):
        a = 0.5 + 3 * rng.random(4)
        basis = np.array([a[0], a[1] / SQ2, a[2], a[3] / SQ2])
        for row in paper["table1_taps"]["rows"]:
            x, sg = orc.table1_tap(a, row["i"])
            np.testing.assert_allclose(x, [np.dot(row["x1"], basis), np.dot(row["x2"], basis)], atol=1e-14)
            assert sg == row["sign"]
        t = orc.tau(a)
        av = np.array([*a, 1.0])
        np.testing.assert_allclose(t, [np.dot(paper["tau"]["tau1"], av), np.dot(paper["tau"]["tau2"], av)], atol=1e-14)


# ----------------------------------------------------------------------------- filter

@pytest.mark.parametrize("shape,tile,seed", [((19, 23), 8, 1), ((30, 17), 5, 2), ((12, 40), 64, 3)])
def test_fast_equals_direct_sum_white_scales(orc, shape, tile, seed):
    H, W = shape
    f = I.uniform_image(H, W, seed)
    a = I.scales_field(H, W, seed, 0.5, 3.2).astype(np.float64)
    fast = orc.filter_scales(f, a, 1, "fast", tile)
    brute = orc.filter_scales(f, a, 1, "brute")
    assert np.max(np.abs(fast - brute)) <= 1e-10 * np.max(np.abs(brute))


@pytest.mark.parametrize("order", [1, 2, 3])
def test_fast_equals_direct_sum_srt_field(orc, order):
    H, W = 28, 26
    f = I.uniform_image(H, W, 10 + order)
    fld = I.srt_field(H, W, 10 + order, (1.0, 3.0), (1.0, 6.0), corr_len=6.0)
    fast = orc.filter(f, fld, orc.FIELD_SRT3, order, method="fast", tile=9)
    brute = orc.filter(f, fld, orc.FIELD_SRT3, order, method="brute")
    assert np.max(np.abs(fast - brute)) <= 1e-11 * np.max(np.abs(brute))


def test_direct_sum_constant_field_is_convolution(orc):
    H, W = 25, 31
    f = I.uniform_image(H, W, 12).astype(np.float64)
    a = np.array([2.3125, 1.09375, 1.625, 2.890625])   # exact in float32
    rx, ry = orc.support_halfwidths(a)
    Rx, Ry = int(np.ceil(rx)), int(np.ceil(ry))
    hk = orc.boxspline_grid(a, -Rx, -Ry, 1.0, 2 * Rx + 1, 2 * Ry + 1)   # h[k] = beta_a(k)
    ref = convolve2d(f, hk, mode="full")[Ry:Ry + H, Rx:Rx + W]
    field = np.broadcast_to(a, (H, W, 4)).astype(np.float32)
    out = orc.filter(f, field, orc.FIELD_SCALES4, 1, method="brute")
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-13)
    fast = orc.filter(f, field, orc.FIELD_SCALES4, 1, method="fast", tile=7)
    np.testing.assert_allclose(fast, ref, rtol=1e-11, atol=1e-12)


def test_zp_scales_give_lattice_stencil(orc):
    H, W = 14, 15
    f = I.uniform_image(H, W, 13).astype(np.float64)
    a = np.broadcast_to([1.0, SQ2, 1.0, SQ2], (H, W, 4)).astype(np.float64)
    out = orc.filter_scales(f, a, 1, "fast", 5)
    p = np.pad(f, 1)
    ref = 0.5 * f + 0.125 * (p[:-2, 1:-1] + p[2:, 1:-1] + p[1:-1, :-2] + p[1:-1, 2:])
    np.testing.assert_allclose(out, ref, atol=1e-13)


def test_unit_mass_integer_a1_a3(orc):
    # Poisson summation: sum_k beta(n-k) = sum_j beta^(2 pi j); a1, a3 in Z make every j != 0 term vanish
    H, W = 30, 30
    f = np.ones((H, W))
    for a in ([2.0, 1.3, 1.0, 2.2], [3.0, 0.8, 2.0, 1.9]):
        out = orc.filter_scales(f, np.broadcast_to(a, (H, W, 4)).astype(np.float64), 1, "fast", 10)
        np.testing.assert_allclose(out[8:-8, 8:-8], 1.0, atol=1e-12)


def _poisson_mass(a, J=240):
    U = np.array([[1.0, 0.0], [1 / SQ2, 1 / SQ2], [0.0, 1.0], [-1 / SQ2, 1 / SQ2]])
    j = np.arange(-J, J + 1)
    J1, J2 = np.meshgrid(j, j, indexing="ij")
    w = 2 * np.pi * np.stack([J1, J2], -1)
    val = np.ones(J1.shape)
    for k in range(4):
        val *= np.sinc(a[k] * (w @ U[k]) / 2 / np.pi)
    return val.sum()


@pytest.mark.parametrize("a", [(2.449, 2.449, 2.449, 2.449), (1.73, 1.73, 1.73, 1.73), (4.1, 2.2, 3.3, 1.5)])
def test_mass_matches_poisson_sum(orc, a):
    H, W = 24, 24
    out = orc.filter_scales(np.ones((H, W)), np.broadcast_to(a, (H, W, 4)).astype(np.float64), 1, "fast", 12)
    assert out[12, 12] == pytest.approx(_poisson_mass(a), abs=5e-7)


def test_region_filter_matches_full(orc):
    H, W = 40, 44
    f = I.uniform_image(H, W, 14)
    fld = I.srt_field(H, W, 14, (1.0, 3.0), (1.0, 4.0), corr_len=8.0)
    full = orc.filter(f, fld, orc.FIELD_SRT3, 2, method="fast", tile=11)
    part = orc.filter_region(f, fld, orc.FIELD_SRT3, 2, (9, 13, 12, 15))
    # different windows round differently (cancellation of the running sums): agree to ~1e-11
    np.testing.assert_allclose(part, full[9:21, 13:28], rtol=1e-10, atol=1e-12)


def test_iterates_approach_gaussian(orc):
    # impulse response of m passes with a/sqrt(m) vs the sampled Gaussian of the same covariance
    H = W = 41
    imp = np.zeros((H, W))
    imp[20, 20] = 1.0
    # per-pass widths sigma/sqrt(m) below ~0.7 px are dominated by lattice aliasing, so the
    # anisotropic case starts at sigma = 1.5
    for sigma, rho in ((1.0, 1.0), (2.0, 1.0), (1.5, 2.0), (3.0, 2.0)):
        fld = I.constant_srt_field(H, W, sigma, rho, 0.5)
        dists = []
        s = 2 * sigma**2
        lmax, lmin = s * rho / (1 + rho), s / (1 + rho)
        c, sn = math.cos(0.5), math.sin(0.5)
        Cm = np.array([[lmax * c * c + lmin * sn * sn, (lmax - lmin) * c * sn], [(lmax - lmin) * c * sn, lmin * c * c + lmax * sn * sn]])
        Ci = np.linalg.inv(Cm)
        y, x = np.mgrid[-20:21, -20:21].astype(np.float64)
        gauss = np.exp(-0.5 * (Ci[0, 0] * x * x + 2 * Ci[0, 1] * x * y + Ci[1, 1] * y * y)) / (2 * np.pi * math.sqrt(np.linalg.det(Cm)))
        for m in (1, 2, 3):
            out = orc.filter(imp, fld, orc.FIELD_SRT3, m, method="fast", tile=41)
            # the impulse response at n is beta(n - 20): flip to compare with the kernel
            dists.append(np.linalg.norm(out[::-1, ::-1] - gauss) / np.linalg.norm(gauss))
        assert dists[0] > dists[1] > dists[2], dists


def test_fourier_correlation_with_gaussian(orc, paper):
    """Normalised correlation (Parseval) between beta^{4,m}_{a/sqrt m} and the Gaussian of equal
    covariance; the paper reports a minimum of about 95% for m = 1 and 99% for m = 2."""
    U = np.array([[1.0, 0.0], [1 / SQ2, 1 / SQ2], [0.0, 1.0], [-1 / SQ2, 1 / SQ2]])
    g = np.linspace(-12, 12, 601)
    W1, W2 = np.meshgrid(g, g, indexing="ij")
    Wv = np.stack([W1, W2], -1)
    worst = {1: 1.0, 2: 1.0}
    for rho in (1.0, 2.0, 3.0, 4.0):
        for theta in np.linspace(0, math.pi / 4, 7):
            a, cl, _ = orc.scales_from_srt(1.0, rho, theta, eps=1e-9)
            if cl:
                continue
            s = 2.0
            lmax, lmin = s * rho / (1 + rho), s / (1 + rho)
            c, sn = math.cos(theta), math.sin(theta)
            Cm = np.array([[lmax * c * c + lmin * sn * sn, (lmax - lmin) * c * sn], [(lmax - lmin) * c * sn, lmin * c * c + lmax * sn * sn]])
            G = np.exp(-0.5 * np.einsum("...i,ij,...j->...", Wv, Cm, Wv))
            for m in (1, 2):
                B = np.ones(W1.shape)
                for k in range(4):
                    B *= np.sinc(a[k] / math.sqrt(m) * (Wv @ U[k]) / 2 / np.pi) ** m
                corr = (B * G).sum() / math.sqrt((B * B).sum() * (G * G).sum())
                worst[m] = min(worst[m], corr)
    assert worst[1] >= paper["gaussian_correlation_min"]["m1"]
    assert worst[2] >= paper["gaussian_correlation_min"]["m2"]
    assert worst[2] > worst[1]


# ----------------------------------------------------------------------------- boundary rules

@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_boundary_index_matches_numpy_pad(orc, N):
    # numpy.pad's 'edge' and 'symmetric' modes define replicate and the half-sample mirror
    P = 3 * N + 4
    base = np.arange(N)
    idx = np.arange(-P, N + P)
    np.testing.assert_array_equal(orc.boundary_index(idx, N, orc.BOUNDARY_REPLICATE), np.pad(base, P, mode="edge"))
    np.testing.assert_array_equal(orc.boundary_index(idx, N, orc.BOUNDARY_SYMMETRIC),
                                  np.pad(base, P, mode="symmetric"))


@pytest.mark.parametrize("boundary,mode", [(1, "edge"), (2, "symmetric")])
@pytest.mark.parametrize("shape,order", [((17, 13), 1), ((9, 22), 2), ((3, 4), 3)])
def test_boundary_equals_direct_sum_on_padded_image(orc, boundary, mode, shape, order):
    # direct sum over the lattice of the image extended by numpy.pad, one pass at a time
    H, W = shape
    f = I.uniform_image(H, W, 40 + H)
    fld = I.srt_field(H, W, 40 + H, (1.0, 5.0), (1.0, 4.0), corr_len=5.0)
    a, _ = orc.scales(fld, orc.FIELD_SRT3, order)
    rx, ry = orc.support_halfwidths(a)
    M = int(np.ceil(max(rx.max(), ry.max()))) + 6
    ref = f.astype(np.float64)
    for _ in range(order):
        ref = orc._pass(np.pad(ref, M, mode=mode), -M, -M, a, 0, 0, "brute", 0)
    got = orc.filter(f, fld, orc.FIELD_SRT3, order, method="fast", tile=5, boundary=boundary)
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("boundary", [1, 2])
def test_boundary_keeps_constants_integer_a1_a3(orc, boundary):
    # unit mass (a1, a3 integers) and a constant extension: the output is the constant up to the border
    H, W = 21, 18
    f = np.full((H, W), 3.5)
    for a in ([2.0, 1.3, 1.0, 2.2], [3.0, 0.8, 2.0, 4.9]):
        av = np.broadcast_to(a, (H, W, 4)).astype(np.float64)
        np.testing.assert_allclose(orc.filter_scales(f, av, 2, "fast", 7, boundary), 3.5, rtol=1e-12)
    zero = orc.filter_scales(f, av, 1, "fast", 7)
    assert zero[0, 0] < 3.0   # the zero rule loses mass at the corner


def test_symmetric_boundary_mirrors_with_the_image(orc):
    # a field and image mirrored left-right give the mirrored output when the box
    # directions are exchanged with their mirror images (u2 <-> u4)
    H, W = 15, 12
    f = I.uniform_image(H, W, 51).astype(np.float64)
    a = I.scales_field(H, W, 51, 0.6, 4.0).astype(np.float64)
    am = a[:, ::-1][..., [0, 3, 2, 1]]
    out = orc.filter_scales(f, a, 1, "fast", 6, orc.BOUNDARY_SYMMETRIC)
    outm = orc.filter_scales(f[:, ::-1], am, 1, "fast", 6, orc.BOUNDARY_SYMMETRIC)
    np.testing.assert_allclose(outm[:, ::-1], out, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("boundary", [1, 2])
def test_boundary_region_matches_full(orc, boundary):
    H, W = 36, 40
    f = I.uniform_image(H, W, 15)
    fld = I.srt_field(H, W, 15, (1.0, 4.0), (1.0, 4.0), corr_len=8.0)
    full = orc.filter(f, fld, orc.FIELD_SRT3, 3, method="fast", tile=11, boundary=boundary)
    for rect in [(0, 0, 7, 9), (30, 33, 6, 7), (10, 0, 5, 40)]:
        r0, c0, h, w = rect
        part = orc.filter_region(f, fld, orc.FIELD_SRT3, 3, rect, boundary=boundary)
        np.testing.assert_allclose(part, full[r0:r0 + h, c0:c0 + w], rtol=1e-10, atol=1e-12)
