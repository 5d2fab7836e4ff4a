"""GPU parity at the full workload sizes, on sampled output regions.

The oracle computes any output region of a large image exactly (it builds the
chain of regions each pass depends on), so the GPU result of the whole image,
in the launch configuration the benchmark times (default options), is
compared with the oracle on regions at the corners, the edges and inside,
element by element:

* 1024 x 1024 FP32, order 2, sigma 1-16 px, elongation 1-4 (correlation 64 px);
* 4096 x 4096 FP32 and uint16, order 2, sigma 1-32 px, elongation 1-6
  (correlation 256 px), every pre-integration variant;
* 4096 x 4096 feature-preserving smoothing (structure-tensor field, order 2),
  mirror and replicate boundaries, on regions at the corners, edges and inside;
* at 4096 x 4096 also regions around the pixels where the arithmetic is worst
  conditioned, picked on the host from the field: the smallest product of the
  pass scales (the difference divides by it), the largest reach (widest
  window), the largest window side^4 / prod(a) (the precision model of the
  running sums: error ~ eps G / prod(a) with G ~ side^4), the smallest product
  among pixels with a scale at the floor eps, and the pixel whose requested
  elongation is lowered the most (clamped);
* order 1 at 4096 x 4096 against the direct sum sum_k f[k] beta(n - k) itself at
  such pixels;
* an image, field and output that are strided crops of larger buffers (the
  layout the batched and serving benchmarks feed), single and batched.

Tolerance: |gpu - ref| <= 1e-5 max(|ref|, 1e-3 max|ref|) per pixel, RMS <= 1e-6
(FP64 and int64 pre-integration); the compensated FP32 variant is held to the
same bar; the FP32 difference is reported only.
"""
import numpy as np
import pytest

from paper_1003_2022_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1003_2022_amd as P  # noqa: E402

DEV = torch.device("cuda:0")


def rel(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    e = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return float(e.max()), float(np.sqrt(np.mean(e * e)))


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def run(ctx, img, tf, order, **opts):
    ti = torch.from_numpy(np.ascontiguousarray(img)).to(DEV)
    out = torch.empty(ti.shape, dtype=torch.float32, device=DEV)
    P.svf_filter(ctx, P.image_of(ti), P.field_of(tf, P.SVF_FIELD_SRT3), 4, order, P.default_opts(**opts),
                 P.image_of(out))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def compare(got, img, fld, order, regions, what, tol=1e-5, rms_tol=1e-6, check=True):
    worst = (0.0, 0.0)
    for r in regions:
        r0, c0, h, w = r
        ref = oracle.filter_region(img, fld, oracle.FIELD_SRT3, order, r)
        mx, rms = rel(got[r0:r0 + h, c0:c0 + w], ref)
        print(f"{what} region {r}: max rel {mx:.2e} rms {rms:.2e}", flush=True)
        worst = (max(worst[0], mx), max(worst[1], rms))
        if check:
            assert mx <= tol and rms <= rms_tol, f"{what} region {r}: max {mx:.2e} rms {rms:.2e}"
    return worst


def test_1024_order2(ctx):
    H = W = 1024
    img = I.uniform_image(H, W, 2000)
    fld = I.srt_field(H, W, 2000, (1.0, 16.0), (1.0, 4.0), corr_len=64.0)
    got = run(ctx, img, torch.from_numpy(fld).to(DEV), 2)
    assert np.isfinite(got).all()
    regions = [(0, 0, 80, 80), (0, 990, 50, 34), (500, 470, 64, 90), (1000, 0, 24, 100), (960, 960, 64, 64)]
    compare(got, img, fld, 2, regions, "1024^2 order 2")


@pytest.fixture(scope="module")
def big():
    H = W = 4096
    fld = I.srt_field(H, W, 3000, (1.0, 32.0), (1.0, 6.0))
    return fld, torch.from_numpy(fld).to(DEV)


REGIONS_4096 = [(0, 0, 64, 64), (0, 4040, 40, 56), (2000, 2040, 64, 72), (4060, 0, 36, 64), (4032, 4032, 64, 64)]


def cov_of_scales(a):
    """Covariance (C11, C12, C22) of the box spline with scales a (eq. (covariance_ZP))."""
    a2 = np.asarray(a, np.float64) ** 2
    return np.stack([2 * a2[..., 0] + a2[..., 1] + a2[..., 3], a2[..., 1] - a2[..., 3],
                     2 * a2[..., 2] + a2[..., 1] + a2[..., 3]], -1) / 24.0


def worst_pixels(fld, order, T=256):
    """Pixels where the filter's arithmetic is worst conditioned (see the module docstring)."""
    a, _ = oracle.scales(fld, oracle.FIELD_SRT3, order)   # per-pass scales
    H, W = a.shape[:2]
    pa = a.prod(-1)
    d = (a[..., 1] + a[..., 3]) / np.sqrt(2.0)
    reach = np.maximum(0.5 * (a[..., 0] + d), 0.5 * (a[..., 2] + d))
    nt = (H + T - 1) // T
    tiles = np.zeros((nt, nt))
    for i in range(nt):
        for j in range(nt):
            tiles[i, j] = reach[i * T:(i + 1) * T, j * T:(j + 1) * T].max()
    side = np.repeat(np.repeat(T + 2 * np.ceil(tiles) + 6, T, 0), T, 1)[:H, :W]
    floor = (a ** 2 <= oracle.DEFAULT_EPS * (1 + 1e-9)).any(-1)
    # clamped: the solved covariance of the whole filter differs most from the request
    af, _ = oracle.scales(fld, oracle.FIELD_SRT3, 1)
    f = fld.astype(np.float64)
    s_, rho, th = 2 * f[..., 0] ** 2, f[..., 1], f[..., 2]
    lmax, lmin = s_ * rho / (1 + rho), s_ / (1 + rho)
    c, sn = np.cos(th), np.sin(th)
    req = np.stack([lmax * c * c + lmin * sn * sn, (lmax - lmin) * c * sn, lmin * c * c + lmax * sn * sn], -1)
    clamp = np.abs(cov_of_scales(af) - req).max(-1) / s_
    picks = {
        "min prod(a)": np.argmin(pa),
        "max reach": np.argmax(reach),
        "side^4 / prod(a)": np.argmax(side ** 4 / pa),
        "floor, min prod(a)": np.argmin(np.where(floor, pa, np.inf)),
        "clamped most": np.argmax(clamp),
    }
    return {k: tuple(int(x) for x in np.unravel_index(v, (H, W))) for k, v in picks.items()}


def around(px, H=4096, W=4096, n=32):
    r0 = min(max(px[0] - n // 2, 0), H - n)
    c0 = min(max(px[1] - n // 2, 0), W - n)
    return (r0, c0, n, n)


@pytest.fixture(scope="module")
def worst(big):
    picks = worst_pixels(big[0], 2)
    print(f"worst-conditioned pixels (order 2): {picks}", flush=True)
    return sorted({around(p) for p in picks.values()})


@pytest.mark.parametrize("pre", ["f64", "f32c"])
def test_4096_f32(ctx, big, worst, pre):
    fld, tf = big
    img = I.uniform_image(4096, 4096, 3000)
    p = P.SVF_PRE_F64 if pre == "f64" else P.SVF_PRE_F32C
    got = run(ctx, img, tf, 2, preint=p)
    assert np.isfinite(got).all()
    compare(got, img, fld, 2, REGIONS_4096 + worst, f"4096^2 f32 {pre}")


@pytest.mark.parametrize("pre", ["i64", "f64", "f32c"])
def test_4096_u16(ctx, big, worst, pre):
    fld, tf = big
    img = I.uniform_image(4096, 4096, 3001, dtype="u16")
    p = {"i64": P.SVF_PRE_I64, "f64": P.SVF_PRE_F64, "f32c": P.SVF_PRE_F32C}[pre]
    got = run(ctx, img, tf, 2, preint=p)
    assert np.isfinite(got).all()
    compare(got, img, fld, 2, REGIONS_4096[1:4] + worst, f"4096^2 u16 {pre}")


def test_4096_order1_direct_sum(ctx, big):
    """Order 1 on the benchmark's image and field against the direct sum at the
    worst-conditioned pixels of order 1, the image corners and a centre pixel."""
    fld, tf = big
    img = I.uniform_image(4096, 4096, 3000)
    got = run(ctx, img, tf, 1)
    pix = list(worst_pixels(fld, 1).values()) + [(0, 0), (0, 4095), (4095, 0), (4095, 4095), (2048, 2048)]
    for (r, c) in pix:
        ref = float(oracle.filter_region(img, fld, oracle.FIELD_SRT3, 1, (r, c, 1, 1), method="brute")[0, 0])
        e = abs(float(got[r, c]) - ref) / max(abs(ref), 1e-3)
        print(f"order 1 direct sum at {(r, c)}: gpu {got[r, c]:.9f} direct {ref:.9f} rel {e:.2e}", flush=True)
        assert e <= 1e-5


def test_strided_views(ctx, big):
    """Image, field and output as crops of larger buffers (row strides above W * C):
    the same result as contiguous copies, bit for bit, single and batched, and the
    oracle's on regions of the crop."""
    fld, tf = big
    img = I.uniform_image(4096, 4096, 3000)
    ti = torch.from_numpy(img).to(DEV)
    r0, c0, h, w = 1000, 333, 700, 1200
    vi, vf = ti[r0:r0 + h, c0:c0 + w], tf[r0:r0 + h, c0:c0 + w]
    assert vi.stride(0) == 4096 and vf.stride(0) == 4096 * 3
    obuf = torch.full((2000, 2000), float("nan"), dtype=torch.float32, device=DEV)
    vo = obuf[10:10 + h, 20:20 + w]
    o = P.default_opts(tile=256)
    P.svf_filter(ctx, P.image_of(vi), P.field_of(vf, P.SVF_FIELD_SRT3), 4, 2, o, P.image_of(vo))
    ci, cf = vi.contiguous(), vf.contiguous()
    co = torch.empty((h, w), dtype=torch.float32, device=DEV)
    P.svf_filter(ctx, P.image_of(ci), P.field_of(cf, P.SVF_FIELD_SRT3), 4, 2, o, P.image_of(co))
    # batched: two strided crops in one launch
    vi2, vf2 = ti[3000:3512, 2500:3012], tf[3000:3512, 2500:3012]
    bo = [torch.full((2000, 2000), float("nan"), dtype=torch.float32, device=DEV) for _ in range(2)]
    bv = [bo[0][5:5 + h, 7:7 + w], bo[1][0:512, 100:612]]
    P.svf_filter_batch(ctx, [P.image_of(vi), P.image_of(vi2)],
                       [P.field_of(vf, P.SVF_FIELD_SRT3), P.field_of(vf2, P.SVF_FIELD_SRT3)], [2, 2], o,
                       [P.image_of(t) for t in bv], torch.cuda.current_stream())
    co2 = torch.empty((512, 512), dtype=torch.float32, device=DEV)
    P.svf_filter(ctx, P.image_of(vi2.contiguous()), P.field_of(vf2.contiguous(), P.SVF_FIELD_SRT3), 4, 2, o,
                 P.image_of(co2))
    torch.cuda.synchronize()
    got = vo.cpu().numpy()
    assert np.array_equal(got, co.cpu().numpy()), "strided views differ from contiguous copies"
    assert torch.isnan(obuf[:10]).all() and torch.isnan(obuf[10 + h:]).all(), "written outside the output view"
    assert torch.isnan(obuf[10:10 + h, :20]).all() and torch.isnan(obuf[10:10 + h, 20 + w:]).all()
    for k, ref in enumerate((co, co2)):
        d = np.abs(bv[k].cpu().numpy().astype(np.float64) - ref.cpu().numpy())
        print(f"batched strided crop {k}: max abs diff from svf_filter {d.max():.2e}", flush=True)
        assert np.array_equal(bv[k].cpu().numpy(), ref.cpu().numpy()), f"batched crop {k} differs from svf_filter"
    sub = img[r0:r0 + h, c0:c0 + w]
    sfl = fld[r0:r0 + h, c0:c0 + w]
    compare(got, sub, sfl, 2, [(0, 0, 48, 48), (300, 500, 40, 64), (652, 1152, 48, 48)], "strided crop")


def test_4096_fd_fp32_reported(ctx, big):
    fld, tf = big
    img = I.uniform_image(4096, 4096, 3000)
    got = run(ctx, img, tf, 2, fd_fp32=1)
    assert np.isfinite(got).all()
    mx, rms = compare(got, img, fld, 2, REGIONS_4096[2:3], "4096^2 f32 fd_fp32", check=False)
    print(f"FP32 finite difference (comparison variant): max rel {mx:.2e} rms {rms:.2e}")


@pytest.mark.parametrize("boundary", [P.SVF_BOUNDARY_SYMMETRIC, P.SVF_BOUNDARY_REPLICATE])
def test_4096_smooth_adaptive(ctx, boundary):
    # the smoothing leg's workload: noisy stripes, structure-tensor field, order 2; the
    # oracle smooths a crop grown by 64 px around each region (clipped at the image:
    # the crop's own border is then the image's, elsewhere it is beyond every reach)
    H = W = 4096
    img = I.oriented_image(H, W, 3002, noise=0.1)
    ti = torch.from_numpy(img).to(DEV)
    out = torch.empty_like(ti)
    prm = P.st_params(sigma_w=2.0, gain=120.0, a_flat=1.0)
    P.svf_smooth_adaptive(ctx, P.image_of(ti), prm, 2, P.default_opts(boundary=boundary), P.image_of(out))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for (r0, c0, h, w) in [(0, 0, 80, 80), (0, 2048, 40, 100), (1500, 4020, 90, 76), (4030, 4030, 66, 66)]:
        R0, C0 = max(0, r0 - 64), max(0, c0 - 64)
        R1, C1 = min(H, r0 + h + 64), min(W, c0 + w + 64)
        ref = oracle.smooth_adaptive(img[R0:R1, C0:C1], 2.0, 1, 120.0, 0.0, 1.0, 2, boundary=boundary)
        ref = ref[r0 - R0:r0 - R0 + h, c0 - C0:c0 - C0 + w]
        mx, rms = rel(got[r0:r0 + h, c0:c0 + w], ref)
        print(f"smooth 4096 boundary {boundary} region {(r0, c0, h, w)}: max rel {mx:.2e} rms {rms:.2e}", flush=True)
        assert mx <= 1e-5 and rms <= 1e-6
