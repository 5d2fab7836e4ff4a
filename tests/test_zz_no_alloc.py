"""GPU: svf_filter_noalloc, the filter with the library's fixed workspace (no
allocation), against svf_filter and the oracle: two calls in a row, the second
with a smaller input (the fixed workspace keeps the first call's contents), and
the refusals (an image too large for the workspace, the table scale map)."""
import ctypes as C

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


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel_check(got, ref, what):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    rel = np.abs(got - ref) / scale
    rms = np.sqrt(np.mean(rel ** 2))
    print(f"{what}: max rel {rel.max():.2e} rms {rms:.2e}", flush=True)
    assert rel.max() <= 1e-5 and rms <= 1e-6


def both(ctx, img, fld, kind, order):
    """(svf_filter_noalloc output, svf_filter output), called through the C ABI."""
    ti, tf = to_dev(img), to_dev(fld)
    o = P.default_opts()
    s = torch.cuda.current_stream()
    a = torch.full(ti.shape, float("nan"), dtype=torch.float32, device=DEV)
    st = P.lib().svf_filter_noalloc(ctx.ptr, C.byref(P.image_of(ti)), C.byref(P.field_of(tf, kind)), 4, order,
                                    C.byref(o), C.byref(P.image_of(a)), C.c_void_p(s.cuda_stream))
    assert st == P.SVF_OK, ctx.last_error()
    b = torch.full(ti.shape, float("nan"), dtype=torch.float32, device=DEV)
    P.svf_filter(ctx, P.image_of(ti), P.field_of(tf, kind), 4, order, o, P.image_of(b), s)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_two_calls(ctx):
    # first: 300 x 420, order 2, (sigma, rho, theta) field
    img = I.uniform_image(300, 420, 6100)
    fld = I.srt_field(300, 420, 6100, (1.0, 12.0), (1.0, 5.0), corr_len=40.0)
    got, ref_gpu = both(ctx, img, fld, P.SVF_FIELD_SRT3, 2)
    assert np.array_equal(got, ref_gpu), "svf_filter_noalloc differs from svf_filter"
    rel_check(got, oracle.filter(img, fld, oracle.FIELD_SRT3, 2), "noalloc 300x420 order 2")
    # second, smaller: 120 x 90, two channels, order 1, covariance field
    img2 = I.uniform_image(120, 90, 6101, channels=2)
    f2 = I.srt_field(120, 90, 6101, (1.0, 6.0), (1.0, 3.0), corr_len=20.0)
    cov = _cov(f2).astype(np.float32)
    got2, ref2_gpu = both(ctx, img2, cov, P.SVF_FIELD_COV3, 1)
    assert np.array_equal(got2, ref2_gpu), "second call differs from svf_filter"
    rel_check(got2, oracle.filter(img2, cov, oracle.FIELD_COV3, 1), "noalloc 120x90x2 order 1")


def _cov(f):
    s = 2.0 * f[..., 0].astype(np.float64) ** 2
    rho, th = f[..., 1].astype(np.float64), f[..., 2].astype(np.float64)
    lmax, lmin = s * rho / (1 + rho), s / (1 + rho)
    c, sn = np.cos(th), np.sin(th)
    return np.stack([lmax * c * c + lmin * sn * sn, (lmax - lmin) * c * sn, lmin * c * c + lmax * sn * sn], -1)


def test_noalloc_refusals(ctx):
    s = torch.cuda.current_stream()
    big = torch.zeros((2048, 2048), dtype=torch.float32, device=DEV)
    bf = to_dev(I.srt_field(2048, 2048, 6102, (1.0, 4.0), (1.0, 2.0), corr_len=64.0))
    out = torch.full_like(big, 7.0)
    o = P.default_opts()
    st = P.lib().svf_filter_noalloc(ctx.ptr, C.byref(P.image_of(big)), C.byref(P.field_of(bf, P.SVF_FIELD_SRT3)), 4, 1,
                                    C.byref(o), C.byref(P.image_of(out)), C.c_void_p(s.cuda_stream))
    assert st == P.SVF_ENOMEM and "fixed maximum" in ctx.last_error()
    small = to_dev(I.uniform_image(32, 32, 6103))
    sf = to_dev(I.srt_field(32, 32, 6103))
    so = torch.empty_like(small)
    ol = P.default_opts(scale_map=P.SVF_SCALE_LUT)
    st = P.lib().svf_filter_noalloc(ctx.ptr, C.byref(P.image_of(small)), C.byref(P.field_of(sf, P.SVF_FIELD_SRT3)), 4,
                                    1, C.byref(ol), C.byref(P.image_of(so)), C.c_void_p(s.cuda_stream))
    assert st == P.SVF_EUNSUPPORTED
    torch.cuda.synchronize()
    assert bool((out == 7.0).all()), "a refused call wrote its output"
