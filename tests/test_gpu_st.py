"""GPU parity of the feature-preserving smoothing (Sec. 4.2) against the CPU
FP64 oracle: the structure tensor J, the (sigma, rho, theta) field it implies,
and the smoothed image.

Tolerances: J per pixel |dJ_k| <= 1e-5 * max(tr J, 1e-3 max tr J) (the GPU
rounds the gradient products to float32 before the window, relative 6e-8,
and |J12| <= tr J / 2); the field through the filter covariance it describes,
|dC_k| <= 1e-5 * s, and sigma to 1e-5 relative (theta alone is undefined where
the eigenvalues are close, rho alone where the smaller one is near 0); the
smoothed image to the filter's own bar (1e-5 per pixel, 1e-6 RMS).
"""
import math

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


def gpu_st(ctx, img, params, **opts):
    H, W = img.shape[:2]
    J = torch.full((H, W, 3), float("nan"), dtype=torch.float32, device=DEV)
    F = torch.full((H, W, 3), float("nan"), dtype=torch.float32, device=DEV)
    P.svf_structure_tensor(ctx, P.image_of(to_dev(img)), params, P.default_opts(**opts), J, F)
    torch.cuda.synchronize()
    return J.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(np.float64)


def check_tensor(got, ref, what):
    tr = ref[..., 0] + ref[..., 2]
    scale = np.maximum(tr, 1e-3 * tr.max())[..., None]
    e = np.abs(got - ref) / scale
    print(f"{what}: J max rel {e.max():.3e}", flush=True)
    assert np.isfinite(got).all() and e.max() <= 1e-5, what


def cov_of(F):
    s = 2.0 * F[..., 0] ** 2
    rho, th = F[..., 1], F[..., 2]
    l1, l2 = s * rho / (1 + rho), s / (1 + rho)
    c, sn = np.cos(th), np.sin(th)
    return np.stack([l1 * c * c + l2 * sn * sn, (l1 - l2) * c * sn, l1 * sn * sn + l2 * c * c], -1), s


def check_field(got, ref, what):
    Cg, _ = cov_of(got)
    Cr, s = cov_of(ref)
    e = np.abs(Cg - Cr) / s[..., None]
    es = np.abs(got[..., 0] - ref[..., 0]) / ref[..., 0]
    print(f"{what}: field cov max rel {e.max():.3e}, sigma max rel {es.max():.3e}", flush=True)
    assert np.isfinite(got).all() and e.max() <= 1e-5 and es.max() <= 1e-5, what
    assert (got[..., 1] >= 1.0).all() and (got[..., 2] >= 0).all() and (got[..., 2] < math.pi + 1e-6).all()


# (H, W, channels, dtype, boundary, sigma_w, order_w)
CASES = [
    (96, 130, 1, "f32", P.SVF_BOUNDARY_SYMMETRIC, 2.0, 1),
    (70, 50, 3, "f32", P.SVF_BOUNDARY_REPLICATE, 1.5, 2),
    (64, 64, 1, "u16", P.SVF_BOUNDARY_ZERO, 3.0, 1),
    (300, 257, 1, "f32", P.SVF_BOUNDARY_SYMMETRIC, 4.0, 3),
    (5, 7, 2, "f32", P.SVF_BOUNDARY_SYMMETRIC, 2.0, 1),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_tensor_and_field_match_oracle(ctx, case):
    H, W, ch, dt, b, sw, ow = CASES[case]
    img = I.oriented_image(H, W, 6000 + case, dtype=dt, channels=ch)
    gain = 30.0 if dt == "f32" else 30.0 / 65535.0 ** 2
    params = P.st_params(sigma_w=sw, order_w=ow, gain=gain)
    print(f"case {case}: {H}x{W}x{ch} {dt} boundary {b} sigma_w {sw} order_w {ow}", flush=True)
    J, F = gpu_st(ctx, img, params, boundary=b, tile=64)
    Jr = oracle.structure_tensor(img, sw, ow, b)
    check_tensor(J, Jr, f"case {case}")
    Fr = oracle.st_field(img, sw, ow, gain=gain, boundary=b).astype(np.float64)
    check_field(F, Fr, f"case {case}")


def test_flat_region(ctx):
    # a noise-free flat square far from the stripes: J there is the running sums'
    # rounding residue only (~1e-14), below lambda_zero on both sides (flat rule);
    # pixels whose eigenvalues lie near lambda_zero (the edge of the window's
    # reach) may take either rule and are left out of the comparison
    H, W = 120, 140
    lz, gain = 1e-9, 10.0
    img = I.oriented_image(H, W, 6100, noise=0.05, flat_box=(30, 40, 60, 60))
    params = P.st_params(sigma_w=1.5, gain=gain, lambda_zero=lz, a_flat=1.7)
    J, F = gpu_st(ctx, img, params, boundary=P.SVF_BOUNDARY_SYMMETRIC)
    Jr = oracle.structure_tensor(img, 1.5, 1, P.SVF_BOUNDARY_SYMMETRIC)
    Fr = oracle.st_field(img, 1.5, 1, gain=gain, lambda_zero=lz, a_flat=1.7,
                         boundary=P.SVF_BOUNDARY_SYMMETRIC).astype(np.float64)
    inner = (slice(48, 72), slice(58, 82))
    assert gain * np.abs(J[inner]).max() < lz
    assert (F[inner][..., 0] == np.float32(math.sqrt(1.7 ** 2 / 6.0))).all()
    assert (F[inner][..., 1] == 1.0).all() and (F[inner][..., 2] == 0.0).all()
    M = gain * np.stack([np.stack([Jr[..., 0], Jr[..., 1]], -1), np.stack([Jr[..., 1], Jr[..., 2]], -1)], -2)
    lam = np.linalg.eigvalsh(M)
    near = ((lam > lz / 4) & (lam < 4 * lz)).any(-1)
    print(f"pixels near lambda_zero: {int(near.sum())}", flush=True)
    keep = ~near
    check_field(F[keep][None], Fr[keep][None], "flat box")


@pytest.mark.parametrize("order,dt,preint", [(2, "f32", P.SVF_PRE_F64), (1, "u16", P.SVF_PRE_I64),
                                             (3, "f32", P.SVF_PRE_F64)])
def test_smooth_adaptive_matches_oracle(ctx, order, dt, preint):
    H, W = 110, 150
    img = I.oriented_image(H, W, 6200 + order, dtype=dt, noise=0.1)
    gain = 120.0 if dt == "f32" else 120.0 / 65535.0 ** 2
    params = P.st_params(sigma_w=2.0, gain=gain, a_flat=1.0)
    b = P.SVF_BOUNDARY_SYMMETRIC
    out = torch.full((H, W), float("nan"), dtype=torch.float32, device=DEV)
    st, rep = P.svf_smooth_adaptive(ctx, P.image_of(to_dev(img)), params, order,
                                    P.default_opts(boundary=b, preint=preint, tile=64), P.image_of(out), report=True)
    torch.cuda.synchronize()
    assert st == P.SVF_OK, ctx.last_error()
    print(f"report: clamped {rep.clamped_px} eps {rep.eps_active_px} reach {rep.max_reach_px:.1f}", flush=True)
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.smooth_adaptive(img, 2.0, 1, gain, 0.0, 1.0, order, boundary=b)
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    e = np.abs(got - ref) / scale
    print(f"smooth order {order} {dt}: max rel {e.max():.3e} rms {np.sqrt(np.mean(e ** 2)):.3e}", flush=True)
    assert e.max() <= 1e-5 and np.sqrt(np.mean(e ** 2)) <= 1e-6


def test_params_and_outputs_rejected(ctx):
    img = to_dev(I.oriented_image(16, 16, 1))
    F = torch.empty((16, 16, 3), dtype=torch.float32, device=DEV)
    for kw in [dict(sigma_w=0.0), dict(order_w=4), dict(gain=-1.0), dict(lambda_zero=-1.0), dict(a_flat=0.0)]:
        with pytest.raises(P.SvfError) as ei:
            P.svf_structure_tensor(ctx, P.image_of(img), P.st_params(**kw), None, None, F)
        assert ei.value.status == P.SVF_EINVAL
    with pytest.raises(P.SvfError):
        P.svf_structure_tensor(ctx, P.image_of(img), P.st_params(), None, None, None)
