"""GPU parity of the boundary rules (replicate, half-sample mirror) against the
CPU FP64 oracle, whose every pass is the direct sum over the image extended by
the same rule.  Same tolerances as the zero rule: per pixel 1e-5 relative (FP64
sums), RMS 1e-6; batched, banded and served launches agree with svf_filter
(bit for bit for bands, 1e-6 for the batched launch).
"""
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
RULES = [P.SVF_BOUNDARY_REPLICATE, P.SVF_BOUNDARY_SYMMETRIC]


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    e = np.abs(got - ref) / scale
    return float(e.max()), float(np.sqrt(np.mean(e ** 2)))


def check(got, ref, what, tol=1e-5, rms_tol=1e-6):
    assert np.isfinite(got).all(), what
    m, r = rel(got, ref)
    print(f"{what}: max rel {m:.3e} rms {r:.3e}", flush=True)
    assert m <= tol and r <= rms_tol, what


def run(ctx, img, fld, kind, order, **opts):
    out, st, _ = P.filter_tensor(ctx, to_dev(img), to_dev(fld), kind, order=order, report=True, **opts)
    torch.cuda.synchronize()
    assert st == P.SVF_OK, ctx.last_error()
    return out.cpu().numpy()


# (H, W, channels, order, dtype, preint, tile, sigma range): ragged tiles, several
# tiles, images narrower than the support (several reflections), a single pixel
CASES = [
    (97, 130, 1, 2, "f32", P.SVF_PRE_F64, 64, (1, 8)),
    (150, 90, 3, 3, "f32", P.SVF_PRE_F64, 64, (1, 6)),
    (200, 333, 1, 1, "f32", P.SVF_PRE_F64, 128, (1, 16)),
    (8, 5, 1, 3, "f32", P.SVF_PRE_F64, 64, (1, 4)),
    (3, 200, 2, 2, "f32", P.SVF_PRE_F64, 64, (1, 5)),
    (1, 1, 1, 2, "f32", P.SVF_PRE_F64, 64, (1, 3)),
    (120, 77, 1, 2, "u16", P.SVF_PRE_I64, 64, (1, 8)),
]


@pytest.mark.parametrize("boundary", RULES)
@pytest.mark.parametrize("case", range(len(CASES)))
def test_boundary_matches_oracle(ctx, boundary, case):
    H, W, ch, order, dt, pre, tile, sr = CASES[case]
    img = I.uniform_image(H, W, 5000 + case, dt, channels=ch)
    fld = I.srt_field(H, W, 5000 + case, sr, (1.0, 5.0), corr_len=max(4.0, min(H, W) / 3))
    print(f"case {case}: {H}x{W}x{ch} order {order} {dt} preint {pre} boundary {boundary}", flush=True)
    got = run(ctx, img, fld, P.SVF_FIELD_SRT3, order, preint=pre, tile=tile, boundary=boundary)
    ref = oracle.filter(img, fld, oracle.FIELD_SRT3, order, boundary=boundary)
    check(got, ref, f"case {case} boundary {boundary}")


@pytest.mark.parametrize("boundary", RULES)
def test_boundary_f32c_sums(ctx, boundary):
    H, W = 140, 150
    img = I.uniform_image(H, W, 5100)
    fld = I.srt_field(H, W, 5100, (1.0, 12.0), (1.0, 4.0), corr_len=25.0)
    got = run(ctx, img, fld, P.SVF_FIELD_SRT3, 2, preint=P.SVF_PRE_F32C, tile=64, boundary=boundary)
    ref = oracle.filter(img, fld, oracle.FIELD_SRT3, 2, boundary=boundary)
    check(got, ref, f"f32c boundary {boundary}", tol=1e-4, rms_tol=1e-5)


@pytest.mark.parametrize("boundary", RULES)
def test_boundary_keeps_constants(ctx, boundary):
    # pass scales a1, a3 integers (unit mass; order 1, since later orders divide the
    # scales by sqrt(order)) and a constant extension: constant everywhere, borders included
    H, W = 90, 70
    img = np.full((H, W), 0.75, dtype=np.float32)
    sc = np.broadcast_to(np.array([3.0, 2.2, 2.0, 1.7], np.float32), (H, W, 4)).copy()
    got = run(ctx, img, sc, P.SVF_FIELD_SCALES4, 1, boundary=boundary)
    np.testing.assert_allclose(got, 0.75, rtol=1e-6)


def test_boundary_bands_bitwise_and_corner(ctx):
    # 1024 x 768, 64-px tiles: 16 tile rows, 4 bands; windows reach across bands and the borders
    H, W = 1024, 768
    img = I.uniform_image(H, W, 5200)
    fld = I.srt_field(H, W, 5200, (1.0, 30.0), (1.0, 5.0), corr_len=96.0)
    ti, tf = to_dev(img), to_dev(fld)
    outs = {}
    for bands in (1, 4):
        out = torch.full(ti.shape, float("nan"), dtype=torch.float32, device=DEV)
        P.svf_filter(ctx, P.image_of(ti), P.field_of(tf, P.SVF_FIELD_SRT3), 4, 2,
                     P.default_opts(tile=64, bands=bands, boundary=P.SVF_BOUNDARY_SYMMETRIC), P.image_of(out))
        torch.cuda.synchronize()
        outs[bands] = out.cpu().numpy()
    assert np.array_equal(outs[4], outs[1])
    for r in [(0, 0, 40, 48), (H - 40, W - 30, 40, 30)]:
        ref = oracle.filter_region(img, fld, oracle.FIELD_SRT3, 2, r, boundary=P.SVF_BOUNDARY_SYMMETRIC)
        check(outs[4][r[0]:r[0] + r[2], r[1]:r[1] + r[3]], ref, f"bands corner {r}")


def test_boundary_batch_and_server(ctx):
    shapes = [(97, 130, 1, 2), (8, 5, 1, 3), (60, 61, 3, 1)]
    cases = []
    for i, (H, W, ch, order) in enumerate(shapes):
        img = I.uniform_image(H, W, 5300 + i, channels=ch)
        fld = I.srt_field(H, W, 5300 + i, (1.0, 6.0), (1.0, 4.0), corr_len=max(4.0, min(H, W) / 3))
        cases.append((img, fld, order, to_dev(img), to_dev(fld)))
    b = P.SVF_BOUNDARY_SYMMETRIC
    singles = [run(ctx, c[0], c[1], P.SVF_FIELD_SRT3, c[2], tile=256, boundary=b) for c in cases]
    outs = [torch.zeros(c[3].shape, dtype=torch.float32, device=DEV) for c in cases]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        P.svf_filter_batch(ctx, [P.image_of(c[3]) for c in cases], [P.field_of(c[4], P.SVF_FIELD_SRT3) for c in cases],
                           [c[2] for c in cases], P.default_opts(tile=256, boundary=b), [P.image_of(t) for t in outs],
                           stream, False)
    stream.synchronize()
    for i, c in enumerate(cases):
        assert rel(outs[i].cpu().numpy(), singles[i])[0] <= 1e-6
        check(singles[i], oracle.filter(c[0], c[1], oracle.FIELD_SRT3, c[2], boundary=b), f"batch case {i}")
    cfg = P.svf_server_cfg()
    cfg.max_inflight = 4
    cfg.queue_capacity = 16
    cfg.hbm_budget_bytes = 1 << 30
    cfg.use_graph = 1
    cfg.opts = P.default_opts(boundary=b)
    P.svf_server_start(ctx, cfg)
    try:
        souts = [torch.zeros(c[3].shape, dtype=torch.float32, device=DEV) for c in cases]
        ids = [P.svf_server_submit(ctx, P.server_request(c[3], c[4], P.SVF_FIELD_SRT3, c[2], souts[i]))
               for i, c in enumerate(cases)]
        for rid in ids:
            res = P.svf_server_wait(ctx, rid, 120.0)
            assert res.done and res.status == P.SVF_OK
    finally:
        P.lib().svf_server_stop(ctx.ptr)
    for i in range(len(cases)):
        assert np.array_equal(souts[i].cpu().numpy(), outs[i].cpu().numpy()), f"server request {i}"


def test_boundary_rejected_out_of_range(ctx):
    img = to_dev(I.uniform_image(16, 16, 1))
    fld = to_dev(I.srt_field(16, 16, 1))
    out = torch.empty_like(img)
    for b in (-1, 3):
        with pytest.raises(P.SvfError) as ei:
            P.svf_filter(ctx, P.image_of(img), P.field_of(fld, P.SVF_FIELD_SRT3), 4, 1, P.default_opts(boundary=b),
                         P.image_of(out))
        assert ei.value.status == P.SVF_EINVAL
