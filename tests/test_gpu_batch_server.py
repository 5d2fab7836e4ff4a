"""GPU tests of the batched launch path and of the serving loop.

* svf_filter_batch (eager and HIP-graph replays) equals per-image svf_filter
  with the same options to 1e-6 (the batched pre-integration sums in another
  order; the outputs are float32), every replay equals the first bit for bit,
  and the oracle to 1e-5;
* the server: every request's output is bitwise identical whether it is served
  alone or in a mix, equals svf_filter with the same options to 1e-6, and
  equals the CPU FP64 oracle to 1e-5 (relative, per pixel);
* admission: a request larger than the memory budget is rejected at submit.
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


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel_err(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return float(np.max(np.abs(got - ref) / scale))


# (H, W, channels, order, sigma range, rho range)
CASES = [
    (97, 130, 1, 2, (1, 8), (1, 4)),
    (64, 64, 1, 1, (1, 4), (1, 3)),
    (150, 90, 3, 3, (1, 6), (1, 6)),
    (33, 257, 1, 2, (1, 12), (1, 4)),
    (201, 199, 3, 1, (1, 16), (1, 6)),
    (8, 5, 1, 3, (1, 3), (1, 2)),
]


def make_case(i, H, W, ch, order, sr, rr):
    img = I.uniform_image(H, W, 4000 + i, channels=ch)
    fld = I.srt_field(H, W, 4000 + i, sr, rr, corr_len=max(4.0, min(H, W) / 4))
    return img, fld


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def cases():
    out = []
    for i, (H, W, ch, order, sr, rr) in enumerate(CASES):
        img, fld = make_case(i, H, W, ch, order, sr, rr)
        out.append((img, fld, order, to_dev(img), to_dev(fld)))
    return out


def single(ctx, timg, tfld, order, **opts):
    out = torch.empty(timg.shape, dtype=torch.float32, device=DEV)
    P.svf_filter(ctx, P.image_of(timg), P.field_of(tfld, P.SVF_FIELD_SRT3), 4, order, P.default_opts(**opts),
                 P.image_of(out))
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_matches_single_and_oracle(ctx, cases, use_graph):
    outs = [torch.zeros(c[3].shape, dtype=torch.float32, device=DEV) for c in cases]
    stream = torch.cuda.Stream()
    o = P.default_opts(tile=256)
    reps = 3 if use_graph else 1
    first = []
    for rep in range(reps):
        for t in outs:
            t.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            P.svf_filter_batch(ctx, [P.image_of(c[3]) for c in cases],
                               [P.field_of(c[4], P.SVF_FIELD_SRT3) for c in cases], [c[2] for c in cases], o,
                               [P.image_of(t) for t in outs], stream, use_graph)
        stream.synchronize()
        for i, c in enumerate(cases):
            ref = single(ctx, c[3], c[4], c[2], tile=256)
            got = outs[i].cpu().numpy()
            e = rel_err(got, ref)
            print(f"graph={use_graph} rep {rep} case {i}: vs single {e:.2e}", flush=True)
            assert e <= 1e-6
            if rep == 0:
                first.append(got)
            else:
                assert np.array_equal(got, first[i]), f"replay {rep} differs from the first"
    for i in (0, 2):
        img, fld, order = cases[i][:3]
        ref = oracle.filter(img, fld, oracle.FIELD_SRT3, order)
        assert rel_err(outs[i].cpu().numpy(), ref) <= 1e-5


def _server(ctx, budget=8 << 30, inflight=8):
    cfg = P.svf_server_cfg()
    cfg.max_inflight = inflight
    cfg.queue_capacity = 64
    cfg.hbm_budget_bytes = budget
    cfg.opts = P.default_opts()
    ctx.check(P.lib().svf_server_start(ctx.ptr, C.byref(cfg)))


def _submit(ctx, timg, tfld, order, out):
    req = P.svf_request()
    req.in_ = P.image_of(timg)
    req.field = P.field_of(tfld, P.SVF_FIELD_SRT3)
    req.order = order
    req.out = P.image_of(out)
    rid = C.c_uint64()
    ctx.check(P.lib().svf_server_submit(ctx.ptr, C.byref(req), C.byref(rid)))
    return rid.value


def _wait(ctx, rid):
    res = P.svf_result()
    st = P.lib().svf_server_wait(ctx.ptr, rid, C.byref(res), 120.0)
    assert st == P.SVF_OK and res.done and res.status == P.SVF_OK, (st, res.status)
    return res


def test_server_mix_equals_alone(ctx, cases):
    # alone: one request at a time through the server
    alone = []
    _server(ctx)
    try:
        for c in cases:
            out = torch.zeros(c[3].shape, dtype=torch.float32, device=DEV)
            _wait(ctx, _submit(ctx, c[3], c[4], c[2], out))
            alone.append(out.cpu().numpy())
    finally:
        P.lib().svf_server_stop(ctx.ptr)
    # mix: everything submitted at once, twice over (requests join while others run)
    _server(ctx, inflight=4)
    try:
        outs = [torch.zeros(c[3].shape, dtype=torch.float32, device=DEV) for c in cases + cases]
        ids = [_submit(ctx, c[3], c[4], c[2], outs[i]) for i, c in enumerate(cases + cases)]
        res = [_wait(ctx, i) for i in ids]
        st = P.svf_server_stats_t()
        P.lib().svf_server_stats(ctx.ptr, C.byref(st))
        print(f"server: {st.completed} done in {st.steps} steps", flush=True)
        assert st.completed >= len(ids)
    finally:
        P.lib().svf_server_stop(ctx.ptr)
    for i, c in enumerate(cases + cases):
        got = outs[i].cpu().numpy()
        assert np.array_equal(got, alone[i % len(cases)]), f"request {i}: mix differs from alone"
        assert res[i].t_done_us >= res[i].t_admit_us >= res[i].t_submit_us
    for i, c in enumerate(cases):
        ref = single(ctx, c[3], c[4], c[2], tile=256)
        assert rel_err(alone[i], ref) <= 1e-6
    img, fld, order = cases[2][:3]
    assert rel_err(alone[2], oracle.filter(img, fld, oracle.FIELD_SRT3, order)) <= 1e-5


def test_server_rejects_over_budget(ctx, cases):
    _server(ctx, budget=1 << 20)   # 1 MiB: no request fits
    try:
        c = cases[0]
        out = torch.zeros(c[3].shape, dtype=torch.float32, device=DEV)
        req = P.svf_request()
        req.in_ = P.image_of(c[3])
        req.field = P.field_of(c[4], P.SVF_FIELD_SRT3)
        req.order = 1
        req.out = P.image_of(out)
        rid = C.c_uint64()
        st = P.lib().svf_server_submit(ctx.ptr, C.byref(req), C.byref(rid))
        assert st == P.SVF_ENOMEM
        stats = P.svf_server_stats_t()
        P.lib().svf_server_stats(ctx.ptr, C.byref(stats))
        assert stats.rejected == 1
    finally:
        P.lib().svf_server_stop(ctx.ptr)
