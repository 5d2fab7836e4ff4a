"""Python binding of libsvf (include/svf.h): space-variant elliptical filtering
with the four-directional box spline on MI355X (gfx950).

Thin ctypes marshalling only: every step of the filter runs in the library's
HIP kernels.  Torch tensors provide device memory and streams.  The functions
keep the C names (``svf_filter``, ``svf_preintegrate``, ...); the helpers
``image_of`` / ``field_of`` build the C descriptors from CUDA (HIP) tensors.

Importing this module requires the built library ``libsvf.so`` next to it
(``python -c "import __graft_entry__ as g; g.build()"``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

_LIB_PATH = Path(__file__).resolve().parent / "libsvf.so"

SVF_OK, SVF_EINVAL, SVF_EUNSUPPORTED, SVF_ENOMEM, SVF_EHIP, SVF_EBUSY, SVF_ECANCELLED, SVF_ERANGE = range(8)
SVF_F32, SVF_U16 = 0, 1
SVF_FIELD_COV3, SVF_FIELD_SRT3, SVF_FIELD_SCALES4 = 0, 1, 2
SVF_PRE_F64, SVF_PRE_F32C, SVF_PRE_I64 = 0, 1, 2
SVF_BOUNDARY_ZERO, SVF_BOUNDARY_REPLICATE, SVF_BOUNDARY_SYMMETRIC = 0, 1, 2
SVF_SCALE_SOLVE, SVF_SCALE_LUT = 0, 1

STATUS_NAMES = {0: "SVF_OK", 1: "SVF_EINVAL", 2: "SVF_EUNSUPPORTED", 3: "SVF_ENOMEM", 4: "SVF_EHIP",
                5: "SVF_EBUSY", 6: "SVF_ECANCELLED", 7: "SVF_ERANGE"}



class svf_image(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("channels", C.c_int32), ("H", C.c_int64),
                ("W", C.c_int64), ("row_stride", C.c_int64)]


class svf_field(C.Structure):
    _fields_ = [("data", C.c_void_p), ("kind", C.c_int32), ("reserved", C.c_int32), ("row_stride", C.c_int64)]


class svf_opts(C.Structure):
    _fields_ = [("preint", C.c_int32), ("fd_fp32", C.c_int32), ("eps_px2", C.c_double), ("tile", C.c_int32),
                ("max_reach_px", C.c_int32), ("bands", C.c_int32), ("boundary", C.c_int32),
                ("scale_map", C.c_int32), ("lut_nodes", C.c_int32), ("lut_eps_rel", C.c_double)]


class svf_st_params(C.Structure):
    _fields_ = [("sigma_w", C.c_double), ("order_w", C.c_int32), ("reserved", C.c_int32), ("gain", C.c_double),
                ("lambda_zero", C.c_double), ("a_flat", C.c_double)]


class svf_report(C.Structure):
    _fields_ = [("clamped_px", C.c_int64), ("eps_active_px", C.c_int64), ("invalid_px", C.c_int64),
                ("overflow_px", C.c_int64), ("max_reach_px", C.c_double)]


class svf_server_cfg(C.Structure):
    _fields_ = [("max_inflight", C.c_int32), ("queue_capacity", C.c_int32), ("hbm_budget_bytes", C.c_uint64),
                ("step_mpixels", C.c_int32), ("use_graph", C.c_int32), ("opts", svf_opts)]


class svf_request(C.Structure):
    _fields_ = [("in_", svf_image), ("field", svf_field), ("order", C.c_int32), ("reserved", C.c_int32),
                ("out", svf_image)]


class svf_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("done", C.c_int32), ("t_submit_us", C.c_double), ("t_admit_us", C.c_double),
                ("t_done_us", C.c_double)]


class svf_server_stats_t(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64), ("steps", C.c_int64),
                ("pixels", C.c_int64), ("busy_us", C.c_double), ("cancelled", C.c_int64)]


_lib = None


def lib() -> C.CDLL:
    """Load libsvf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists():
        raise ImportError(f"{_LIB_PATH} is missing: build it first (__graft_entry__.build()); there is no fallback path")
    L = C.CDLL(str(_LIB_PATH))
    vp, st = C.c_void_p, C.c_int
    P = C.POINTER
    L.svf_default_opts.restype = None
    L.svf_default_opts.argtypes = [P(svf_opts)]
    L.svf_create.restype = st
    L.svf_create.argtypes = [P(vp), C.c_int, C.c_size_t]
    L.svf_destroy.restype = st
    L.svf_destroy.argtypes = [vp]
    L.svf_last_error.restype = C.c_char_p
    L.svf_last_error.argtypes = [vp]
    L.svf_workspace_bytes.restype = st
    L.svf_workspace_bytes.argtypes = [P(svf_image), C.c_int, C.c_int, P(svf_opts), P(C.c_size_t)]
    L.svf_scale_map.restype = st
    L.svf_scale_map.argtypes = [vp, P(svf_field), C.c_int64, C.c_int64, C.c_int, P(svf_opts), vp, vp]
    L.svf_preintegrate.restype = st
    L.svf_preintegrate.argtypes = [vp, P(svf_image), C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int, vp, vp]
    L.svf_filter.restype = st
    L.svf_filter_single.restype = st
    L.svf_filter_single.argtypes = [vp, P(svf_image), P(svf_field), C.c_int, P(svf_opts), P(svf_image), vp,
                                    P(svf_report)]
    L.svf_filter.argtypes = [vp, P(svf_image), P(svf_field), C.c_int, C.c_int, P(svf_opts), P(svf_image), vp, P(svf_report)]
    L.svf_filter_batch.restype = st
    L.svf_filter_batch.argtypes = [vp, C.c_int, P(svf_image), P(svf_field), P(C.c_int), P(svf_opts), P(svf_image), vp, C.c_int]
    L.svf_filter_noalloc.restype = st
    L.svf_filter_noalloc.argtypes = [vp, P(svf_image), P(svf_field), C.c_int, C.c_int, P(svf_opts), P(svf_image), vp]
    L.svf_filter_batch_report.restype = st
    L.svf_filter_batch_report.argtypes = [vp, C.c_int, P(svf_report)]
    L.svf_st_default_params.restype = None
    L.svf_st_default_params.argtypes = [P(svf_st_params)]
    L.svf_structure_tensor.restype = st
    L.svf_structure_tensor.argtypes = [vp, P(svf_image), P(svf_st_params), P(svf_opts), vp, C.c_int64, vp, C.c_int64,
                                       vp]
    L.svf_smooth_adaptive.restype = st
    L.svf_smooth_adaptive.argtypes = [vp, P(svf_image), P(svf_st_params), C.c_int, P(svf_opts), P(svf_image), vp,
                                      P(svf_report)]
    L.svf_set_timing.restype = st
    L.svf_set_timing.argtypes = [vp, C.c_int]
    L.svf_kernel_time.restype = st
    L.svf_kernel_time.argtypes = [vp, C.c_char_p, P(C.c_double), P(C.c_int64), C.c_int]
    if hasattr(L, "svf_server_start"):
        L.svf_server_start.restype = st
        L.svf_server_start.argtypes = [vp, P(svf_server_cfg)]
        L.svf_server_submit.restype = st
        L.svf_server_submit.argtypes = [vp, P(svf_request), P(C.c_uint64)]
        L.svf_server_poll.restype = st
        L.svf_server_poll.argtypes = [vp, C.c_uint64, P(svf_result)]
        L.svf_server_wait.restype = st
        L.svf_server_wait.argtypes = [vp, C.c_uint64, P(svf_result), C.c_double]
        L.svf_server_stats.restype = st
        L.svf_server_stats.argtypes = [vp, P(svf_server_stats_t)]
        L.svf_server_cancel.restype = st
        L.svf_server_cancel.argtypes = [vp, C.c_uint64]
        L.svf_server_stop.restype = st
        L.svf_server_stop.argtypes = [vp]
    _lib = L
    return L


class SvfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# ----------------------------------------------------------------------------- descriptors from tensors

def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


def image_of(t) -> svf_image:
    """Descriptor of a device tensor (H, W) or (H, W, C), float32 or uint16, rows contiguous."""
    import torch

    if t.dim() == 2:
        H, W = t.shape
        Cc = 1
        if t.stride(1) != 1:
            raise ValueError("columns must be contiguous")
        rs = t.stride(0)
    elif t.dim() == 3:
        H, W, Cc = t.shape
        if t.stride(2) != 1 or t.stride(1) != Cc:
            raise ValueError("channels must be interleaved and contiguous")
        rs = t.stride(0)
    else:
        raise ValueError("image must be (H, W) or (H, W, C)")
    if t.dtype == torch.float32:
        dt = SVF_F32
    elif t.dtype == torch.uint16:
        dt = SVF_U16
    else:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return svf_image(t.data_ptr(), dt, Cc, H, W, rs)


def field_of(t, kind: int) -> svf_field:
    """Descriptor of a float32 device field (H, W, 3) or (H, W, 4)."""
    import torch

    if t.dtype != torch.float32 or t.dim() != 3 or t.stride(2) != 1 or t.stride(1) != t.shape[2]:
        raise ValueError("field must be a float32 (H, W, K) tensor with contiguous pixels")
    return svf_field(t.data_ptr(), kind, 0, t.stride(0))


def default_opts(**kw) -> svf_opts:
    o = svf_opts()
    lib().svf_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


# ----------------------------------------------------------------------------- the ABI, same names

class Context:
    """Owns an svf_ctx (one device, one workspace)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.ptr = C.c_void_p()
        st = lib().svf_create(C.byref(self.ptr), device, hbm_budget_bytes)
        if st != SVF_OK:
            raise SvfError(st, "svf_create failed")

    def close(self):
        if self.ptr:
            lib().svf_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return lib().svf_last_error(self.ptr).decode()

    def check(self, st: int):
        if st != SVF_OK:
            raise SvfError(st, self.last_error())
        return st


def svf_workspace_bytes(img: svf_image, N: int, order: int, opts: svf_opts | None = None) -> int:
    n = C.c_size_t()
    st = lib().svf_workspace_bytes(C.byref(img), N, order, C.byref(opts) if opts else None, C.byref(n))
    if st != SVF_OK:
        raise SvfError(st, "svf_workspace_bytes")
    return n.value


def svf_scale_map(ctx: Context, field: svf_field, H: int, W: int, order: int, opts: svf_opts | None, scales_out,
                  stream=None):
    return ctx.check(lib().svf_scale_map(ctx.ptr, C.byref(field), H, W, order, C.byref(opts) if opts else None,
                                         scales_out.data_ptr(), _stream_handle(stream)))


def svf_preintegrate(ctx: Context, img: svf_image, channel: int, r0: int, c0: int, h: int, w: int, preint: int, g_out,
                     stream=None):
    return ctx.check(lib().svf_preintegrate(ctx.ptr, C.byref(img), channel, r0, c0, h, w, preint, g_out.data_ptr(),
                                            _stream_handle(stream)))


def svf_filter(ctx: Context, img: svf_image, field: svf_field, N: int, order: int, opts: svf_opts | None,
               out: svf_image, stream=None, report: bool = False):
    rep = svf_report() if report else None
    st = lib().svf_filter(ctx.ptr, C.byref(img), C.byref(field), N, order, C.byref(opts) if opts else None,
                          C.byref(out), _stream_handle(stream), C.byref(rep) if rep is not None else None)
    if report:
        return st, rep
    return ctx.check(st)


def svf_filter_single(ctx: Context, img: svf_image, field: svf_field, m: int, opts: svf_opts | None,
                      out: svf_image, stream=None, report: bool = False):
    rep = svf_report() if report else None
    st = lib().svf_filter_single(ctx.ptr, C.byref(img), C.byref(field), m, C.byref(opts) if opts else None,
                                 C.byref(out), _stream_handle(stream), C.byref(rep) if rep is not None else None)
    if report:
        return st, rep
    return ctx.check(st)


def svf_filter_batch(ctx: Context, imgs, fields, orders, opts: svf_opts | None, outs, stream=None, use_graph=False):
    n = len(imgs)
    IA, FA, OA, RA = svf_image * n, svf_field * n, svf_image * n, C.c_int * n
    return ctx.check(lib().svf_filter_batch(ctx.ptr, n, IA(*imgs), FA(*fields), RA(*orders),
                                            C.byref(opts) if opts else None, OA(*outs), _stream_handle(stream),
                                            1 if use_graph else 0))


def svf_filter_noalloc(ctx: Context, img: svf_image, field: svf_field, N: int, order: int, opts: svf_opts | None,
                       out: svf_image, stream=None):
    return ctx.check(lib().svf_filter_noalloc(ctx.ptr, C.byref(img), C.byref(field), N, order,
                                              C.byref(opts) if opts else None, C.byref(out), _stream_handle(stream)))


def svf_filter_batch_report(ctx: Context, n: int):
    """Reports of the last batch: (status, [svf_report] * n); SVF_EINVAL / SVF_ERANGE are returned, not raised."""
    reps = (svf_report * n)()
    st = lib().svf_filter_batch_report(ctx.ptr, n, reps)
    if st not in (SVF_OK, SVF_EINVAL, SVF_ERANGE):
        ctx.check(st)
    return st, list(reps)


def st_params(**kw) -> svf_st_params:
    """svf_st_default_params, then the given fields."""
    p = svf_st_params()
    lib().svf_st_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def svf_structure_tensor(ctx: Context, img: svf_image, params: svf_st_params, opts: svf_opts | None, tensor_out=None,
                         field_out=None, stream=None):
    """tensor_out / field_out: float32 (H, W, 3) device tensors or None."""
    def ptr_rs(t):
        if t is None:
            return None, 0
        if t.dim() != 3 or t.shape[2] != 3 or t.stride(2) != 1 or t.stride(1) != 3:
            raise ValueError("outputs are (H, W, 3) float32 with contiguous pixels")
        return t.data_ptr(), t.stride(0)

    tp, trs = ptr_rs(tensor_out)
    fp, frs = ptr_rs(field_out)
    return ctx.check(lib().svf_structure_tensor(ctx.ptr, C.byref(img), C.byref(params),
                                                C.byref(opts) if opts else None, tp, trs, fp, frs,
                                                _stream_handle(stream)))


def svf_smooth_adaptive(ctx: Context, img: svf_image, params: svf_st_params, order: int, opts: svf_opts | None,
                        out: svf_image, stream=None, report: bool = False):
    rep = svf_report() if report else None
    st = lib().svf_smooth_adaptive(ctx.ptr, C.byref(img), C.byref(params), order, C.byref(opts) if opts else None,
                                   C.byref(out), _stream_handle(stream), C.byref(rep) if rep is not None else None)
    if report:
        return st, rep
    return ctx.check(st)


def svf_set_timing(ctx: Context, enable: bool):
    return ctx.check(lib().svf_set_timing(ctx.ptr, 1 if enable else 0))


def svf_kernel_time(ctx: Context, kernel: str, reset: bool = False):
    ms, n = C.c_double(), C.c_int64()
    ctx.check(lib().svf_kernel_time(ctx.ptr, kernel.encode(), C.byref(ms), C.byref(n), 1 if reset else 0))
    return ms.value, n.value


# ----------------------------------------------------------------------------- convenience

def filter_tensor(ctx: Context, img, field, kind: int, order: int = 1, out=None, stream=None, report=False, **opts):
    """Filter a device tensor; returns the float32 output tensor (and the report if asked)."""
    import torch

    if out is None:
        out = torch.empty(img.shape, dtype=torch.float32, device=img.device)
    o = default_opts(**opts)
    r = svf_filter(ctx, image_of(img), field_of(field, kind), 4, order, o, image_of(out), stream, report)
    if report:
        st, rep = r
        return out, st, rep
    return out


# ----------------------------------------------------------------------------- serving loop (same names as the ABI)

def svf_server_start(ctx: Context, cfg: svf_server_cfg):
    return ctx.check(lib().svf_server_start(ctx.ptr, C.byref(cfg)))


def svf_server_submit(ctx: Context, req: svf_request) -> int:
    """Queue a request; returns its id (raises SvfError with SVF_EBUSY / SVF_ENOMEM when refused)."""
    rid = C.c_uint64()
    ctx.check(lib().svf_server_submit(ctx.ptr, C.byref(req), C.byref(rid)))
    return rid.value


def svf_server_poll(ctx: Context, rid: int) -> svf_result:
    res = svf_result()
    ctx.check(lib().svf_server_poll(ctx.ptr, C.c_uint64(rid), C.byref(res)))
    return res


def svf_server_wait(ctx: Context, rid: int, timeout_s: float = -1.0) -> svf_result:
    res = svf_result()
    ctx.check(lib().svf_server_wait(ctx.ptr, C.c_uint64(rid), C.byref(res), timeout_s))
    return res


def svf_server_cancel(ctx: Context, rid: int) -> bool:
    """Cancel a request: True if it will end with SVF_ECANCELLED, False if it was
    already completing (done, or its last pass launched); raises for an unknown id."""
    st = lib().svf_server_cancel(ctx.ptr, C.c_uint64(rid))
    if st == SVF_EBUSY:
        return False
    ctx.check(st)
    return True


def svf_server_stats(ctx: Context) -> svf_server_stats_t:
    st = svf_server_stats_t()
    ctx.check(lib().svf_server_stats(ctx.ptr, C.byref(st)))
    return st


def svf_server_stop(ctx: Context):
    return ctx.check(lib().svf_server_stop(ctx.ptr))


def server_request(img, field, kind: int, order: int, out) -> svf_request:
    """Request descriptor from device tensors (views with row strides are fine)."""
    r = svf_request()
    r.in_ = image_of(img)
    r.field = field_of(field, kind)
    r.order = order
    r.out = image_of(out)
    return r
