"""CPU FP64 oracle for the space-variant elliptical box-spline filter.

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product package never imports
it.  The arithmetic lives in ``svf_oracle.c`` (plain C, binary64); this module
only marshals numpy arrays, composes passes and gathers boundary extensions.

What it computes (Chaudhury, Munoz-Barrutia, Unser, "Fast space-variant
elliptical filtering using box splines"):

* ``boxspline(a, x, y)``, ``zp(x, y)`` -- the four-directional box spline of
  Sec. 3 (eq. (const) with N = 4) and its special case the ZP element.
* ``scales(field, kind, order, eps)`` -- the scale-vector solve of Sec. 3.2.2
  for every pixel, divided by sqrt(order) for the iterated filter of Sec. 3.3.
* ``preint_window_f64`` / ``preint_window_i64`` -- the running sums RS1..RS4
  (Algorithm 1, step 2) on a window.
* ``filter(...)`` -- order-m space-variant filtering, either with the fast
  algorithm (Algorithm 1: pre-integration, eq. (final_eqn) with Table 1 taps and
  ZP interpolation) or with the direct sum  sum_k f[k] beta^4_{a(n)}(n - k).
* ``filter_region(...)`` -- the same on a sub-rectangle of a large image (for
  sampled parity checks), pulling in only the region every pass depends on.
* ``boundary`` (both) -- what each pass reads outside the image: zero, the
  nearest pixel, or the half-sample mirror; the recursion of Sec. 2.1 needs some
  such condition and the paper does not fix one.  Each pass then is the direct
  sum over the image extended by ``boundary_index``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "svf_oracle.c"
_LIB = _HERE / "libsvf_oracle.so"

FIELD_COV3, FIELD_SRT3, FIELD_SCALES4 = 0, 1, 2
DEFAULT_EPS = 0.25  # floor on a_k^2 per pass (px^2): a_k >= 0.5 px


def build(force: bool = False) -> Path:
    """Compile the oracle with gcc (binary64, no FMA contraction, OpenMP)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = str(_LIB) + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", str(_SRC), "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(str(_LIB))
        dp, fp, vp, lp, ip = C.POINTER(C.c_double), C.POINTER(C.c_float), C.c_void_p, C.POINTER(C.c_long), C.POINTER(C.c_int)
        L.svfo_boxspline.restype = C.c_double
        L.svfo_boxspline.argtypes = [dp, C.c_double, C.c_double]
        L.svfo_zp.restype = C.c_double
        L.svfo_zp.argtypes = [C.c_double, C.c_double]
        L.svfo_boxspline_grid.restype = None
        L.svfo_boxspline_grid.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_long, C.c_long, dp]
        L.svfo_rho_max.restype = C.c_double
        L.svfo_rho_max.argtypes = [C.c_double, C.c_double, C.c_double]
        L.svfo_scales_from_srt.restype = C.c_int
        L.svfo_scales_from_srt.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp, ip, ip]
        L.svfo_scales_from_cov.restype = C.c_int
        L.svfo_scales_from_cov.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp, ip, ip]
        L.svfo_scale_field.restype = C.c_int
        L.svfo_scale_field.argtypes = [fp, C.c_int, C.c_long, C.c_long, C.c_int, C.c_double, dp, lp, lp, lp]
        L.svfo_preint_window_f64.restype = None
        L.svfo_preint_window_f64.argtypes = [vp, C.c_int, C.c_long, C.c_long, C.c_long, C.c_long, C.c_long,
                                             C.c_long, C.c_long, C.c_long, dp]
        L.svfo_preint_window_i64.restype = None
        L.svfo_preint_window_i64.argtypes = [vp, C.c_long, C.c_long, C.c_long, C.c_long, C.c_long, C.c_long, vp]
        L.svfo_fd_pixel.restype = C.c_double
        L.svfo_fd_pixel.argtypes = [dp, C.c_long, C.c_long, C.c_long, C.c_long, C.c_double, C.c_long, C.c_long, dp]
        L.svfo_pass_fast.restype = C.c_int
        L.svfo_pass_fast.argtypes = [vp, C.c_int, C.c_long, C.c_long, C.c_long, C.c_long, dp, C.c_long, C.c_long,
                                     C.c_long, C.c_long, C.c_long, dp]
        L.svfo_pass_brute.restype = C.c_int
        L.svfo_pass_brute.argtypes = [vp, C.c_int, C.c_long, C.c_long, C.c_long, C.c_long, dp, C.c_long, C.c_long,
                                      C.c_long, C.c_long, dp]
        L.svfo_table1_tap.restype = None
        L.svfo_table1_tap.argtypes = [dp, C.c_int, dp, dp, dp]
        L.svfo_tau.restype = None
        L.svfo_tau.argtypes = [dp, dp, dp]
        _lib = L
    return _lib


def _dp(x: np.ndarray):
    return x.ctypes.data_as(C.POINTER(C.c_double))


def _img_code(x: np.ndarray) -> int:
    if x.dtype == np.float64:
        return 0
    if x.dtype == np.float32:
        return 1
    if x.dtype == np.uint16:
        return 2
    raise TypeError(f"unsupported image dtype {x.dtype}")


# ----------------------------------------------------------------------------- point evaluations

def boxspline(a, x: float, y: float) -> float:
    """beta^4_a(x, y) (Sec. 2.2.1 eq. (const), N = 4), a = (a1, a2, a3, a4)."""
    av = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return lib().svfo_boxspline(_dp(av), float(x), float(y))


def zp(x: float, y: float) -> float:
    """ZP element beta^4_b, b = (1, sqrt2, 1, sqrt2) (Sec. 3.1)."""
    return lib().svfo_zp(float(x), float(y))


def boxspline_grid(a, x0: float, y0: float, h: float, nx: int, ny: int, hy: float | None = None) -> np.ndarray:
    """beta^4_a sampled at (x0 + i h, y0 + j hy); returns (ny, nx)."""
    av = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    out = np.empty((ny, nx), dtype=np.float64)
    lib().svfo_boxspline_grid(_dp(av), x0, y0, h, h if hy is None else hy, nx, ny, _dp(out))
    return out


def table1_tap(a, i: int):
    """Tap i of Table 1: (x_i as a 2-vector, sign of w_i)."""
    av = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    x1, x2, sg = C.c_double(), C.c_double(), C.c_double()
    lib().svfo_table1_tap(_dp(av), i, C.byref(x1), C.byref(x2), C.byref(sg))
    return np.array([x1.value, x2.value]), sg.value


def tau(a):
    """Shift tau of Sec. 3.1 step (2)."""
    av = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    t1, t2 = C.c_double(), C.c_double()
    lib().svfo_tau(_dp(av), C.byref(t1), C.byref(t2))
    return np.array([t1.value, t2.value])


def support_halfwidths(a):
    a = np.asarray(a, dtype=np.float64)
    s = (a[..., 1] + a[..., 3]) / np.sqrt(2.0)
    return 0.5 * (a[..., 0] + s), 0.5 * (a[..., 2] + s)


# ----------------------------------------------------------------------------- scale solve

def rho_max(s: float, theta: float, eps: float) -> float:
    """Largest feasible elongation at size s, orientation theta, floor eps on a^2."""
    return lib().svfo_rho_max(s, theta, eps)


def scales_from_srt(sigma, rho, theta, eps=DEFAULT_EPS):
    """Full-filter scales for one (sigma, rho, theta); returns (a[4], clamped, eps_active)."""
    a = np.zeros(4)
    cl, ea = C.c_int(0), C.c_int(0)
    rc = lib().svfo_scales_from_srt(sigma, rho, theta, eps, _dp(a), C.byref(cl), C.byref(ea))
    if rc != 0:
        raise ValueError(f"scale solve failed (rc={rc}) for {(sigma, rho, theta)}")
    return a, bool(cl.value), bool(ea.value)


def scales_from_cov(c11, c12, c22, eps=DEFAULT_EPS):
    a = np.zeros(4)
    cl, ea = C.c_int(0), C.c_int(0)
    rc = lib().svfo_scales_from_cov(c11, c12, c22, eps, _dp(a), C.byref(cl), C.byref(ea))
    if rc != 0:
        raise ValueError(f"scale solve failed (rc={rc}) for {(c11, c12, c22)}")
    return a, bool(cl.value), bool(ea.value)


def scales(field: np.ndarray, kind: int, order: int = 1, eps: float = DEFAULT_EPS):
    """Per-pass scales (H, W, 4) f64 for a field (H, W, 3|4) float32.

    eps is the per-pass floor on a_k^2; the full-filter solve uses order*eps and
    each pass uses a / sqrt(order) (Sec. 3.3).  Returns (a, stats dict).
    """
    field = np.ascontiguousarray(field, dtype=np.float32)
    H, W = field.shape[:2]
    out = np.empty((H, W, 4), dtype=np.float64)
    ncl, nep, ninv = C.c_long(0), C.c_long(0), C.c_long(0)
    lib().svfo_scale_field(field.ctypes.data_as(C.POINTER(C.c_float)), kind, H, W, order, eps, _dp(out),
                           C.byref(ncl), C.byref(nep), C.byref(ninv))
    return out, {"clamped": ncl.value, "eps_active": nep.value, "invalid": ninv.value}


# ----------------------------------------------------------------------------- running sums

def preint_window_f64(img: np.ndarray, r0: int, c0: int, h: int, w: int) -> np.ndarray:
    """RS1..RS4 of img restricted to rows [r0, r0+h) x cols [c0, c0+w) (zero outside the image)."""
    img = np.ascontiguousarray(img)
    H, W = img.shape
    g = np.empty((h, w), dtype=np.float64)
    lib().svfo_preint_window_f64(img.ctypes.data, _img_code(img), 0, 0, H, W, r0, c0, h, w, _dp(g))
    return g


def preint_window_i64(img: np.ndarray, r0: int, c0: int, h: int, w: int) -> np.ndarray:
    """Integer running sums (no sqrt2 factors) of a uint16 image on a window; int64 (wrapping)."""
    img = np.ascontiguousarray(img, dtype=np.uint16)
    H, W = img.shape
    g = np.empty((h, w), dtype=np.int64)
    lib().svfo_preint_window_i64(img.ctypes.data, H, W, r0, c0, h, w, g.ctypes.data)
    return g


def fd_pixel(g: np.ndarray, wr0: int, wc0: int, n1: int, n2: int, a, gscale: float = 1.0) -> float:
    """eq. (final_eqn) at one pixel from a pre-integrated window g whose [0,0] is lattice (wr0, wc0)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    av = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return lib().svfo_fd_pixel(_dp(g), g.shape[0], g.shape[1], wr0, wc0, gscale, n1, n2, _dp(av))


# ----------------------------------------------------------------------------- passes and filters

def _pass(img, fr0, fc0, a_rect, r0, c0, method, tile):
    img = np.ascontiguousarray(img)
    if img.dtype not in (np.float64, np.float32, np.uint16):
        img = img.astype(np.float64)
    fh, fw = img.shape
    h, w = a_rect.shape[:2]
    a_rect = np.ascontiguousarray(a_rect, dtype=np.float64)
    out = np.empty((h, w), dtype=np.float64)
    if h == 0 or w == 0:
        return out
    if method == "fast":
        rc = lib().svfo_pass_fast(img.ctypes.data, _img_code(img), fr0, fc0, fh, fw, _dp(a_rect), r0, c0, h, w,
                                  tile, _dp(out))
    elif method == "brute":
        rc = lib().svfo_pass_brute(img.ctypes.data, _img_code(img), fr0, fc0, fh, fw, _dp(a_rect), r0, c0, h, w,
                                   _dp(out))
    else:
        raise ValueError(method)
    if rc != 0:
        raise RuntimeError("oracle pass failed")
    return out


# Values of the image outside its border (the paper leaves the boundary conditions
# of the running sums open, Sec. 2.1): zero, replicate the nearest pixel, or the
# half-sample symmetric mirror (f[-1] = f[0], f[-2] = f[1], ...; period 2N).
BOUNDARY_ZERO, BOUNDARY_REPLICATE, BOUNDARY_SYMMETRIC = 0, 1, 2


def boundary_index(i, N: int, boundary: int):
    """Image index whose value the (possibly outside) index i takes under the rule."""
    i = np.asarray(i, dtype=np.int64)
    if boundary == BOUNDARY_REPLICATE:
        return np.clip(i, 0, N - 1)
    if boundary == BOUNDARY_SYMMETRIC:
        m = np.mod(i, 2 * N)
        return np.where(m >= N, 2 * N - 1 - m, m)
    raise ValueError(boundary)


def _margins(a):
    """Rows / columns beyond an output rectangle that its pixels may read (support + ZP reach)."""
    rx, ry = support_halfwidths(a)
    return int(np.ceil(float(ry.max()))) + 3, int(np.ceil(float(rx.max()))) + 3


def _pass_rule(src, sr0, sc0, H, W, a_rect, r0, c0, method, tile, boundary):
    """One pass on the output rectangle (r0, c0) + a_rect.shape[:2] of an H x W image.

    src holds the pass input on image rows sr0.. and columns sc0.. .  Zero rule:
    nothing outside the image.  Other rules: the input on the rectangle grown by
    every read's reach is gathered through boundary_index (so an output reads the
    direct sum over the extended lattice), and the pass runs on that extension.
    """
    if boundary == BOUNDARY_ZERO:
        return _pass(src, sr0, sc0, a_rect, r0, c0, method, tile)
    h, w = a_rect.shape[:2]
    gy, gx = _margins(a_rect)
    ri = boundary_index(np.arange(r0 - gy, r0 + h + gy), H, boundary) - sr0
    ci = boundary_index(np.arange(c0 - gx, c0 + w + gx), W, boundary) - sc0
    if ri.min() < 0 or ri.max() >= src.shape[0] or ci.min() < 0 or ci.max() >= src.shape[1]:
        raise RuntimeError("pass input does not cover the reflected reads")
    return _pass(np.asarray(src)[np.ix_(ri, ci)], r0 - gy, c0 - gx, a_rect, r0, c0, method, tile)


def filter_scales(img: np.ndarray, a_pass: np.ndarray, order: int = 1, method: str = "fast", tile: int = 32,
                  boundary: int = BOUNDARY_ZERO):
    """Order-m filter of a whole single-channel image given per-pass scales (H, W, 4).

    Pass p reads the (binary64) output of pass p-1, extended beyond the image by the
    boundary rule (zero by default) (Sec. 3.3).
    """
    H, W = img.shape
    cur = img
    for _ in range(order):
        cur = _pass_rule(cur, 0, 0, H, W, a_pass, 0, 0, method, tile, boundary)
    return cur


def filter(img: np.ndarray, field: np.ndarray, kind: int, order: int = 1, eps: float = DEFAULT_EPS,
           method: str = "fast", tile: int = 32, boundary: int = BOUNDARY_ZERO):
    """Order-m filter of an image (H, W) or (H, W, C) with a field (H, W, 3|4); returns float64."""
    a, _ = scales(field, kind, order, eps)
    if img.ndim == 3:
        return np.stack([filter_scales(img[..., ch], a, order, method, tile, boundary) for ch in range(img.shape[2])],
                        -1)
    return filter_scales(img, a, order, method, tile, boundary)


def _grow(rect, gy, gx, H, W):
    r0, c0, h, w = rect
    R0, C0 = max(0, r0 - gy), max(0, c0 - gx)
    R1, C1 = min(H, r0 + h + gy), min(W, c0 + w + gx)
    return (R0, C0, R1 - R0, C1 - C0)


def filter_region(img: np.ndarray, field: np.ndarray, kind: int, order: int, rect, eps: float = DEFAULT_EPS,
                  method: str = "fast", tile: int = 32, boundary: int = BOUNDARY_ZERO) -> np.ndarray:
    """Order-m output on rect = (r0, c0, h, w) of a large single-channel image.

    Pass m needs pass m-1 on rect grown by pass m's reach, clipped to the image;
    the chain of regions is built backwards from the per-pass scales, computed
    only where needed.  Values outside the image follow the boundary rule; a
    grown region that crosses a border reaches it, so the reflected or
    replicated reads stay inside the region below.
    """
    H, W = img.shape
    regions = [tuple(rect)]
    a_cache = {}

    def a_for(rr):
        key = tuple(rr)
        if key not in a_cache:
            r0, c0, h, w = rr
            a_cache[key], _ = scales(field[r0:r0 + h, c0:c0 + w], kind, order, eps)
        return a_cache[key]

    for _ in range(order - 1):
        cur = regions[-1]
        gy, gx = _margins(a_for(cur))
        regions.append(_grow(cur, gy, gx, H, W))
    regions = regions[::-1]   # regions[0] is pass 1's output region
    cur_img, fr0, fc0 = img, 0, 0
    for rr in regions:
        r0, c0, h, w = rr
        out = _pass_rule(cur_img, fr0, fc0, H, W, a_for(rr), r0, c0, method, tile, boundary)
        cur_img, fr0, fc0 = out, r0, c0
    return cur_img
