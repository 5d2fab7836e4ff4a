"""CPU FP64 oracle for the space-variant elliptical box-spline filter.

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product package never imports
it.  The arithmetic lives in ``svf_oracle.c`` (plain C, binary64); this module
marshals numpy arrays, composes passes and gathers boundary extensions; the
structure-tensor step is numpy in binary64.

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
* ``gradient``, ``structure_tensor``, ``st_triple``, ``st_field``,
  ``smooth_adaptive`` -- the feature-preserving smoothing of Sec. 4.2: the
  structure tensor J = w * (g g^T), the triple (s*, rho*, theta*) from its
  eigen-decomposition (numpy.linalg.eigh) by the printed rules, and the filter
  driven by it.
* ``boxspline_m``, ``zp_m``, ``pass_single``, ``filter_single`` -- the iterated box
  spline beta^{4,m}_a (Sec. 2.3, eq. (iterated_spline) / (conv2)) evaluated exactly
  (a B-spline convolution integrated cell by cell) and one single pass with it: the
  direct sum, or m-fold running sums with (m+1)^4 differences and ZP^{*m}
  interpolation (a reading of Sec. 3.3: the paper applies the iterated spline by m
  passes, and this is the single-pass form of the same kernel).
* ``lut_table``, ``scales_lut``, ``filter_lut`` -- the look-up-table scale map
  of Sec. 3.2.2 (unit-size solutions over elongation and one octant, O1/O2).
* ``boundary`` (all) -- what each pass reads outside the image: zero, the
  nearest pixel, or the half-sample mirror; the recursion of Sec. 2.1 needs some
  such condition and the paper does not fix one.  Each pass then is the direct
  sum over the image extended by ``boundary_index``.
"""
from __future__ import annotations

import ctypes as C
import functools
import math
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
        L.svfo_boxspline_m.restype = C.c_double
        L.svfo_boxspline_m.argtypes = [dp, C.c_int, C.c_double, C.c_double]
        L.svfo_zp_m.restype = C.c_double
        L.svfo_zp_m.argtypes = [C.c_int, C.c_double, C.c_double]
        L.svfo_pass_fast_m.restype = C.c_int
        L.svfo_pass_fast_m.argtypes = [vp, C.c_int, C.c_long, C.c_long, C.c_long, C.c_long, dp, C.c_long, C.c_long,
                                       C.c_long, C.c_long, C.c_int, dp]
        L.svfo_pass_brute_m.restype = C.c_int
        L.svfo_pass_brute_m.argtypes = [vp, C.c_int, C.c_long, C.c_long, C.c_long, C.c_long, dp, C.c_long, C.c_long,
                                        C.c_long, C.c_long, C.c_int, dp]
        L.svfo_preint_window_m_f64.restype = None
        L.svfo_preint_window_m_f64.argtypes = [vp, C.c_int, C.c_long, C.c_long, C.c_long, C.c_long, C.c_long,
                                               C.c_long, C.c_long, C.c_long, C.c_int, dp]
        L.svfo_set_threads.restype = C.c_int
        L.svfo_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops (n <= 0: the runtime's default); returns the count in use."""
    return int(lib().svfo_set_threads(int(n)))


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


def boxspline_m(a, m: int, x: float, y: float) -> float:
    """beta^{4,m}_a(x, y): the m-fold self-convolution of beta^4_a (eq. (iterated_spline))."""
    av = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return lib().svfo_boxspline_m(_dp(av), int(m), float(x), float(y))


def zp_m(m: int, x: float, y: float) -> float:
    """The m-fold self-convolution of the ZP element (beta^{4,m}_b, b = (1, sqrt2, 1, sqrt2))."""
    return lib().svfo_zp_m(int(m), float(x), float(y))


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


def preint_window_m_f64(img: np.ndarray, r0: int, c0: int, h: int, w: int, m: int) -> np.ndarray:
    """RS1..RS4 applied m times (sqrt2 factors each time) to img on a window."""
    img = np.ascontiguousarray(img)
    H, W = img.shape
    g = np.empty((h, w), dtype=np.float64)
    lib().svfo_preint_window_m_f64(img.ctypes.data, _img_code(img), 0, 0, H, W, r0, c0, h, w, int(m), _dp(g))
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


# ----------------------------------------------------------------------------- structure tensor (Sec. 4.2)
#
# The application of Sec. 4.2 estimates the filter at every pixel from the
# image itself: the structure tensor J = w * (g g^T) with g the gradient and w
# an isotropic averaging window; theta* is the direction of the eigenvector of
# the smallest eigenvalue of J (the direction of least intensity variation, along
# which the filter is elongated); rho* and s* follow the printed rules on the two
# eigenvalues.  Readings (the paper refers elsewhere for the details):
# * g: central differences, g1 along x (columns), g2 along y (rows), the image
#   extended by the boundary rule; several channels add their g g^T;
# * w: the isotropic four-directional box spline of covariance sigma_w^2 I
#   (all scales sigma_w sqrt 6, Thm. 2.2), iterated order_w times (Sec. 3.3),
#   applied by this oracle's own filter with the same boundary rule;
# * gain: the rules act on gain * J (gain 1: the eigenvalues in the image's units,
#   as printed); an eigenvalue <= lambda_zero counts as zero;
# * both eigenvalues zero: the isotropic box spline with all scales a_flat.


def gradient(img: np.ndarray, boundary: int = BOUNDARY_ZERO):
    """Central differences (g1 along columns, g2 along rows) in binary64, per channel."""
    f = np.asarray(img, dtype=np.float64)
    if f.ndim == 2:
        f = f[..., None]
    H, W = f.shape[:2]
    if boundary == BOUNDARY_ZERO:
        e = np.zeros((H + 2, W + 2, f.shape[2]))
        e[1:-1, 1:-1] = f
    else:
        ri = boundary_index(np.arange(-1, H + 1), H, boundary)
        ci = boundary_index(np.arange(-1, W + 1), W, boundary)
        e = f[np.ix_(ri, ci)]
    g1 = 0.5 * (e[1:-1, 2:] - e[1:-1, :-2])
    g2 = 0.5 * (e[2:, 1:-1] - e[:-2, 1:-1])
    return g1, g2


def structure_tensor(img: np.ndarray, sigma_w: float, order_w: int = 1, boundary: int = BOUNDARY_ZERO,
                     method: str = "fast", tile: int = 32) -> np.ndarray:
    """J = w * (sum over channels of g g^T), (H, W, 3) = (J11, J12, J22), binary64."""
    g1, g2 = gradient(img, boundary)
    P = np.stack([(g1 * g1).sum(-1), (g1 * g2).sum(-1), (g2 * g2).sum(-1)], -1)
    H, W = P.shape[:2]
    a = np.broadcast_to(np.full(4, sigma_w * np.sqrt(6.0)) / np.sqrt(order_w), (H, W, 4))
    return np.stack([filter_scales(P[..., k], np.ascontiguousarray(a), order_w, method, tile, boundary)
                     for k in range(3)], -1)


def st_triple(J: np.ndarray, gain: float = 1.0, lambda_zero: float = 0.0, a_flat: float = 1.0):
    """(s*, rho*, theta*) per pixel from J (..., 3) by the rules of Sec. 4.2.

    Eigen-decomposition by numpy.linalg.eigh; theta* in [0, pi).  Returns three
    arrays (s, rho, theta); flat pixels get s = a_flat^2 / 3 (the size of the
    box spline with all scales a_flat: covariance a_flat^2 / 6 I), rho = 1, theta = 0.
    """
    J = gain * np.asarray(J, dtype=np.float64)
    M = np.stack([np.stack([J[..., 0], J[..., 1]], -1), np.stack([J[..., 1], J[..., 2]], -1)], -2)
    lam, vec = np.linalg.eigh(M)            # ascending eigenvalues, eigenvectors in columns
    lmin, lmax = lam[..., 0], lam[..., 1]
    zmin, zmax = lmin <= lambda_zero, lmax <= lambda_zero
    vmin = vec[..., :, 0]
    theta = np.mod(np.arctan2(vmin[..., 1], vmin[..., 0]), np.pi)
    lmin_eff = np.where(zmin, 0.0, lmin)
    lmax_eff = np.where(zmax, 0.0, lmax)
    with np.errstate(divide="ignore", invalid="ignore"):
        rho = np.where(~zmin & ~zmax, lmax_eff / np.where(zmin, 1.0, lmin_eff), 1.0)
    one = zmin & ~zmax                      # only the larger eigenvalue is non-zero
    rho = np.where(one, np.maximum(1.0, lmax_eff), rho)
    s = lmax_eff + lmin_eff
    flat = zmin & zmax
    s = np.where(flat, a_flat * a_flat / 3.0, s)
    rho = np.where(flat, 1.0, rho)
    theta = np.where(flat, 0.0, theta)
    return s, rho, theta


def st_field(img: np.ndarray, sigma_w: float, order_w: int = 1, gain: float = 1.0, lambda_zero: float = 0.0,
             a_flat: float = 1.0, boundary: int = BOUNDARY_ZERO) -> np.ndarray:
    """The (sigma, rho, theta) field (H, W, 3) float32 that drives the filter: sigma = sqrt(s / 2)."""
    J = structure_tensor(img, sigma_w, order_w, boundary)
    s, rho, theta = st_triple(J, gain, lambda_zero, a_flat)
    return np.stack([np.sqrt(s / 2.0), rho, theta], -1).astype(np.float32)


def smooth_adaptive(img: np.ndarray, sigma_w: float, order_w: int, gain: float, lambda_zero: float, a_flat: float,
                    order: int, boundary: int = BOUNDARY_ZERO, eps: float = DEFAULT_EPS):
    """Feature-preserving smoothing of Sec. 4.2: the structure-tensor field, then the order-m filter."""
    fld = st_field(img, sigma_w, order_w, gain, lambda_zero, a_flat, boundary)
    return filter(img, fld, FIELD_SRT3, order, eps, boundary=boundary)


# ----------------------------------------------------------------------------- scale look-up table (Sec. 3.2.2)
#
# The paper's alternative to a solve per pixel: tabulate the solution for unit
# size, s = 1, over elongation and the orientations of one octant, then per pixel
# (O1) reduce theta to phi in [0, pi/4) and its octant k, (O2) look up and
# permute by k and scale by sqrt(s).  Readings: the table is over
# u = 1 / rho in [0, 1] (u = 0: unbounded elongation, which the solve clamps)
# and phi, nodes equally spaced, values float32, bilinear interpolation; the
# permutation for octant k is the rotation of the scale vector by k places,
# (a1, a2, a3, a4) -> (a4, a1, a2, a3) per quarter of a right angle (the printed
# rows for the second and fourth octants are exchanged); the floor on a^2 is
# relative, eps_rel * s, since the unit-size solution is scaled by sqrt(s).

LUT_DEFAULT_NODES = 129
LUT_DEFAULT_EPS_REL = 0.125


def lut_table(nodes: int = LUT_DEFAULT_NODES, eps_rel: float = LUT_DEFAULT_EPS_REL) -> np.ndarray:
    """(nodes, nodes, 4) float32: entry [i, j] solves s = 1, rho = (nodes-1)/i, phi = j pi / (4 (nodes-1))."""
    return _lut_table(int(nodes), float(eps_rel)).copy()


@functools.lru_cache(maxsize=8)
def _lut_table(nodes: int, eps_rel: float) -> np.ndarray:
    T = np.empty((nodes, nodes, 4), dtype=np.float32)
    sig1 = math.sqrt(0.5)   # s = 2 sigma^2 = 1
    for i in range(nodes):
        rho = (nodes - 1) / i if i > 0 else 1e300
        for j in range(nodes):
            a, _, _ = scales_from_srt(sig1, rho, j * (math.pi / 4) / (nodes - 1), eps_rel)
            T[i, j] = a
    return T


def srt_of_field(field: np.ndarray, kind: int):
    """(s, rho, theta, valid) per pixel from an SRT3 or COV3 field (float64)."""
    f = np.asarray(field, dtype=np.float64)
    if kind == FIELD_SRT3:
        sig, rho, th = f[..., 0], f[..., 1], f[..., 2]
        valid = np.isfinite(f).all(-1) & (sig > 0) & (rho >= 1)
        return 2 * sig * sig, rho, th, valid
    c11, c12, c22 = f[..., 0], f[..., 1], f[..., 2]
    det = c11 * c22 - c12 * c12
    valid = np.isfinite(f).all(-1) & (c11 > 0) & (c22 > 0) & (det > 0)
    s = c11 + c22
    dd = np.sqrt((c11 - c22) ** 2 + 4 * c12 * c12)
    lmax, lmin = 0.5 * (s + dd), 0.5 * (s - dd)
    with np.errstate(divide="ignore", invalid="ignore"):
        rho = np.where(valid, lmax / np.where(lmin > 0, lmin, 1.0), 1.0)
    return s, rho, 0.5 * np.arctan2(2 * c12, c11 - c22), valid


def scales_lut(field: np.ndarray, kind: int, order: int = 1, nodes: int = LUT_DEFAULT_NODES,
               eps_rel: float = LUT_DEFAULT_EPS_REL, table: np.ndarray | None = None) -> np.ndarray:
    """Per-pass scales (H, W, 4) float64 by the look-up table (O1, O2); NaN where the field is invalid."""
    T = lut_table(nodes, eps_rel).astype(np.float64) if table is None else np.asarray(table, np.float64)
    n = T.shape[0]
    s, rho, th, valid = srt_of_field(field, kind)
    rho = np.where(valid, rho, 1.0)
    s = np.where(valid, s, 1.0)
    th = np.mod(np.where(valid, th, 0.0), math.pi)
    k = np.clip(np.floor(th / (math.pi / 4)), 0, 3).astype(np.int64)
    phi = th - k * (math.pi / 4)
    fu = (1.0 / rho) * (n - 1)
    fp = phi / (math.pi / 4) * (n - 1)
    i0 = np.clip(np.floor(fu), 0, n - 2).astype(np.int64)
    j0 = np.clip(np.floor(fp), 0, n - 2).astype(np.int64)
    wu, wp = (fu - i0)[..., None], (fp - j0)[..., None]
    a1 = ((1 - wu) * (1 - wp) * T[i0, j0] + (1 - wu) * wp * T[i0, j0 + 1]
          + wu * (1 - wp) * T[i0 + 1, j0] + wu * wp * T[i0 + 1, j0 + 1])
    out = np.empty_like(a1)
    for q in range(4):   # octant q: the tabulated vector rotated by q places
        m = k == q
        out[m] = np.roll(a1[m], q, axis=-1)
    out *= np.sqrt(s)[..., None]
    out[~valid] = np.nan
    return out / math.sqrt(order)


def filter_lut(img: np.ndarray, field: np.ndarray, kind: int, order: int = 1, nodes: int = LUT_DEFAULT_NODES,
               eps_rel: float = LUT_DEFAULT_EPS_REL, method: str = "fast", tile: int = 32,
               boundary: int = BOUNDARY_ZERO):
    """The filter with the look-up-table scale map."""
    a = scales_lut(field, kind, order, nodes, eps_rel)
    if img.ndim == 3:
        return np.stack([filter_scales(img[..., ch], a, order, method, tile, boundary) for ch in range(img.shape[2])],
                        -1)
    return filter_scales(img, a, order, method, tile, boundary)


# ----------------------------------------------------------------------------- single pass with beta^{4,m}

def pass_single(img: np.ndarray, a_rect: np.ndarray, m: int, method: str = "brute", r0: int = 0, c0: int = 0):
    """One pass with the iterated box spline beta^{4,m}_{a(n)} over the output rectangle
    (r0, c0) + a_rect.shape[:2] of img (zero outside): 'brute' is the direct sum
    sum_k f[k] beta^{4,m}_{a(n)}(n - k), 'fast' the m-fold running sums with the
    (m+1)^4-tap difference and ZP^{*m} interpolation on per-pixel windows."""
    img = np.ascontiguousarray(img)
    if img.dtype not in (np.float64, np.float32, np.uint16):
        img = img.astype(np.float64)
    fh, fw = img.shape
    h, w = a_rect.shape[:2]
    a_rect = np.ascontiguousarray(a_rect, dtype=np.float64)
    out = np.empty((h, w), dtype=np.float64)
    if h == 0 or w == 0:
        return out
    fn = {"brute": lib().svfo_pass_brute_m, "fast": lib().svfo_pass_fast_m}[method]
    rc = fn(img.ctypes.data, _img_code(img), 0, 0, fh, fw, _dp(a_rect), r0, c0, h, w, int(m), _dp(out))
    if rc != 0:
        raise RuntimeError("oracle single pass failed")
    return out


def filter_single(img: np.ndarray, field: np.ndarray, kind: int, m: int, eps: float = DEFAULT_EPS,
                  method: str = "brute"):
    """Single-pass filter with beta^{4,m}_{a(n) / sqrt(m)} (the iterated spline of Sec. 3.3 with
    the covariance of beta^4_{a(n)}: the scale solve of Sec. 3.2.2, then a / sqrt(m)), zero
    outside the image; (H, W) or (H, W, C) images; returns float64."""
    a, _ = scales(field, kind, m, eps)
    if img.ndim == 3:
        return np.stack([pass_single(img[..., ch], a, m, method) for ch in range(img.shape[2])], -1)
    return pass_single(img, a, m, method)

