"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and shapes them into images and smooth
parameter fields.  It contains none of the filter's arithmetic (no covariance
to scale mapping, no running sums, no finite differences), so it can feed both
the GPU path and the CPU oracle without coupling them.

Workloads follow the paper's experiments (Sec. 4.1, Table 2: a 512x512 image
filtered with kernels of several sizes) and the build's parity/bench configs:

* images: FP32 uniform [0, 1) or uint16 uniform {0..65535};
* noisy oriented images (the feature-preserving smoothing of Sec. 4.2:
  stripes whose orientation and period vary smoothly, plus Gaussian noise,
  optionally with a noise-free flat rectangle);
* fields: per-pixel (sigma, rho, theta) with sigma = isotropic standard
  deviation in pixels, rho = elongation (variance ratio lambda_max/lambda_min,
  Sec. 3.2.1 descriptor D1), theta = orientation of the major axis in [0, pi),
  measured from +x (column axis) toward +y (row axis).  Each parameter is a
  Gaussian-smoothed white-noise field mapped to [0, 1) by its empirical CDF.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "seed_for",
    "uniform_image",
    "smooth_uniform_field",
    "srt_field",
    "scales_field",
    "constant_srt_field",
    "oriented_image",
]


def seed_for(config: int, item: int = 0) -> int:
    """Seed convention: configuration k, item i -> 1000*k + i."""
    return 1000 * int(config) + int(item)


def uniform_image(h: int, w: int, seed: int, dtype: str = "f32", channels: int = 1) -> np.ndarray:
    """H x W (x C) image, FP32 uniform [0,1) or uint16 uniform {0..65535}.

    Returned as a C-contiguous array of shape (H, W) when channels == 1,
    else (H, W, C) (channel-interleaved).
    """
    rng = np.random.default_rng(seed)
    shape = (h, w) if channels == 1 else (h, w, channels)
    if dtype == "f32":
        return rng.random(shape, dtype=np.float32)
    if dtype == "u16":
        return rng.integers(0, 65536, size=shape, dtype=np.uint16)
    raise ValueError(f"unknown dtype {dtype!r}")


def _gauss_smooth_periodic(x: np.ndarray, std: float) -> np.ndarray:
    """Periodic Gaussian smoothing via FFT (input generation only)."""
    h, w = x.shape
    ky = np.fft.fftfreq(h)[:, None]
    kx = np.fft.rfftfreq(w)[None, :]
    tf = np.exp(-2.0 * (np.pi * std) ** 2 * (ky * ky + kx * kx))
    return np.fft.irfft2(np.fft.rfft2(x) * tf, s=(h, w))


def smooth_uniform_field(h: int, w: int, rng: np.random.Generator, corr_len: float) -> np.ndarray:
    """Smooth field with values in [0, 1): smoothed noise ranked by its empirical CDF."""
    z = _gauss_smooth_periodic(rng.standard_normal((h, w)), corr_len)
    order = np.argsort(z, axis=None, kind="stable")
    u = np.empty(h * w, dtype=np.float64)
    u[order] = (np.arange(h * w, dtype=np.float64) + 0.5) / (h * w)
    return u.reshape(h, w)


def srt_field(
    h: int,
    w: int,
    seed: int,
    sigma_range=(1.0, 4.0),
    rho_range=(1.0, 3.0),
    corr_len: float | None = None,
) -> np.ndarray:
    """Smooth (sigma, rho, theta) field, shape (H, W, 3), float32.

    sigma = smin + u1 (smax - smin); rho = rmin + u2 (rmax - rmin);
    theta = atan2(n2, n1)/2 mod pi from two smoothed zero-mean noises, which is
    smooth and pi-periodic.  Default correlation length scales with the image
    (16 px at 64, 64 px at 1024, 256 px at 4096).
    """
    if corr_len is None:
        corr_len = max(4.0, 16.0 * (max(h, w) / 64.0) ** 0.5) if max(h, w) <= 1024 else max(h, w) / 16.0
    rng = np.random.default_rng(seed + 7_777_777)
    u1 = smooth_uniform_field(h, w, rng, corr_len)
    u2 = smooth_uniform_field(h, w, rng, corr_len)
    n1 = _gauss_smooth_periodic(rng.standard_normal((h, w)), corr_len)
    n2 = _gauss_smooth_periodic(rng.standard_normal((h, w)), corr_len)
    sigma = sigma_range[0] + u1 * (sigma_range[1] - sigma_range[0])
    rho = rho_range[0] + u2 * (rho_range[1] - rho_range[0])
    theta = np.mod(0.5 * np.arctan2(n2, n1), np.pi)
    return np.ascontiguousarray(np.stack([sigma, rho, theta], axis=-1).astype(np.float32))


def constant_srt_field(h: int, w: int, sigma: float, rho: float = 1.0, theta: float = 0.0) -> np.ndarray:
    """Spatially constant (sigma, rho, theta) field, shape (H, W, 3), float32."""
    f = np.empty((h, w, 3), dtype=np.float32)
    f[..., 0] = sigma
    f[..., 1] = rho
    f[..., 2] = theta
    return f


def scales_field(h: int, w: int, seed: int, lo: float = 0.6, hi: float = 3.0, smooth: bool = False) -> np.ndarray:
    """Per-pixel box scales (a1, a2, a3, a4), shape (H, W, 4), float32.

    Independent uniform draws in [lo, hi) per pixel and direction (white, the
    hardest case for tiling), or smoothly varying when smooth=True.
    """
    rng = np.random.default_rng(seed + 5_555_555)
    if smooth:
        u = np.stack([smooth_uniform_field(h, w, rng, max(2.0, min(h, w) / 8.0)) for _ in range(4)], axis=-1)
    else:
        u = rng.random((h, w, 4))
    return np.ascontiguousarray((lo + u * (hi - lo)).astype(np.float32))


def oriented_image(h: int, w: int, seed: int, period=(6.0, 14.0), amplitude: float = 0.4, noise: float = 0.1,
                   corr_len: float | None = None, flat_box=None, dtype: str = "f32", channels: int = 1) -> np.ndarray:
    """Noisy stripes: 0.5 + amplitude cos(2 pi (x cos t + y sin t) / period) + noise.

    The orientation t and the period vary smoothly (correlation length corr_len,
    default max(h, w) / 8); the noise is white Gaussian (std `noise`, drawn per
    channel).  flat_box = (r0, c0, rh, rw) sets that rectangle to 0.5 exactly (no
    stripes, no noise).  uint16 images map [0, 1] to {0..65535} (rounded, clipped).
    """
    if corr_len is None:
        corr_len = max(4.0, max(h, w) / 8.0)
    rng = np.random.default_rng(seed + 3_333_333)
    n1 = _gauss_smooth_periodic(rng.standard_normal((h, w)), corr_len)
    n2 = _gauss_smooth_periodic(rng.standard_normal((h, w)), corr_len)
    t = 0.5 * np.arctan2(n2, n1)
    lam = period[0] + smooth_uniform_field(h, w, rng, corr_len) * (period[1] - period[0])
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    base = 0.5 + amplitude * np.cos(2.0 * np.pi * (x * np.cos(t) + y * np.sin(t)) / lam)
    chans = []
    for _ in range(channels):
        f = base + noise * rng.standard_normal((h, w))
        if flat_box is not None:
            r0, c0, rh, rw = flat_box
            f[r0:r0 + rh, c0:c0 + rw] = 0.5
        chans.append(f)
    f = chans[0] if channels == 1 else np.stack(chans, axis=-1)
    if dtype == "u16":
        return np.ascontiguousarray(np.clip(np.rint(f * 65535.0), 0, 65535).astype(np.uint16))
    return np.ascontiguousarray(f.astype(np.float32))
