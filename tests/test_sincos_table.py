"""The scale map's sine/cosine table: the committed header is what its generator
writes, k h is exact, the entries are sin/cos(k h) to within one ulp, and the
reduction + table + short series the kernel uses reproduces sin/cos of float32
angles in [0, pi) to a few 1e-16 (emulated here in binary64)."""
import math
import re
import tempfile
from pathlib import Path

import numpy as np

HDR = Path(__file__).resolve().parents[1] / "paper_1003_2022_amd" / "csrc" / "svf_sincos_table.h"


def load():
    src = HDR.read_text()
    h = float.fromhex(re.search(r"kSinCosH = ([^;]+);", src).group(1))
    ih = float.fromhex(re.search(r"kSinCosInvH = ([^;]+);", src).group(1))
    tab = [(float.fromhex(a), float.fromhex(b)) for a, b in re.findall(r"\{(\S+), (\S+)\},", src)]
    return h, ih, tab


def test_header_is_generated():
    from paper_1003_2022_amd import gen_sincos_table

    with tempfile.TemporaryDirectory() as d:
        assert gen_sincos_table.main(Path(d) / "t.h") == HDR.read_text()


def test_entries():
    h, ih, tab = load()
    assert len(tab) == 65 and abs(h - math.pi / 128) < 1e-15
    for k in range(-32, 33):
        s, c = tab[k + 32]
        x = k * h
        assert abs(s - math.sin(x)) <= math.ulp(abs(s) or 1e-300) and abs(c - math.cos(x)) <= math.ulp(c)
        assert abs(s * s + c * c - 1.0) < 4e-16


def test_reduction_and_series():
    h, ih, tab = load()
    pio2_hi, pio2_lo = 1.57079632679489655800e+00, 6.12323399573676603587e-17
    rng = np.random.default_rng(31)
    worst = 0.0
    for th in list(rng.uniform(0, math.pi, 20000).astype(np.float32)) + [0.0, math.pi / 4, 3.1415925]:
        th = float(th)
        q = round(th * 0.63661977236758134308)
        r = (th - q * pio2_hi) - q * pio2_lo
        k = max(-32, min(32, round(r * ih)))
        e = r - k * h
        sk, ck = tab[k + 32]
        e2 = e * e
        se = e + e * e2 * (-1 / 6 + e2 / 120)
        ce = 1 + e2 * (-0.5 + e2 * (1 / 24 - e2 / 720))
        sv, cv = sk * ce + ck * se, ck * ce - sk * se
        s, c = [(sv, cv), (cv, -sv), (-sv, -cv), (-cv, sv)][q & 3]
        worst = max(worst, abs(s - math.sin(th)), abs(c - math.cos(th)))
    assert worst < 5e-16
