"""The interpolation table of the single-pass beta^{4,2} kernel (generated from the
refinement equation of box splines in exact rational arithmetic) against the oracle's
ZP*ZP (exact quadrature of a B-spline convolution): two independent derivations of
the same piecewise polynomial.  Also checks that the committed header is what the
generator writes, and the quarter-turn map of the four mesh triangles of the unit
square onto the tabulated one (the map the kernel applies per tap)."""
import re
from pathlib import Path

import numpy as np
import pytest

HDR = Path(__file__).resolve().parents[1] / "paper_1003_2022_amd" / "csrc" / "svf_zp2_table.h"


def load():
    """(monomials, C[36][28]): the coefficients in (u, dy), u = dx - 1/2, of every offset
    (i % 6 - 2, i / 6 - 2), rebuilt from the mirror pairs the header keeps."""
    src = HDR.read_text()
    mono = [tuple(map(int, m)) for m in re.findall(r"\{(\d), (\d)\}", src.split("kZp2Mono[28][2] =")[1].split(";")[0])]
    den = float(re.search(r"kZp2Den = ([0-9.]+);", src).group(1))
    body = src.split("kZp2Half[18][28] = {")[1].split("};")[0]
    vals = [float(v) for v in re.findall(r"[-+]?\d[\d.eE+-]*", re.sub(r"//[^\n]*", "", body))]
    half = np.array(vals).reshape(18, 28) / den
    C = np.zeros((36, 28))
    sign = np.array([(-1.0) ** p for p, q in mono])
    for i in range(18):
        lx, ly = i % 3 - 2, i // 3 - 2
        C[(ly + 2) * 6 + lx + 2] = half[i]
        C[(ly + 2) * 6 + (1 - lx) + 2] = half[i] * sign
    return mono, C


def weights(mono, C, dx, dy):
    """(lx, ly) -> weight of lattice offset l at fractional position (dx, dy)."""
    below, low = dy <= dx, dx + dy <= 1
    if below and low:
        q, px, py = 0, dx, dy
    elif below:
        q, px, py = 1, dy, 1 - dx
    elif not low:
        q, px, py = 2, 1 - dx, 1 - dy
    else:
        q, px, py = 3, 1 - dy, dx
    out = {}
    for i in range(36):
        a, b = i % 6 - 2, i // 6 - 2
        l = [(a, b), (1 - b, a), (1 - a, 1 - b), (b, 1 - a)][q]
        out[l] = sum(c * (px - 0.5) ** p * py ** qq for c, (p, qq) in zip(C[i], mono))
    return out


def test_header_is_generated():
    from paper_1003_2022_amd import gen_zp2_table

    import tempfile

    with tempfile.TemporaryDirectory() as d:
        text = gen_zp2_table.main(Path(d) / "t.h")
    assert text == HDR.read_text()


def test_table_equals_oracle_zp_conv(orc):
    mono, C = load()
    rng = np.random.default_rng(21)
    pts = list(rng.uniform(0, 1, (24, 2))) + [(0.3, 0.3), (0.7, 0.2), (0.5, 0.9), (0.1, 0.6)]
    for dx, dy in pts:
        w = weights(mono, C, dx, dy)
        assert sum(w.values()) == pytest.approx(1.0, abs=1e-14)
        for (lx, ly), v in w.items():
            assert v == pytest.approx(orc.zp_m(2, dx - lx, dy - ly), abs=2e-15)
