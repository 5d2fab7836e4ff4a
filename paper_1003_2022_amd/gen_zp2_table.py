"""Generate the interpolation table of the single-pass filter with beta^{4,2}.

The fast single pass with the iterated box spline beta^{4,m} (the box spline whose
four directions are each taken m times, eq. (iterated_spline)) interpolates the
m-fold running sums with the m-fold convolution of the ZP element, ZP*ZP for m = 2.
ZP*ZP is the box spline M with the lattice directions (1,0), (1,1), (0,1), (-1,1),
each twice: a piecewise polynomial of degree 6 on the four-direction mesh.  This
script derives its pieces in exact rational arithmetic from the refinement
equation of box splines

    M(x) = sum_j a_j M(2x - j),   a(z) = 2^(2-8) prod_xi (1 + z^xi),

(values on the integer lattice: the eigenvector of the refinement operator with
sum 1; then on the grids of step 1/2, 1/4, 1/8, 1/16), then fits, for each
lattice offset l of the 6 x 6 stencil, the polynomial W_l(dx, dy) = M_c((dx, dy) - l)
(M_c = M centred) on the mesh triangle T0 = {0 <= dy <= dx, dx + dy <= 1} from its
values on the order-8 principal lattice of T0 (45 points, exact least squares;
the residual is checked to be zero).  The other three triangles of the unit square
map onto T0 by the square's quarter turns, under which M_c is invariant.

T0 is symmetric about dx = 1/2 and M_c under x -> -x, so with u = dx - 1/2 the
offsets l = (lx, ly) and l' = (1 - lx, ly) have W_l'(u, dy) = W_l(-u, dy) (checked
exactly): for the pair, g_l W_l + g_l' W_l' = sum over the monomials u^p dy^q of
c_l[p, q] u^p dy^q times (g_l + g_l') for even p and (g_l - g_l') for odd p.  The
table keeps the 18 offsets with lx <= 0.

Writes csrc/svf_zp2_table.h: kZp2Half[18][28], the exact rational coefficients times
their common denominator kZp2Den (integers below 2^21), pair i = offsets
(i % 3 - 2, i / 3 - 2) and (3 - i % 3, i / 3 - 2), monomial u^p dy^q in the order
p + q = 0, 1, ..., 6 and, within a degree, q = 0, 1, ....

Usage: python -m paper_1003_2022_amd.gen_zp2_table   (a few seconds)
"""
from __future__ import annotations

from fractions import Fraction as Fr
from math import comb, lcm
from pathlib import Path

DIRS = [(1, 0), (1, 1), (0, 1), (-1, 1)] * 2
DEG = 6
MONO = [(d - q, q) for d in range(DEG + 1) for q in range(d + 1)]   # (p, q) of dx^p dy^q


def mask():
    poly = {(0, 0): Fr(1)}
    for xi in DIRS:
        nxt = {}
        for (x, y), c in poly.items():
            for s in ((0, 0), xi):
                k = (x + s[0], y + s[1])
                nxt[k] = nxt.get(k, Fr(0)) + c
        poly = nxt
    scale = Fr(1, 2 ** (len(DIRS) - 2))
    return {k: v * scale for k, v in poly.items()}


def solve(A, b):
    """Exact Gauss-Jordan elimination; A square (list of lists of Fractions)."""
    n = len(A)
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [vr - f * vc for vr, vc in zip(M[r], M[c])]
    return [M[r][n] for r in range(n)]


def box_values(levels: int):
    """M on the grid of step 2^-levels: dict (X, Y) -> value at (X, Y) / 2^levels."""
    a = mask()
    # support of M: sum of [0, 1] xi over the directions
    xs = [sum(min(0, d[0]) for d in DIRS), sum(max(0, d[0]) for d in DIRS)]
    ys = [sum(min(0, d[1]) for d in DIRS), sum(max(0, d[1]) for d in DIRS)]
    # integer lattice: unknowns strictly inside the bounding box (M vanishes on the
    # support's boundary, being continuous)
    pts = [(x, y) for x in range(xs[0] + 1, xs[1]) for y in range(ys[0] + 1, ys[1])]
    idx = {p: i for i, p in enumerate(pts)}
    n = len(pts)
    A = [[Fr(0)] * n for _ in range(n)]
    for i, (x, y) in enumerate(pts):
        A[i][i] -= 1
        for (jx, jy), c in a.items():
            k = (2 * x - jx, 2 * y - jy)
            if k in idx:
                A[i][idx[k]] += c
    b = [Fr(0)] * n
    A[0] = [Fr(1)] * n          # replace one equation by the normalisation sum = 1
    b[0] = Fr(1)
    v = solve(A, b)
    vals = {p: v[i] for i, p in enumerate(pts)}
    for lev in range(1, levels + 1):
        s = 2 ** lev
        nxt = {}
        for X in range(xs[0] * s + 1, xs[1] * s):
            for Y in range(ys[0] * s + 1, ys[1] * s):
                acc = Fr(0)
                for (jx, jy), c in a.items():
                    # 2x - j at the previous level: (2X/s - j) = (X - j s/2) / (s/2)
                    k = (X - jx * (s // 2), Y - jy * (s // 2))
                    w = vals.get(k)
                    if w:
                        acc += c * w
                if acc:
                    nxt[(X, Y)] = acc
        vals = nxt
    return vals, xs, ys


def main(out: Path | None = None) -> str:
    levels = 4
    s = 2 ** levels
    vals, xs, ys = box_values(levels)
    cx = Fr(sum(d[0] for d in DIRS), 2)
    cy = Fr(sum(d[1] for d in DIRS), 2)

    def mc(x: Fr, y: Fr) -> Fr:   # centred M at a point of the 1/16 grid
        X, Y = (x + cx) * s, (y + cy) * s
        assert X.denominator == 1 and Y.denominator == 1
        return vals.get((int(X), int(Y)), Fr(0))

    # order-8 principal lattice of T0 = (0,0), (1,0), (1/2,1/2)
    P = [(Fr(k1, 8) + Fr(k2, 16), Fr(k2, 16)) for k1 in range(9) for k2 in range(9 - k1)]
    V = [[px ** p * py ** q for (p, q) in MONO] for (px, py) in P]
    VtV = [[sum(V[i][r] * V[i][c] for i in range(len(P))) for c in range(len(MONO))] for r in range(len(MONO))]
    table = []
    for i in range(36):
        lx, ly = i % 6 - 2, i // 6 - 2
        yv = [mc(px - lx, py - ly) for (px, py) in P]
        rhs = [sum(V[k][r] * yv[k] for k in range(len(P))) for r in range(len(MONO))]
        coef = solve(VtV, rhs)
        res = max(abs(sum(c * v for c, v in zip(coef, V[k])) - yv[k]) for k in range(len(P)))
        assert res == 0, f"offset {(lx, ly)}: not a polynomial of degree {DEG} on T0"
        # and at further grid points of T0 (on the 1/16 grid, inside the closed triangle)
        for X in range(0, s + 1):
            for Y in range(0, s // 2 + 1):
                x, y = Fr(X, s), Fr(Y, s)
                if y <= x and x + y <= 1:
                    val = sum(c * x ** p * y ** q for c, (p, q) in zip(coef, MONO))
                    assert val == mc(x - lx, y - ly)
        table.append(coef)
    # partition of unity, as a polynomial identity
    for r in range(len(MONO)):
        assert sum(t[r] for t in table) == (1 if r == 0 else 0)
    # in u = dx - 1/2: expand (u + 1/2)^p
    def shift(coef):
        out = {m: Fr(0) for m in MONO}
        for c, (p, q) in zip(coef, MONO):
            if c == 0:
                continue
            for k in range(p + 1):   # (u + 1/2)^p = sum_k C(p, k) u^k (1/2)^(p - k)
                out[(k, q)] += c * Fr(comb(p, k)) * Fr(1, 2 ** (p - k))
        return [out[m] for m in MONO]
    cu = [shift(t) for t in table]
    half = []
    for i in range(18):
        lx, ly = i % 3 - 2, i // 3 - 2
        a = cu[(ly + 2) * 6 + (lx + 2)]
        b = cu[(ly + 2) * 6 + (1 - lx + 2)]
        for (p, q), ca, cb in zip(MONO, a, b):
            assert cb == (ca if p % 2 == 0 else -ca), f"mirror pair {(lx, ly)}"
        half.append(a)
    # one common denominator makes every coefficient a small integer: exact in binary64
    # and, with at most 21 significant bits, an immediate operand of the FMAs
    den = 1
    for row in half:
        for c in row:
            den = lcm(den, c.denominator)
    rows = []
    for i, coef in enumerate(half):
        lx, ly = i % 3 - 2, i // 3 - 2
        ints = [c * den for c in coef]
        assert all(v.denominator == 1 and abs(v) < 2 ** 21 for v in ints)
        body = ", ".join(f"{int(v)}.0" for v in ints)
        rows.append(f"    {body},   // ({lx}, {ly}) and ({1 - lx}, {ly})")
    text = (
        "// svf_zp2_table.h -- generated by paper_1003_2022_amd/gen_zp2_table.py; do not edit.\n"
        "// ZP*ZP (the box spline with the lattice directions (1,0), (1,1), (0,1), (-1,1) each\n"
        "// twice), centred: on the mesh triangle T0 = {0 <= dy <= dx, dx + dy <= 1}, with\n"
        "// u = dx - 1/2, the weights of the stencil offsets (lx, ly) = (i % 3 - 2, i / 3 - 2) and\n"
        "// (1 - lx, ly) at (dx, dy) are sum_r kZp2Half[i][r] (+-u)^p dy^q / kZp2Den,\n"
        "// (p, q) = kZp2Mono[r] (+u for the first, -u for the second); the coefficients are\n"
        "// exact integers.\n"
        "#pragma once\n\nnamespace svf {\n\n"
        f"constexpr int kZp2Deg = {DEG};\n"
        f"constexpr double kZp2Den = {den}.0;\n"
        "constexpr int kZp2Mono[28][2] = {" + ", ".join(f"{{{p}, {q}}}" for p, q in MONO) + "};\n\n"
        "constexpr double kZp2Half[18][28] = {\n" + "\n".join(rows) + "\n};\n\n}  // namespace svf\n")
    if out is None:
        out = Path(__file__).resolve().parent / "csrc" / "svf_zp2_table.h"
    out.write_text(text)
    return text


if __name__ == "__main__":
    print("wrote", main() and "csrc/svf_zp2_table.h")
