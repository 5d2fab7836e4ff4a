"""The scale map's root finding (the GPU kernel's sequence of steps, emulated in binary64
with its hardware reciprocal / square-root / cube-root estimates perturbed by their
~1e-7 error) against exact rational roots of zeta' (bisection in fractions):

* Cardano's seed and two Newton steps on the depressed cubic reach ~3e-14 of the scale
  where P >= scale^2 / 100;
* where P is smaller, the extra Newton step on zeta' evaluated from the shifted
  components reaches ~1e-16 of the scale.
Inputs: requests (s, rho, theta) over s 10^-2.5 .. 10^3.5 px^2, rho 1 .. 10^3.5."""
from fractions import Fraction as F

import numpy as np

RNG = np.random.default_rng(41)


def est(x):
    return x * (1 + RNG.uniform(-1.2e-7, 1.2e-7))


def kd(pb, t):
    q1, q2, q3, q4 = pb[0] + t, pb[1] - t, pb[2] + t, pb[3] - t
    A, B = q1 * q1 + q3 * q3, q2 * q2 + q4 * q4
    s13, s24 = q1 + q3, q2 + q4
    d1 = 4 * (q1 ** 3 - q2 ** 3 + q3 ** 3 - q4 ** 3) + 2 * s13 * B - 2 * s24 * A
    d2 = 16 * (A + B) - 8 * s13 * s24
    return d1, d2


def solve_model(pb):
    p1, p2, p3, p4 = pb
    scale = max(abs(p1), abs(p2), abs(p3), 1.0)
    s13, s24 = p1 + p3, p2 + p4
    z2 = 24 * (s13 - s24)
    z3 = 16 * (p1 * p1 + p2 * p2 + p3 * p3 + p4 * p4) - 8 * s13 * s24
    z4 = 4 * (p1 ** 3 - p2 ** 3 + p3 ** 3 - p4 ** 3) + 2 * s13 * (p2 * p2 + p4 * p4) - 2 * s24 * (p1 * p1 + p3 * p3)
    b = z2 / 96
    e3 = z3 / 32
    P = e3 - 3 * b * b
    Q = b * (2 * b * b - e3) + z4 / 32
    D = 0.25 * Q * Q + P * P * P / 27
    u = -0.5 * Q - np.copysign(est(np.sqrt(D)), Q)
    au = np.float32(abs(u))
    A = np.copysign(float(np.float32(2.0) ** (np.float32(np.log2(au)) * np.float32(1 / 3))), u)
    x = A - P / 3 * est(1 / A)
    for _ in range(2):
        x2 = x * x
        x -= (x * (x2 + P) + Q) * est(1 / (3 * x2 + P))
    t = x - b
    if not P >= 0.01 * scale * scale:
        d1, d2 = kd(pb, t)
        t -= d1 * est(1 / d2)
    return t, scale, P / scale ** 2


def exact_root(pb, scale):
    pbF = [F(v) for v in pb]
    lo, hi = F(-10 * scale - 10), F(10 * scale + 10)
    for _ in range(80):
        m = (lo + hi) / 2
        if kd(pbF, m)[0] > 0:
            hi = m
        else:
            lo = m
    return float(lo)


def test_root_accuracy_both_regimes():
    worst = {"large P": 0.0, "small P": 0.0}
    seen = {"large P": 0, "small P": 0}
    while min(seen.values()) < 40:
        s = 10 ** RNG.uniform(-2.5, 3.5)
        rho = 10 ** RNG.uniform(0, 3.5)
        th = RNG.uniform(0, np.pi)
        lmin = s / (1 + rho)
        dl = lmin * (rho - 1)
        c, sn = np.cos(th), np.sin(th)
        C11, C12, C22 = lmin + dl * c * c, dl * c * sn, lmin + dl * sn * sn
        pb = [12 * (C11 - C12) - 1, 24 * C12 + 1, 12 * (C22 - C12) - 1, 1.0]
        t, scale, pr = solve_model(pb)
        key = "large P" if pr >= 0.01 else "small P"
        if seen[key] >= 40:
            continue
        seen[key] += 1
        worst[key] = max(worst[key], abs(t - exact_root(pb, scale)) / scale)
    print(worst)
    assert worst["large P"] < 1e-13
    assert worst["small P"] < 1e-15
