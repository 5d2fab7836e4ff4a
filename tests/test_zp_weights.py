"""The branch-free form of the ZP interpolation weights used by the finite
difference (App. F: F(y) = sum_m g[m] ZP(y - m) over the 3 x 3 lattice block
around the nearest lattice point), checked against the oracle's ZP evaluated by
polygon clipping (eq. (const) with a = b).

With d = (dx, dy) the remainder, u = dx - dy, v = dx + dy, U = u|u|, V = v|v|,
8 x the weights are
  (0, 0): 4 - 2 (|U| + |V|)
  (+-1, 0): 1 + 2uv +- 4dx -+ (U + V)
  (0, +-1): 1 - 2uv +- 4dy +- (U - V)
  (1, 1): |V| + V, (-1, -1): |V| - V, (1, -1): |U| + U, (-1, 1): |U| - U
((i, j) = column offset i, row offset j).  The kernel reads 7 samples: of each
diagonal pair of corners only the one on the remainder's side, with weight 2|V|
(v >= 0: (1, 1), else (-1, -1)) and 2|U| (u >= 0: (1, -1), else (-1, 1)).
"""
import numpy as np
import pytest


def weights9(dx, dy):
    u, v = dx - dy, dx + dy
    U, V = u * abs(u), v * abs(v)
    S, D = U + V, U - V
    A = 1 + 2 * u * v
    B = 2 - A
    return {(0, 0): 4 - 2 * (abs(U) + abs(V)), (1, 0): A + 4 * dx - S, (-1, 0): A - 4 * dx + S,
            (0, 1): B + 4 * dy + D, (0, -1): B - 4 * dy - D, (1, 1): abs(V) + V, (-1, -1): abs(V) - V,
            (1, -1): abs(U) + U, (-1, 1): abs(U) - U}


def weights7(dx, dy):
    u, v = dx - dy, dx + dy
    w = {k: val for k, val in weights9(dx, dy).items() if 0 in k}
    w[(1, 1) if v >= 0 else (-1, -1)] = 2 * abs(v * abs(v))
    w[(1, -1) if u >= 0 else (-1, 1)] = 2 * abs(u * abs(u))
    return w


def _points(rng, n):
    pts = [tuple(rng.uniform(-0.5, 0.5, 2)) for _ in range(n)]
    # the diagonals and the cell border, where the pieces meet
    for t in np.linspace(-0.5, 0.5, 21):
        pts += [(t, t), (t, -t), (0.5, t), (-0.5, t), (t, 0.5), (t, -0.5)]
    return pts


@pytest.mark.parametrize("form", [weights9, weights7])
def test_weights_equal_zp(orc, form):
    rng = np.random.default_rng(7)
    worst = 0.0
    for dx, dy in _points(rng, 400):
        w = form(dx, dy)
        for i in (-1, 0, 1):
            for j in (-1, 0, 1):
                ref = 8.0 * orc.zp(dx - i, dy - j)
                worst = max(worst, abs(w.get((i, j), 0.0) - ref))
    assert worst < 1e-13


def test_no_weight_outside_block(orc):
    # lattice points two steps away carry no weight for any remainder in the cell
    rng = np.random.default_rng(8)
    for dx, dy in _points(rng, 200):
        for i in (-2, 2):
            for j in (-2, -1, 0, 1, 2):
                assert abs(orc.zp(dx - i, dy - j)) < 1e-15
                assert abs(orc.zp(dx - j, dy - i)) < 1e-15


def test_partition_of_unity():
    rng = np.random.default_rng(9)
    for dx, dy in _points(rng, 200):
        assert abs(sum(weights7(dx, dy).values()) - 8.0) < 1e-13
