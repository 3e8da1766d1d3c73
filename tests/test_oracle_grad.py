"""Pins of the oracle's layout-optimisation loss and its analytic gradient.

L = w_a (1 - E_ca) + w_l M_l with the crossing set S frozen.  Independent
checks: central finite differences of the loss, the three exact symmetry
identities of a translation-, rotation- and scale-invariant function, the
metrics of Algorithms 3 and 5 at integer coordinates, and a closed-form
derivative (rotating one edge of a crossing pair).
"""
import math

import numpy as np
import pytest

from paper_2411_09809_amd import gen

IDEAL = gen.IDEAL_ANGLE


def jittered(seed, n=60, m=120, extent=400):
    """An integer layout, its crossing set, and coordinates moved off the
    grid by a small random amount (away from every kink)."""
    import oracle
    L = gen.uniform_layout(n, m, extent=extent, seed=seed)
    S = oracle.crossing_pairs(L.x, L.y, L.src, L.dst)
    rng = np.random.default_rng(seed)
    x = L.x.astype(np.float64) + rng.uniform(-0.3, 0.3, size=n)
    y = L.y.astype(np.float64) + rng.uniform(-0.3, 0.3, size=n)
    return L, S, x, y


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradient_matches_central_differences(orc, seed):
    L, S, x, y = jittered(seed)
    assert S.shape[0] > 20
    f0, gx, gy = orc.loss_grad(x, y, L.src, L.dst, S, IDEAL)
    h = 1e-5
    scale = max(np.abs(gx).max(), np.abs(gy).max())
    for v in range(L.n_nodes):
        for arr, g in ((x, gx), (y, gy)):
            old = arr[v]
            arr[v] = old + h
            fp = orc.loss(x, y, L.src, L.dst, S, IDEAL)
            arr[v] = old - h
            fm = orc.loss(x, y, L.src, L.dst, S, IDEAL)
            arr[v] = old
            fd = (fp - fm) / (2 * h)
            assert abs(fd - g[v]) <= 1e-6 * scale, (v, fd, g[v])


@pytest.mark.parametrize("seed", [4, 5])
def test_gradient_symmetry_identities(orc, seed):
    """L is invariant under translation, rotation and scaling, so its
    gradient has zero net force, zero torque and zero virial."""
    L, S, x, y = jittered(seed, n=200, m=500, extent=3000)
    _, gx, gy = orc.loss_grad(x, y, L.src, L.dst, S, IDEAL, 1.0, 1.0)
    mag = np.abs(gx).sum() + np.abs(gy).sum()
    r = np.abs(x).max() + np.abs(y).max()
    assert abs(gx.sum()) <= 1e-12 * mag
    assert abs(gy.sum()) <= 1e-12 * mag
    assert abs((x * gy - y * gx).sum()) <= 1e-12 * mag * r
    assert abs((x * gx + y * gy).sum()) <= 1e-12 * mag * r


def test_loss_at_integer_points_is_the_metrics(orc):
    L = gen.uniform_layout(400, 900, extent=2000, seed=8)
    S = orc.crossing_pairs(L.x, L.y, L.src, L.dst)
    eca, cnt, _ = orc.crossing_angle(L.x, L.y, L.src, L.dst, IDEAL)
    ml, _ = orc.edge_length_variation(L.x, L.y, L.src, L.dst)
    assert S.shape[0] == cnt
    assert orc.loss(L.x, L.y, L.src, L.dst, S, IDEAL, 1.0, 1.0) == pytest.approx(
        (1 - eca) + ml, rel=1e-13)
    assert orc.loss(L.x, L.y, L.src, L.dst, S, IDEAL, 2.5, 0.0) == pytest.approx(
        2.5 * (1 - eca), rel=1e-13)


def test_rotating_one_edge_of_a_crossing_pair(orc):
    """Edges (0,0)-(4,0) and (1,-1)-(3,1) cross at a = 45 deg < ideal.
    Rotating the second edge about its midpoint by dphi changes a by dphi,
    so d(|ideal - a| / ideal)/dphi = -1/ideal."""
    x = np.array([0.0, 4.0, 1.0, 3.0])
    y = np.array([0.0, 0.0, -1.0, 1.0])
    src, dst = np.array([0, 2]), np.array([1, 3])
    S = np.array([[0, 1]])
    f, gx, gy = orc.loss_grad(x, y, src, dst, S, IDEAL, 1.0, 0.0)
    assert f == pytest.approx((IDEAL - math.pi / 4) / IDEAL, rel=1e-14)
    # infinitesimal rotation about (2, 0): p -> p + dphi * (-(p_y - 0), p_x - 2)
    dphi = gx[2] * 1.0 + gy[2] * (-1.0) + gx[3] * (-1.0) + gy[3] * 1.0
    assert dphi == pytest.approx(-1.0 / IDEAL, rel=1e-12)
    # sliding an end of the horizontal edge along its own line keeps a
    assert gx[0] == pytest.approx(0.0, abs=1e-15) and gx[1] == pytest.approx(0.0, abs=1e-15)


def test_kinks_contribute_zero(orc):
    """Perpendicular crossing (g = 0) and parallel overlap (c = 0) give no
    angle gradient; equal edge lengths give no length gradient."""
    x = np.array([0.0, 2.0, 0.0, 2.0])
    y = np.array([0.0, 2.0, 2.0, 0.0])
    f, gx, gy = orc.loss_grad(x, y, [0, 2], [1, 3], [[0, 1]], IDEAL, 1.0, 1.0)
    assert f == pytest.approx(20 / 70, rel=1e-14)
    assert np.abs(gx).max() == 0.0 and np.abs(gy).max() == 0.0
    x = np.array([0.0, 4.0, 2.0, 6.0])
    y = np.zeros(4)
    f, gx, gy = orc.loss_grad(x, y, [0, 2], [1, 3], [[0, 1]], IDEAL, 1.0, 0.0)
    assert f == pytest.approx(1.0) and np.abs(gx).max() == 0.0 and np.abs(gy).max() == 0.0


# ---------------------------------------------------- the minimum-angle term

def test_min_angle_term_at_integer_points_is_one_minus_the_metric(orc):
    for seed in (1, 2):
        L = gen.uniform_layout(500, 1400, extent=3000, seed=seed)
        ma, _, _ = orc.min_angle(L.x, L.y, L.src, L.dst)
        assert orc.min_angle_term(L.x, L.y, L.src, L.dst, 1.0) == pytest.approx(1 - ma, rel=1e-12)
        assert orc.min_angle_term(L.x, L.y, L.src, L.dst, 2.5) == pytest.approx(2.5 * (1 - ma),
                                                                              rel=1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_min_angle_gradient_matches_central_differences(orc, seed):
    L, S, x, y = jittered(seed, n=60, m=150)
    t0, gx, gy = orc.min_angle_term(x, y, L.src, L.dst, 1.0, grad=True)
    h = 1e-6
    scale = max(np.abs(gx).max(), np.abs(gy).max())
    assert scale > 0
    for v in range(L.n_nodes):
        for arr, g in ((x, gx), (y, gy)):
            old = arr[v]
            arr[v] = old + h
            fp = orc.min_angle_term(x, y, L.src, L.dst, 1.0)
            arr[v] = old - h
            fm = orc.min_angle_term(x, y, L.src, L.dst, 1.0)
            arr[v] = old
            assert abs((fp - fm) / (2 * h) - g[v]) <= 1e-6 * scale, (v, (fp - fm) / (2 * h), g[v])


def test_min_angle_gradient_symmetry_identities(orc):
    L, S, x, y = jittered(6, n=300, m=900, extent=3000)
    _, gx, gy = orc.min_angle_term(x, y, L.src, L.dst, 1.0, grad=True)
    mag = np.abs(gx).sum() + np.abs(gy).sum()
    r = np.abs(x).max() + np.abs(y).max()
    assert mag > 0
    assert abs(gx.sum()) <= 1e-12 * mag and abs(gy.sum()) <= 1e-12 * mag
    assert abs((x * gy - y * gx).sum()) <= 1e-12 * mag * r
    assert abs((x * gx + y * gy).sum()) <= 1e-12 * mag * r


def test_min_angle_term_rotating_one_edge_closed_form(orc):
    """Node 0 with neighbours at angle 0 (node 1) and 60 degrees (node 2):
    phi = pi/3, 1 - M_a = 1 - (1/3)(phi*2/(2 pi) + 1 + 1).  Turning node 2
    about node 0 by +dphi widens phi by dphi: dT/dphi = -2/(2 pi * 3)."""
    x = np.array([0.0, 10.0, 5.0])
    y = np.array([0.0, 0.0, 5.0 * math.sqrt(3.0)])
    src, dst = np.array([0, 0]), np.array([1, 2])
    t, gx, gy = orc.min_angle_term(x, y, src, dst, 1.0, grad=True)
    assert t == pytest.approx(1 - (1 / 3) * (1 / 3 + 2), rel=1e-12)
    # rotation of node 2 about node 0: d(x2, y2)/dphi = (-y2, x2)
    dphi = gx[2] * -y[2] + gy[2] * x[2]
    assert dphi == pytest.approx(-2.0 / (2 * math.pi * 3), rel=1e-12)
    # kinks give no gradient: a tie (neighbours at 0 and 180 degrees, two gaps
    # of exactly pi) and a zero gap (two neighbours in one direction)
    for xs, ys in (([0.0, 10.0, -7.0], [0.0, 0.0, 0.0]), ([0.0, 10.0, 4.0], [0.0, 5.0, 2.0])):
        _, gx, gy = orc.min_angle_term(np.array(xs), np.array(ys), np.array([0, 0]),
                                       np.array([1, 2]), 1.0, grad=True)
        assert np.abs(gx).max() == 0.0 and np.abs(gy).max() == 0.0


# Two smallest gaps that are equal as real numbers but not as differences of
# rounded atan2 values: directions (2,1), (1,1), (1,2) from the centre give
# gaps pi/4 - atan(1/2) and atan(2) - pi/4, equal since atan(2) + atan(1/2) =
# pi/2.  Likewise (3,1)/(1,1)/(1,3) and (7,3)/(1,1)/(3,7).  A smallest gap
# attained twice is a kink of the minimum-angle term: no gradient.
TIE_STARS = [((2, 1), (1, 1), (1, 2)), ((3, 1), (1, 1), (1, 3)), ((7, 3), (1, 1), (3, 7)),
             ((5, 2), (3, 3), (2, 5))]


def _star(dirs, centre=(1000, 2000), turn=0):
    """Centre node 0 and one neighbour per direction, turned by turn * 90 deg."""
    xs, ys = [float(centre[0])], [float(centre[1])]
    for dx, dy in dirs:
        for _ in range(turn):
            dx, dy = -dy, dx
        xs.append(float(centre[0] + dx))
        ys.append(float(centre[1] + dy))
    k = len(dirs)
    return np.array(xs), np.array(ys), np.zeros(k, np.int32), np.arange(1, k + 1, dtype=np.int32)


@pytest.mark.parametrize("dirs", TIE_STARS)
@pytest.mark.parametrize("turn", [0, 1, 2, 3])
def test_min_angle_exact_ties_off_the_axes_give_no_gradient(orc, dirs, turn):
    x, y, s, d = _star(dirs, turn=turn)
    t, gx, gy = orc.min_angle_term(x, y, s, d, 1.0, grad=True)
    assert np.abs(gx).max() == 0.0 and np.abs(gy).max() == 0.0
    # the value is still the metric's: phi = the tied gap
    ma, _, _ = orc.min_angle(x, y, s, d)
    assert t == pytest.approx(1.0 - ma, rel=1e-12)


def test_min_angle_near_tie_moves_only_the_smaller_gap(orc):
    """(2,1), (1,1), (1,3): gaps pi/4 - atan(1/2) = 0.3218 and
    atan(3) - pi/4 = 0.4636.  Only the first bounds phi: turning (1,1) about
    the centre by +dt widens it by dt, turning (2,1) by +dt narrows it, and
    (1,3) has no gradient.  dT/dphi = -k / (2 pi N) with k = 3, N = 4."""
    x, y, s, d = _star(((2, 1), (1, 1), (1, 3)))
    _, gx, gy = orc.min_angle_term(x, y, s, d, 1.0, grad=True)
    c = -3.0 / (2 * math.pi * 4)
    turn = lambda i: gx[i] * -(y[i] - y[0]) + gy[i] * (x[i] - x[0])
    assert turn(2) == pytest.approx(c, rel=1e-12)
    assert turn(1) == pytest.approx(-c, rel=1e-12)
    assert gx[3] == 0.0 and gy[3] == 0.0
    assert gx.sum() == pytest.approx(0.0, abs=1e-15) and gy.sum() == pytest.approx(0.0, abs=1e-15)


def test_min_angle_tie_inside_a_layout(orc):
    """A tie star embedded in a random layout: the centre and its three
    neighbours get exactly the gradient the rest of the layout gives them
    (the star's own term is a kink), checked against the same layout with
    the tie broken by moving one neighbour one unit."""
    L = gen.uniform_layout(200, 380, extent=1 << 12, seed=9)
    x, y = L.x.astype(np.float64).copy(), L.y.astype(np.float64).copy()
    # four fresh nodes far from the others, wired as the (3,1)/(1,1)/(1,3) star
    sx, sy = [3500.0, 3503.0, 3501.0, 3501.0], [3500.0, 3501.0, 3501.0, 3503.0]
    n = L.n_nodes
    x = np.concatenate([x, sx]); y = np.concatenate([y, sy])
    src = np.concatenate([L.src, [n, n, n]]).astype(np.int32)
    dst = np.concatenate([L.dst, [n + 1, n + 2, n + 3]]).astype(np.int32)
    _, gx, gy = orc.min_angle_term(x, y, src, dst, 1.0, grad=True)
    assert np.abs(gx[n:]).max() == 0.0 and np.abs(gy[n:]).max() == 0.0
    assert np.abs(gx[:n]).max() > 0.0
    y2 = y.copy(); y2[n + 3] += 1.0                      # (1,3) -> (1,4): no tie
    _, gx2, gy2 = orc.min_angle_term(x, y2, src, dst, 1.0, grad=True)
    assert np.abs(gx2[n:]).max() > 0.0
