"""The crossing classification of the sweep kernels, checked against
Algorithm 4's printed form in exact integer arithmetic (CPU only).

The kernels never form the orientation products o1 o2 and o3 o4.  They hold
each edge as its end-point sum S = P + Q, its direction D = Q - P and 2c
(c = D x P), and compute

    t1 = dx_e S_f.y - dy_e S_f.x - 2 c_e   (= 2 o1 + cross)
    t3 = dx_f S_e.y - dy_f S_e.x - 2 c_f   (= 2 o3 - cross)
    t  = max(|t1|, |t3|),  cross = dx_e dy_f - dy_e dx_f

and classify a pair as crossing properly iff t < |cross| and as the rare case
(the larger product zero) iff t == |cross|.  These tests pin that reading to
max(o1 o2, o3 o4) < 0 and == 0, and check that every intermediate stays below
2^53 at the coordinate limit 2^20, so the kernels' FP64 arithmetic is exact.
"""
import math
import random

import pytest

LIM = 1 << 20


def orient(px, py, dx, dy, qx, qy):
    """Algorithm 4's CCW determinant of q against the line through p along d."""
    return dx * (qy - py) - dy * (qx - px)


def printed(e, f):
    """max(o1 o2, o3 o4) as Algorithm 4 forms it."""
    (ax, ay), (bx, by) = e
    (cx, cy), (qx, qy) = f
    o1 = orient(ax, ay, bx - ax, by - ay, cx, cy)
    o2 = orient(ax, ay, bx - ax, by - ay, qx, qy)
    o3 = orient(cx, cy, qx - cx, qy - cy, ax, ay)
    o4 = orient(cx, cy, qx - cx, qy - cy, bx, by)
    return max(o1 * o2, o3 * o4)


def sweep_form(seg):
    (px, py), (qx, qy) = seg
    dx, dy = qx - px, qy - py
    c = dx * py - dy * px
    return px + qx, py + qy, dx, dy, 2 * c


def kernel(e, f):
    """The kernels' classification and the largest intermediate magnitude."""
    sxe, sye, dxe, dye, c2e = sweep_form(e)
    sxf, syf, dxf, dyf, c2f = sweep_form(f)
    t1 = dxe * syf - dye * sxf - c2e
    t3 = dxf * sye - dyf * sxe - c2f
    cross = dxe * dyf - dye * dxf
    t = max(abs(t1), abs(t3))
    big = max(abs(v) for v in (sxe, sye, dxe, dye, c2e, sxf, syf, dxf, dyf, c2f,
                               dxe * syf, dye * sxf, dxf * sye, dyf * sxe, t1, t3,
                               dxe * dyf, dye * dxf, cross))
    return (t < abs(cross)), (t == abs(cross)), big


def classify(m):
    return m < 0, m == 0


def test_sign_identity_on_integers():
    """o (o + c) and |2 o + c| - |c| have the same sign, zero included."""
    rng = random.Random(1)
    vals = [0, 1, -1, 2, -2, 3, (1 << 44) - 1, -(1 << 44)]
    pairs = [(a, b) for a in vals for b in vals]
    pairs += [(rng.randint(-(1 << 44), 1 << 44), rng.randint(-(1 << 44), 1 << 44))
              for _ in range(20000)]
    pairs += [(a, -2 * a) for a in vals] + [(a, -a) for a in vals]
    for o, c in pairs:
        p = o * (o + c)
        q = abs(2 * o + c) - abs(c)
        assert (p > 0) == (q > 0) and (p < 0) == (q < 0) and (p == 0) == (q == 0), (o, c)


def _segments(rng, n, lim):
    out = []
    for _ in range(n):
        out.append(((rng.randint(-lim, lim), rng.randint(-lim, lim)),
                    (rng.randint(-lim, lim), rng.randint(-lim, lim))))
    return out


@pytest.mark.parametrize("lim", [4, 40, LIM])
def test_kernel_form_equals_printed_form(lim):
    """Random segment pairs, small canvases (many touching and collinear
    pairs) and the full coordinate range: the same decision every time, and
    every intermediate below 2^53."""
    rng = random.Random(lim)
    segs = _segments(rng, 400, lim)
    biggest = 0
    for i in range(0, len(segs), 2):
        for j in range(len(segs)):
            e, f = segs[i], segs[j]
            crossing, rare, big = kernel(e, f)
            assert (crossing, rare) == classify(printed(e, f)), (e, f)
            biggest = max(biggest, big)
    assert biggest < 1 << 53


def test_constructed_cases():
    """Shared end points, T-junctions, collinear overlaps and disjoint
    collinear pieces, zero-length edges and parallel lines."""
    cases = [
        (((0, 0), (4, 4)), ((0, 4), (4, 0))),      # proper crossing
        (((0, 0), (4, 0)), ((4, 0), (4, 4))),      # shared end point
        (((0, 0), (4, 0)), ((2, 0), (2, 3))),      # T-junction
        (((0, 0), (4, 0)), ((2, 0), (6, 0))),      # collinear overlap
        (((0, 0), (1, 0)), ((2, 0), (3, 0))),      # collinear, disjoint
        (((0, 0), (0, 0)), ((0, 0), (3, 3))),      # zero-length edge on the other
        (((1, 1), (1, 1)), ((0, 0), (0, 3))),      # zero-length edge off the other
        (((0, 0), (4, 0)), ((0, 1), (4, 1))),      # parallel lines
        (((-LIM, -LIM), (LIM, LIM)), ((-LIM, LIM), (LIM, -LIM))),   # extreme corners
        (((-LIM, 0), (LIM, 0)), ((LIM, -LIM), (LIM, LIM))),         # extreme T-junction
    ]
    want = [(True, False), (False, True), (False, True), (False, True), (False, True),
            (False, True), (False, False), (False, False), (True, False), (False, True)]
    for (e, f), w in zip(cases, want):
        got = kernel(e, f)[:2]
        assert got == classify(printed(e, f)) == w, (e, f, got)
        assert kernel(f, e)[:2] == got, (e, f)


# ---------------------------------------------------------------- node sweep
def cell(v):
    """The node sweep's cell coordinate: floor((v + 2^20) / 32) in [0, 65535]."""
    return min(max((v + LIM) >> 5, 0), 65535)


def cell_limit(T):
    """t of the node sweep's filter: isqrt(2 T) / 32 + 2 (None: no pair occludes)."""
    return None if T < 0 else math.isqrt(2 * T) // 32 + 2


def threshold(d):
    """Largest integer below d^2 (the occlusion test is |p - q|^2 <= T)."""
    return -1 if d <= 0 else math.ceil(d * d) - 1


@pytest.mark.parametrize("d", [0.5, 1.0, 8.0, 16.0, 45.3, 64.0, 1000.0, 30000.0])
def test_cell_filter_keeps_every_occluding_pair(d):
    """Every pair with |p - q|^2 <= T has cell distance |dcx| + |dcy| <= t:
    offsets on and near the boundary circle (the largest L1 for a given
    distance is on the diagonals), at every alignment to the 32-unit cells,
    including the clamped extremes of the coordinate range."""
    T = threshold(d)
    t = cell_limit(T)
    rng = random.Random(int(d * 100))
    r = math.isqrt(T)
    offsets = set()
    for dx in range(0, r + 1, max(1, r // 200)):
        dy = math.isqrt(T - dx * dx)
        offsets.update({(dx, dy), (dy, dx), (dx, max(dy - 1, 0))})
    for dx, dy in offsets:
        assert dx * dx + dy * dy <= T
        for _ in range(12):
            px = rng.choice([rng.randint(-LIM, LIM), -LIM, LIM - dx, rng.randint(-64, 64)])
            py = rng.choice([rng.randint(-LIM, LIM), -LIM, LIM - dy, rng.randint(-64, 64)])
            for sx, sy in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
                qx, qy = px + sx * dx, py + sy * dy
                if not (-LIM <= qx <= LIM and -LIM <= qy <= LIM):
                    continue
                dist = abs(cell(px) - cell(qx)) + abs(cell(py) - cell(qy))
                assert dist <= t, (d, px, py, qx, qy, dist, t)
    # the benchmark diameters attain the bound: from the last point of a
    # cell along the diagonal
    if d in (8.0, 16.0, 64.0):
        h = math.isqrt(T // 2)
        p = -LIM + 31
        assert abs(cell(p) - cell(p + h)) * 2 == t, (d, h, t)


def test_cell_limit_special_cases():
    assert cell_limit(threshold(0.0)) is None          # nothing occludes
    assert cell_limit(threshold(0.5)) == 2             # T = 0: coincident nodes only
    assert cell_limit(threshold(16.0)) == 2            # 2 T = 510: isqrt 22
    assert cell_limit(threshold(64.0)) == 4            # 2 T = 8190: isqrt 90
    assert cell(-LIM) == 0 and cell(LIM) == cell(LIM - 32) == 65535 and cell(LIM - 33) == 65534


# ------------------------------------------------------- integer line angles
ANGLE_UNIT = math.pi / 2 ** 26          # pi/2 is exactly 2^25 units
HALF_PI_Q = 1 << 25


def quantize(th):
    """The edge preparation's rint(th / u) (round half to even, as rint)."""
    return round(th * (2 ** 26 / math.pi))


def deviation_double(th_e, th_f, ideal):
    """|ideal - a| with a = pi/2 - ||th_e - th_f| - pi/2| (the acute angle)."""
    a = math.pi / 2 - abs(abs(th_e - th_f) - math.pi / 2)
    return abs(ideal - a)


def deviation_integer(tq_e, tq_f, beta_q):
    """The sweep's three v_sad_u32: ||tq_e - tq_f| - 2^25| then |. - beta|."""
    e = abs(abs(tq_e - tq_f) - HALF_PI_Q)
    return abs(e - beta_q)


@pytest.mark.parametrize("ideal", [math.radians(70), math.pi / 2, math.radians(45),
                                   math.radians(1), 1e-3])
def test_integer_angle_deviation_within_one_and_a_half_units(ideal):
    """Each crossing's deviation on the integer angles is within 1.5 units of
    the double expression, stays in [0, 2^25], and 4 rows x 16 columns of
    them cannot overflow the lanes' 32-bit sums."""
    rng = random.Random(int(ideal * 1e6))
    beta_q = quantize(math.pi / 2 - ideal)
    worst = 0.0
    cases = [(rng.uniform(0, math.pi), rng.uniform(0, math.pi)) for _ in range(20000)]
    cases += [(0.0, math.pi / 2), (0.0, 0.0), (math.pi - 1e-12, 0.0), (1.0, 1.0 + ideal),
              (0.3, 0.3 + math.pi / 2 - ideal), (2.0, 2.0 - ideal)]
    for th_e, th_f in cases:
        q = deviation_integer(quantize(th_e), quantize(th_f), beta_q)
        assert 0 <= q <= HALF_PI_Q
        err = abs(q * ANGLE_UNIT - deviation_double(th_e, th_f, ideal))
        worst = max(worst, err)
    assert worst <= 1.5 * ANGLE_UNIT + 1e-15
    assert 4 * 16 * HALF_PI_Q < 2 ** 32


def test_integer_deviation_invariant_under_a_quarter_turn():
    """A 90-degree rotation adds pi/2 to every line angle (mod pi), which is
    2^25 units: adding 2^25 (mod 2^26) to both angles of a pair leaves its
    integer deviation unchanged."""
    rng = random.Random(5)
    for _ in range(5000):
        a, b = rng.randrange(0, 2 ** 26), rng.randrange(0, 2 ** 26)
        ra, rb = (a + HALF_PI_Q) % 2 ** 26, (b + HALF_PI_Q) % 2 ** 26
        for beta_q in (0, 123456, HALF_PI_Q // 3):
            assert deviation_integer(a, b, beta_q) == deviation_integer(ra, rb, beta_q)
