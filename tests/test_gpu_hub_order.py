"""Edge sweeps of at least 2^20 edges run over records sorted by hub (the end
point of larger degree); smaller ones, and every shard call, keep the input
order.  The record order changes no pair, so both orders must give the
closed-form result of gen.hatch_and_stars: hubs of degree 65,538 beside a
hatch of 2^18 x 2^18 right-angle crossings, node ids and edge order shuffled.

Counts exact; the crossing angle within the bound of the sweeps' integer
line angles (see _angle_tol), and within 1e-9 between the two orders.
"""
import sys

import pytest

from paper_2411_09809_amd import gen
from _angle_tol import approx_dev, approx_eca
from test_oracle_pins import hatch_and_stars_closed_form

pytestmark = pytest.mark.gpu
IDEAL = gen.IDEAL_ANGLE
N_LINES, N_STARS, R = 1 << 18, 8, 30000


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def metrics():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2411_09809_amd import metrics
    return metrics


# q = 16384: 1,048,600 edges (hub order); q = 16380: 1,048,472 (input order)
@pytest.mark.parametrize("q,seed", [(16384, 5), (16380, 6)])
def test_hatch_and_stars_at_the_hub_sort_threshold(metrics, q, seed):
    L = gen.hatch_and_stars(N_LINES, N_STARS, q, R, seed)
    want_c, want_d = hatch_and_stars_closed_form(N_LINES, N_STARS, q, R, IDEAL)
    say(f"[hub] V={L.n_nodes} E={L.n_edges} sorted={L.n_edges >= 1 << 20} want {want_c}")
    D = metrics.DeviceLayout.from_host(L)
    eca, cnt, dev = metrics.crossing_angle(D.x, D.y, D.src, D.dst, IDEAL)
    say(f"[hub] whole: count {cnt} dev {dev!r}")
    assert cnt == want_c
    assert dev == approx_dev(want_d, want_c, IDEAL)
    assert eca == approx_eca(1 - want_d / want_c, IDEAL)
    c, p = metrics.edge_crossing(D.x, D.y, D.src, D.dst)
    say(f"[hub] count only: {c} proper {p}")
    assert c == p == want_c
    # one shard of one: the same pairs in input order
    sc, sdev, r0, r1 = metrics.crossing_angle_shard(D.x, D.y, D.src, D.dst, 0, 1, IDEAL)
    say(f"[hub] shard 0/1: count {sc} dev {sdev!r} rows [{r0}, {r1})")
    assert (sc, r0, r1) == (want_c, 0, L.n_edges)
    assert sdev == pytest.approx(dev, rel=1e-9)
