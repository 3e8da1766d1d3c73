"""Randomised parity on tiny layouts (hypothesis): every metric, the pruned
and grid paths and the overlapped evaluation against the oracle.

Coordinates come from small grids, so collinear, touching, coincident and
zero-length configurations are frequent; ids are distinct pairs without
self-loops (the layout preconditions).  Counts must match bit for bit,
floating metrics within 1e-9 relative (the bar is 1e-5), the crossing angle
within the bound of its integer line angles (see _angle_tol).  The examples are
derandomised, so every run checks the same layouts.
"""
import sys

import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import HealthCheck, given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402
from paper_2411_09809_amd import gen  # noqa: E402
from _angle_tol import approx_dev, approx_eca  # noqa: E402

pytestmark = pytest.mark.gpu
IDEAL = gen.IDEAL_ANGLE


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


@st.composite
def layouts(draw):
    n = draw(st.integers(2, 24))
    span = draw(st.sampled_from([3, 6, 12, 1 << 20]))
    lo = draw(st.sampled_from([0, -span // 2]))
    xs = draw(st.lists(st.integers(lo, lo + span), min_size=n, max_size=n))
    ys = draw(st.lists(st.integers(lo, lo + span), min_size=n, max_size=n))
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    k = draw(st.integers(1, min(len(pairs), 60)))
    idx = draw(st.lists(st.integers(0, len(pairs) - 1), min_size=k, max_size=k, unique=True))
    flip = draw(st.lists(st.booleans(), min_size=k, max_size=k))
    e = [pairs[i][::-1] if f else pairs[i] for i, f in zip(idx, flip)]
    d = draw(st.sampled_from([0.5, 1.0, 1.5, 2.0, 3.0, 7.0]))
    src = np.array([a for a, _ in e]); dst = np.array([b for _, b in e])
    return gen._finish(np.array(xs), np.array(ys), src, dst, diameter=d, name=f"fuzz span {span}")


def close(a, b):
    return abs(a - b) <= 1e-9 * abs(b) + 1e-12


@settings(max_examples=150, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.function_scoped_fixture, HealthCheck.too_slow])
@given(L=layouts())
def test_tiny_layouts_match_the_oracle(torch_mod, L):
    from paper_2411_09809_amd import metrics
    D = metrics.DeviceLayout.from_host(L)
    want = oracle.all_metrics(L)
    c, p = metrics.edge_crossing(D.x, D.y, D.src, D.dst)
    assert (c, p) == (want["edge_crossing"], want["proper_crossing"]), (L.x, L.y, L.src, L.dst)
    eca, cnt, dev = metrics.crossing_angle(D.x, D.y, D.src, D.dst, IDEAL)
    assert cnt == want["edge_crossing"]
    assert eca == approx_eca(want["crossing_angle"], IDEAL)
    assert dev == approx_dev(want["crossing_dev_sum"], cnt, IDEAL)
    assert metrics.node_occlusion(D.x, D.y, L.diameter) == want["node_occlusion"]
    assert metrics.node_occlusion_grid(D.x, D.y, L.diameter) == want["node_occlusion"]
    pr = metrics.crossing_angle_pruned(D.x, D.y, D.src, D.dst, IDEAL)
    assert pr[1] == want["edge_crossing"] and pr[0] == approx_eca(want["crossing_angle"], IDEAL)
    ma, sdv, used = metrics.min_angle(D.x, D.y, D.src, D.dst)
    assert used == want["min_angle_n_used"] and close(ma, want["min_angle"])
    ml, mu = metrics.edge_length_variation(D.x, D.y, D.src, D.dst)
    assert close(ml, want["edge_length_variation"])
    got = metrics.evaluate(D)
    for k in ("node_occlusion", "edge_crossing", "min_angle_n_used"):
        assert got[k] == want[k]
    assert got["crossing_angle"] == approx_eca(want["crossing_angle"], IDEAL)
    for k in ("min_angle", "edge_length_variation"):
        assert close(got[k], want[k])


@settings(max_examples=80, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.function_scoped_fixture, HealthCheck.too_slow])
@given(L=layouts(), wm=st.sampled_from([0.0, 0.7]))
def test_tiny_loss_gradients_match_the_oracle(torch_mod, L, wm):
    """On small grids two smallest gaps at a vertex are often equal as real
    numbers (a kink: no gradient from that vertex); both sides decide such
    ties exactly on the integer directions, so every grid is fuzzed."""
    from paper_2411_09809_amd import metrics, optim
    D = metrics.DeviceLayout.from_host(L)
    S = oracle.crossing_pairs(L.x, L.y, L.src, L.dst)
    f_ref, gx_ref, gy_ref = oracle.loss_grad(L.x, L.y, L.src, L.dst, S, IDEAL, 0.9, 1.1, wm)
    for pruned in (False, True):
        f, gx, gy, cnt = optim.loss_grad(D.x, D.y, D.src, D.dst, IDEAL, 0.9, 1.1, pruned=pruned,
                                         w_min_angle=wm)
        assert int(cnt) == S.shape[0]
        assert close(float(f), f_ref)
        scale = max(np.abs(gx_ref).max(), np.abs(gy_ref).max(), 1e-300)
        for g, ref in ((gx.cpu().numpy(), gx_ref), (gy.cpu().numpy(), gy_ref)):
            assert np.abs(g - ref).max() <= 1e-9 * scale, (pruned, np.abs(g - ref).max(), scale)
