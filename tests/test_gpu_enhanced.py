"""The strip approximation of Sections 3.2.2 / 3.2.3 (rb_enhanced_crossing)
against the oracle's strip method: the count bit for bit and the deviation
sum to 1e-9 relative, for vertical and horizontal strips of several widths,
on crowded, uniform, clustered and single-strip layouts.  Also: the count
never exceeds the exact E_c, and it equals E_c when every crossing lies
strictly inside a strip both edges span.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2411_09809_amd import gen
from _angle_tol import approx_dev

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


CASES = [(60, 150, 24, 1, f) for f in (1, 5, 24)] + \
        [(400, 1000, 256, 2, f) for f in (1, 8, 64, 256)] + \
        [(2000, 5000, 4096, 3, f) for f in (1, 8, 64)] + \
        [(3000, 7000, 1 << 16, 4, f) for f in (1, 16, 64)]


@pytest.mark.parametrize("V,E,extent,seed,frac", CASES)
@pytest.mark.parametrize("horizontal", [False, True])
def test_matches_oracle(torch_mod, V, E, extent, seed, frac, horizontal):
    from paper_2411_09809_amd import metrics
    L = gen.uniform_layout(V, E, extent=extent, seed=seed)
    D = metrics.DeviceLayout.from_host(L)
    width = max(1, extent // frac)
    eca, cnt, dev, pieces = metrics.enhanced_crossing(D.x, D.y, D.src, D.dst, width, horizontal)
    rc, rdev = oracle.enhanced_crossing(L.x, L.y, L.src, L.dst, width, horizontal, IDEAL)
    assert cnt == rc
    assert dev == pytest.approx(rdev, rel=1e-9, abs=1e-12)
    assert eca == pytest.approx(1.0 - rdev / rc if rc else 1.0, rel=1e-9, abs=1e-12)
    exact = oracle.edge_crossing(L.x, L.y, L.src, L.dst)[0]
    assert cnt <= exact


def test_single_strip_is_exact(torch_mod):
    from paper_2411_09809_amd import metrics
    rng = np.random.default_rng(3)
    n = 3000
    p = rng.permutation(n)
    x = np.concatenate([np.zeros(n), np.full(n, 1 << 19)])
    y = np.concatenate([np.arange(n) * 7, p * 7])
    L = gen._finish(x, y, np.arange(n), np.arange(n) + n, diameter=1.0, name="perm")
    D = metrics.DeviceLayout.from_host(L)
    eca, cnt, dev, _ = metrics.enhanced_crossing(D.x, D.y, D.src, D.dst, 1 << 19)
    ex = metrics.crossing_angle(D.x, D.y, D.src, D.dst)
    assert cnt == ex[1]
    # the strip kernel works on double line angles, the sweep on integer ones
    assert dev == approx_dev(ex[2], cnt, gen.IDEAL_ANGLE)


def test_clustered_and_workspace_growth(torch_mod):
    from paper_2411_09809_amd import metrics
    L = gen.ba_cluster_layout(n_nodes=3000, seed=5)
    D = metrics.DeviceLayout.from_host(L)
    for width in (1 << 18, 1 << 15, 1 << 13):
        eca, cnt, dev, pieces = metrics.enhanced_crossing(D.x, D.y, D.src, D.dst, width)
        rc, rdev = oracle.enhanced_crossing(L.x, L.y, L.src, L.dst, width, False, IDEAL)
        say(f"[enhanced] width={width} pieces={pieces} count={cnt}")
        assert cnt == rc
        assert dev == pytest.approx(rdev, rel=1e-9, abs=1e-12)


def test_force_directed_layout(torch_mod):
    from paper_2411_09809_amd import metrics
    L = gen.force_directed_layout(n_nodes=1000, n_groups=8, intra=1200, inter=500, seed=3)
    D = metrics.DeviceLayout.from_host(L)
    for width, hz in ((65, False), (33, True), (1024, False)):
        eca, cnt, dev, _ = metrics.enhanced_crossing(D.x, D.y, D.src, D.dst, width, hz)
        rc, rdev = oracle.enhanced_crossing(L.x, L.y, L.src, L.dst, width, hz, IDEAL)
        assert cnt == rc
        assert dev == pytest.approx(rdev, rel=1e-9, abs=1e-12)
