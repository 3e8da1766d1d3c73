"""Shards of the two all-pairs sweeps (rb_crossing_angle_shard,
rb_node_occlusion_shard) and the 1M-node / 3M-edge power-law layout.

* the shard row ranges are contiguous, tile-aligned and cover every row, and
  the shard results sum to the whole-layout result (exactly for counts);
* each shard equals the oracle's row slice (pairs (i, j), r0 <= i < r1,
  i < j) of the same layout;
* at 1M nodes / 3M edges, where the full O(|E|^2) oracle is out of reach:
  the first and last shard of 4096 against the oracle's row slices, the
  whole result against a 90-degree rotation of the layout (exact integer
  transform; counts are invariant), against the single shard (input record
  order; the whole call sweeps in hub order) and a different sweep variant,
  and minimum angle and edge length variation against the oracle.
Tolerance for deviation sums: 1e-9 relative (FP64, different summation order).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2411_09809_amd import gen
from _angle_tol import approx_dev, approx_eca

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


def _check_cover(ranges, n):
    assert ranges[0][0] == 0 and ranges[-1][1] == n
    for (a0, a1), (b0, b1) in zip(ranges, ranges[1:]):
        assert a1 == b0 and a0 <= a1


@pytest.mark.parametrize("n_shards", [1, 2, 3, 7, 64])
def test_shards_sum_to_whole(torch_mod, n_shards):
    from paper_2411_09809_amd import metrics
    L = gen.uniform_layout(20000, 50000, extent=1 << 14, seed=21)
    D = metrics.DeviceLayout.from_host(L)
    say(f"[shard] uniform V=20000 E=50000 n_shards={n_shards}")
    eca, cnt, dev = metrics.crossing_angle(D.x, D.y, D.src, D.dst, IDEAL)
    parts = [metrics.crossing_angle_shard(D.x, D.y, D.src, D.dst, k, n_shards, IDEAL)
             for k in range(n_shards)]
    _check_cover([(p[2], p[3]) for p in parts], L.n_edges)
    assert sum(p[0] for p in parts) == cnt
    assert sum(p[1] for p in parts) == pytest.approx(dev, rel=1e-9)
    occ = metrics.node_occlusion(D.x, D.y, 24.0)
    oparts = [metrics.node_occlusion_shard(D.x, D.y, 24.0, k, n_shards) for k in range(n_shards)]
    _check_cover([(p[1], p[2]) for p in oparts], L.n_nodes)
    assert sum(p[0] for p in oparts) == occ
    if n_shards <= 7:          # equal work: no shard empty while there are enough tiles
        assert all(p[3] > p[2] for p in parts)


@pytest.mark.parametrize("n_shards", [1, 3, 64])
def test_node_shards_with_two_units_per_block(torch_mod, n_shards):
    """At 40,000 nodes the default node sweep splits chunks 4 ways and takes
    two units per block: shards still cover every row once, sum to the whole
    and match the oracle's row slices."""
    from paper_2411_09809_amd import metrics
    L = gen.uniform_layout(40000, 0, extent=1 << 12, diameter=9.0, seed=23)
    D = metrics.DeviceLayout.from_host(L)
    occ = metrics.node_occlusion(D.x, D.y, 9.0)
    assert occ == oracle.node_occlusion(L.x, L.y, 9.0)
    parts = [metrics.node_occlusion_shard(D.x, D.y, 9.0, k, n_shards) for k in range(n_shards)]
    _check_cover([(p[1], p[2]) for p in parts], L.n_nodes)
    assert sum(p[0] for p in parts) == occ
    for o, q0, q1 in parts[:2] + parts[-1:]:
        assert o == oracle.node_occlusion_rows(L.x, L.y, 9.0, q0, q1)


def test_shards_match_oracle_rows(torch_mod):
    from paper_2411_09809_amd import metrics
    L = gen.uniform_layout(6000, 15000, extent=1 << 11, seed=22)
    D = metrics.DeviceLayout.from_host(L)
    for k in range(3):
        c, dev, r0, r1 = metrics.crossing_angle_shard(D.x, D.y, D.src, D.dst, k, 3, IDEAL)
        say(f"[shard-oracle] edges [{r0}, {r1})")
        rc, rdev = oracle.crossing_angle_rows(L.x, L.y, L.src, L.dst, IDEAL, r0, r1)
        assert c == rc
        assert dev == approx_dev(rdev, c, IDEAL)
        o, q0, q1 = metrics.node_occlusion_shard(D.x, D.y, 10.0, k, 3)
        assert o == oracle.node_occlusion_rows(L.x, L.y, 10.0, q0, q1)


def test_shard_argument_errors(torch_mod):
    from paper_2411_09809_amd import metrics
    from paper_2411_09809_amd._lib import RBError
    L = gen.uniform_layout(100, 200, seed=1)
    D = metrics.DeviceLayout.from_host(L)
    for k, n in ((0, 0), (-1, 2), (2, 2)):
        with pytest.raises(RBError):
            metrics.crossing_angle_shard(D.x, D.y, D.src, D.dst, k, n)
        with pytest.raises(RBError):
            metrics.node_occlusion_shard(D.x, D.y, 4.0, k, n)


@pytest.fixture(scope="module")
def powerlaw(torch_mod):
    from paper_2411_09809_amd import metrics
    L = gen.powerlaw_layout(seed=0)
    say(f"[powerlaw] V={L.n_nodes} E={L.n_edges} digest={L.digest()}")
    return L, metrics.DeviceLayout.from_host(L)


def test_powerlaw_shards_match_oracle_rows(powerlaw):
    from paper_2411_09809_amd import metrics
    L, D = powerlaw
    n = 4096
    for k in (0, n - 1):
        c, dev, r0, r1 = metrics.crossing_angle_shard(D.x, D.y, D.src, D.dst, k, n, IDEAL)
        say(f"[powerlaw] crossing shard {k}/{n}: edges [{r0}, {r1}) count {c}")
        assert r1 > r0
        rc, rdev = oracle.crossing_angle_rows(L.x, L.y, L.src, L.dst, IDEAL, r0, r1)
        assert c == rc
        assert dev == approx_dev(rdev, c, IDEAL)
        o, q0, q1 = metrics.node_occlusion_shard(D.x, D.y, L.diameter, k, n)
        say(f"[powerlaw] occlusion shard {k}/{n}: nodes [{q0}, {q1}) count {o}")
        assert o == oracle.node_occlusion_rows(L.x, L.y, L.diameter, q0, q1)


def test_powerlaw_whole_invariants(powerlaw, torch_mod):
    torch = torch_mod
    from paper_2411_09809_amd import metrics
    from paper_2411_09809_amd._lib import lib
    L, D = powerlaw
    eca, cnt, dev = metrics.crossing_angle(D.x, D.y, D.src, D.dst, IDEAL)
    occ = metrics.node_occlusion(D.x, D.y, L.diameter)
    say(f"[powerlaw] E_c={cnt} E_ca={eca:.12f} N_c={occ}")
    assert cnt > 0 and 0.0 < eca < 1.0
    # 90-degree rotation (x, y) -> (-y, x): exact on integers, metrics invariant
    xr, yr = (-D.y).contiguous(), D.x.clone()
    eca_r, cnt_r, dev_r = metrics.crossing_angle(xr, yr, D.src, D.dst, IDEAL)
    assert cnt_r == cnt and dev_r == pytest.approx(dev, rel=1e-9)
    assert metrics.node_occlusion(xr, yr, L.diameter) == occ
    # one shard of one sweeps the records in input order, the whole call in
    # hub order (3M edges): the same pairs, so the same count and angle terms
    c1, dev1, r0, r1 = metrics.crossing_angle_shard(D.x, D.y, D.src, D.dst, 0, 1, IDEAL)
    say(f"[powerlaw] input order: E_c={c1} rows [{r0}, {r1})")
    assert (c1, r0, r1) == (cnt, 0, L.n_edges) and dev1 == pytest.approx(dev, rel=1e-9)
    # a different sweep variant (other rows per thread, other tiles)
    import ctypes as C
    import os
    import tempfile
    rows, waves = C.c_int(), C.c_int()
    assert lib().rb_tune_query(1, 0, L.n_edges, C.byref(rows), C.byref(waves), None) == 0
    with tempfile.TemporaryDirectory() as tmp:
        saved = os.path.join(tmp, "tune.txt").encode()
        assert lib().rb_tune_save(saved) == 0
        assert lib().rb_tune_set(1, 0, L.n_edges, 0 if rows.value != 1 else 3) == 0
        try:
            r2, w2 = C.c_int(), C.c_int()
            lib().rb_tune_query(1, 0, L.n_edges, C.byref(r2), C.byref(w2), None)
            assert (r2.value, w2.value) != (rows.value, waves.value)
            say(f"[powerlaw] variant rows={r2.value} waves={w2.value}")
            eca_v, cnt_v, dev_v = metrics.crossing_angle(D.x, D.y, D.src, D.dst, IDEAL)
        finally:
            assert lib().rb_tune_load(saved) == 0
    assert cnt_v == cnt and dev_v == pytest.approx(dev, rel=1e-9)
    torch.cuda.synchronize()


def test_powerlaw_small_metrics_match_oracle(powerlaw):
    from paper_2411_09809_amd import metrics
    L, D = powerlaw
    ma, sdv, used = metrics.min_angle(D.x, D.y, D.src, D.dst)
    rma, rsdv, rused = oracle.min_angle(L.x, L.y, L.src, L.dst)
    assert used == rused
    assert ma == pytest.approx(rma, rel=1e-9) and sdv == pytest.approx(rsdv, rel=1e-9)
    ml, mu = metrics.edge_length_variation(D.x, D.y, D.src, D.dst)
    rml, rmu = oracle.edge_length_variation(L.x, L.y, L.src, L.dst)
    assert ml == pytest.approx(rml, rel=1e-9) and mu == pytest.approx(rmu, rel=1e-12)


def test_powerlaw_whole_equals_the_stored_oracle(powerlaw):
    """The full 1M-node / 3M-edge result against the oracle's, computed once
    by tests/golden/make_golden.py in row slices (oracle only; the input
    digest is checked): E_c, the proper crossings and N_c bit for bit,
    E_ca, the deviation sum, M_a and M_l to 1e-5 relative (Algorithms 1-5)."""
    import json
    import os
    from paper_2411_09809_amd import metrics
    L, D = powerlaw
    with open(os.path.join(os.path.dirname(__file__), "golden", "workloads.json")) as fh:
        want = json.load(fh)["powerlaw_V1000000_s0"]
    assert want["digest"] == L.digest()
    assert want["slices"] == {"crossing": 480, "occlusion": 40}
    eca, cnt, dev = metrics.crossing_angle(D.x, D.y, D.src, D.dst, IDEAL)
    c, p = metrics.edge_crossing(D.x, D.y, D.src, D.dst)
    occ = metrics.node_occlusion(D.x, D.y, L.diameter)
    say(f"[powerlaw] E_c={cnt} (oracle {want['edge_crossing']}) proper={p} "
        f"(oracle {want['proper_crossing']}) N_c={occ} (oracle {want['node_occlusion']})")
    assert cnt == c == want["edge_crossing"]
    assert p == want["proper_crossing"]
    assert occ == want["node_occlusion"]
    assert metrics.node_occlusion_grid(D.x, D.y, L.diameter) == want["node_occlusion"]
    assert eca == pytest.approx(want["crossing_angle"], rel=1e-5)
    assert dev == pytest.approx(want["crossing_dev_sum"], rel=1e-5)
    ma, sdv, used = metrics.min_angle(D.x, D.y, D.src, D.dst)
    assert used == want["min_angle_n_used"]
    assert ma == pytest.approx(want["min_angle"], rel=1e-5)
    ml, mu = metrics.edge_length_variation(D.x, D.y, D.src, D.dst)
    assert ml == pytest.approx(want["edge_length_variation"], rel=1e-5)
