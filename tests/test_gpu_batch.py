"""Batched evaluation (rb_batch_*), hipGraph replay and sweep variants.

* every layout of a batch matches the oracle (all 512 layouts of the batched
  workload through stored oracle values) and the single-layout calls:
  counts bit for bit, floats to 1e-5 against the oracle, 1e-12 against the
  single calls;
* graph replays match the eager evaluation, with eager work in between;
* every sweep variant (tile shape) gives identical results.
"""
import math
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


def mixed_layouts(seed=0):
    """Uneven sizes with edge cases: empty edge set, one node, crowded grids."""
    rng = np.random.default_rng(seed)
    out = [gen.uniform_layout(2, 1, extent=4, seed=1), gen.uniform_layout(1, 0, seed=2)]
    out[-1].diameter = 3.0
    for k in range(14):
        V = int(rng.integers(3, 1500))
        E = int(min(V * (V - 1) // 2, rng.integers(1, 4 * V)))
        ext = int(rng.choice([8, 64, 4096, 1 << 16]))
        out.append(gen.uniform_layout(V, E, extent=ext, diameter=float(rng.choice([2.5, 8, 40])),
                                      seed=100 + k))
    out.append(gen._finish(np.arange(5), np.zeros(5), np.zeros(0), np.zeros(0), diameter=1.5,
                           name="no_edges"))
    out.append(gen.complete_convex(12))
    out.append(gen.grid(7, 9))
    return out


def single_results(torch, B):
    from paper_2411_09809_amd import metrics
    res = []
    for i in range(B.n):
        x, y, s, d, diam = B.layout_views(i)
        occ = metrics.node_occlusion(x, y, diam)
        eca, cnt, _ = metrics.crossing_angle(x, y, s, d)
        ma = metrics.min_angle(x, y, s, d)[0]
        ml = metrics.edge_length_variation(x, y, s, d)[0]
        res.append((occ, cnt, eca, ma, ml))
    return res


def check_against_single(R, single):
    for i, (occ, cnt, eca, ma, ml) in enumerate(single):
        assert R["node_occlusion"][i] == occ, i
        assert R["edge_crossing"][i] == cnt, i
        assert R["crossing_angle"][i] == pytest.approx(eca, rel=1e-12, abs=1e-14), i
        assert R["min_angle"][i] == pytest.approx(ma, rel=1e-12, abs=1e-14), i
        assert R["edge_length_variation"][i] == pytest.approx(ml, rel=1e-12, abs=1e-14), i


def check_against_oracle(R, layouts, idx):
    for i in idx:
        L = layouts[i]
        want = oracle.all_metrics(L)
        assert R["node_occlusion"][i] == want["node_occlusion"], i
        assert R["edge_crossing"][i] == want["edge_crossing"], i
        for k in ("crossing_angle", "min_angle", "edge_length_variation"):
            assert abs(R[k][i] - want[k]) <= 1e-5 * abs(want[k]) + 1e-12, (i, k, R[k][i], want[k])


def test_mixed_batch_matches_oracle_and_single(torch_mod):
    from paper_2411_09809_amd.batch import Batch
    layouts = mixed_layouts()
    say(f"[batch] mixed {len(layouts)} layouts")
    B = Batch(layouts)
    B.evaluate()
    R = B.results()
    check_against_oracle(R, layouts, range(len(layouts)))
    check_against_single(R, single_results(torch_mod, B))


def test_graph_replay_matches_eager(torch_mod):
    from paper_2411_09809_amd import metrics
    from paper_2411_09809_amd.batch import Batch
    layouts = mixed_layouts(seed=3)
    say("[batch] graph replay")
    B = Batch(layouts)
    B.evaluate()
    eager = B.results()
    B.capture()
    for rep in range(3):
        for t in (B.out_occlusion, B.out_crossings, B.out_crossing_angle, B.out_min_angle,
                  B.out_elv):
            t.fill_(-7)
        # eager work on the same stream and workspace tables between replays
        x, y, s, d, diam = B.layout_views(5)
        metrics.crossing_angle(x, y, s, d)
        B.replay()
        torch_mod.cuda.synchronize()
        R = B.results()
        for k in eager:
            np.testing.assert_array_equal(R[k], eager[k], err_msg=f"replay {rep} {k}")
    B.release_graph()


def test_graph_is_refused_after_the_plan_is_uploaded_again(torch_mod):
    """A re-upload (here directly through the C ABI, as rb_batch_autotune
    also does) may rewrite the unit tables for another sweep variant; the
    graph captured before must not replay over them."""
    from paper_2411_09809_amd import _lib
    from paper_2411_09809_amd.batch import Batch
    layouts = mixed_layouts(seed=4)
    B = Batch(layouts)
    B.evaluate()
    eager = B.results()
    B.capture()
    B.replay()
    torch_mod.cuda.synchronize()
    B._upload()
    with pytest.raises(_lib.RBError) as err:
        B.replay()
    assert err.value.status == _lib.RB_EINVAL and "capture a new graph" in str(err.value)
    B.capture()
    for t in (B.out_occlusion, B.out_crossings):
        t.fill_(-7)
    B.replay()
    torch_mod.cuda.synchronize()
    R = B.results()
    for k in eager:
        np.testing.assert_array_equal(R[k], eager[k], err_msg=k)
    B.release_graph()


def test_batch_of_512_uneven_layouts(torch_mod):
    """The 512-layout workload (|V| log-uniform in [200, 20000], |E| =
    U[1.5,4]|V|, coords in [0,2^16)^2): every layout against the oracle's
    stored values (tests/golden/batch512_s0.json, written by
    tests/golden/make_golden.py from the oracle alone; each layout's input
    digest is checked first) and against the single-layout calls."""
    import json
    import os
    from paper_2411_09809_amd.batch import Batch
    layouts = gen.batch_layouts(512, seed=0)
    with open(os.path.join(os.path.dirname(__file__), "golden", "batch512_s0.json")) as fh:
        want = json.load(fh)
    assert [L.digest() for L in layouts] == want["digest"]
    say(f"[batch] 512 layouts, {sum(L.n_edges for L in layouts)} edges")
    B = Batch(layouts)
    B.evaluate()
    R = B.results()
    np.testing.assert_array_equal(R["node_occlusion"], np.array(want["node_occlusion"]))
    np.testing.assert_array_equal(R["edge_crossing"], np.array(want["edge_crossing"]))
    for k in ("crossing_angle", "min_angle", "edge_length_variation"):
        ref = np.array(want[k])
        err = np.abs(np.asarray(R[k]) - ref)
        assert (err <= 1e-5 * np.abs(ref) + 1e-12).all(), (k, int(np.argmax(err)), err.max())
    say(f"[batch] 512 layouts equal the oracle: {int(np.sum(want['edge_crossing']))} crossings, "
        f"{int(np.sum(want['node_occlusion']))} occlusions")
    check_against_single(R, single_results(torch_mod, B))


def test_batch_autotune_keeps_results(torch_mod):
    from paper_2411_09809_amd.batch import Batch
    layouts = mixed_layouts(seed=5)
    B = Batch(layouts)
    B.evaluate()
    before = B.results()
    ms = B.autotune(repeats=1)
    assert ms > 0
    B.evaluate()
    after = B.results()
    for k in before:
        if k in ("node_occlusion", "edge_crossing"):
            np.testing.assert_array_equal(after[k], before[k])
        else:
            np.testing.assert_allclose(after[k], before[k], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_every_sweep_variant_agrees(torch_mod, kind):
    """All tile shapes give identical counts (and angle sums to rounding)."""
    import ctypes as C
    from paper_2411_09809_amd import _lib, metrics
    L = gen.uniform_layout(3000, 7000, extent=300, diameter=6.0, seed=9)
    D = metrics.DeviceLayout.from_host(L)
    n_items = L.n_nodes if kind == 2 else L.n_edges
    lib = _lib.lib()
    rows, waves = C.c_int(), C.c_int()
    _lib.check(lib.rb_tune_query(kind, 0, n_items, C.byref(rows), C.byref(waves), None), "query")
    default = None
    for v in range(12 if kind == 2 else 4):
        _lib.check(lib.rb_tune_set(kind, 0, n_items, v), "rb_tune_set")
        say(f"[variant] kind {kind} variant {v}")
        if kind == 0:
            r = metrics.edge_crossing(D.x, D.y, D.src, D.dst)
        elif kind == 1:
            r = metrics.crossing_angle(D.x, D.y, D.src, D.dst)
        else:
            r = metrics.node_occlusion(D.x, D.y, L.diameter)
        if default is None:
            default = r
        elif kind == 1:
            assert r[1] == default[1] and r[0] == pytest.approx(default[0], rel=1e-12)
        else:
            assert r == default
    want = oracle.all_metrics(L)
    if kind == 0:
        assert default == (want["edge_crossing"], want["proper_crossing"])
    elif kind == 1:
        assert default[1] == want["edge_crossing"]
    else:
        assert default == want["node_occlusion"]


def test_autotune_single_layout(torch_mod):
    import ctypes as C
    from paper_2411_09809_amd import _lib, metrics
    L = gen.uniform_layout(5000, 12000, extent=1 << 14, diameter=20.0, seed=4)
    D = metrics.DeviceLayout.from_host(L)
    before = metrics.evaluate(D)
    ws = metrics.workspace(L.n_nodes, L.n_edges, D.x.device)
    w, wb = metrics._ws_args(ws)
    ms = C.c_double()
    _lib.check(_lib.lib().rb_autotune(D.x.data_ptr(), D.y.data_ptr(), L.n_nodes, D.src.data_ptr(),
                                      D.dst.data_ptr(), L.n_edges, L.diameter, IDEAL, 2,
                                      C.byref(ms), w, wb, metrics._stream(D.x.device)),
               "rb_autotune")
    assert ms.value > 0
    after = metrics.evaluate(D)
    for k in ("node_occlusion", "edge_crossing", "min_angle_n_used"):
        assert after[k] == before[k]
    assert after["crossing_angle"] == pytest.approx(before["crossing_angle"], rel=1e-12)


@pytest.mark.parametrize("d", [0.0, 1.0, 6.0])
def test_every_node_sweep_variant_on_ragged_sizes(torch_mod, d, tmp_path):
    """Every node-sweep variant, single-layout and batched, on sizes around
    its row tiles (256 K nodes) and column chunks (256, 64 or 32 nodes).  The
    sweep counts a tile's own square as ordered pairs less its self pairs and
    halves the total: that must hold with padding rows and columns, at
    diameter 0 (no pair occludes, not even a node with itself), at 1 (only
    coincident nodes) and at 6 on a crowded 40 x 40 canvas (Algorithm 1).
    From 2^15 nodes the split variants of a single layout take two units per
    block (32768 and 40961 nodes)."""
    from paper_2411_09809_amd import _lib, metrics
    from paper_2411_09809_amd.batch import Batch
    lib = _lib.lib()
    sizes = [1, 2, 3, 31, 255, 256, 257, 1023, 1025, 2049, 4100, 32768, 40961]
    layouts = [gen.uniform_layout(n, 0, extent=40, diameter=d, seed=n) for n in sizes]
    want = [oracle.node_occlusion(L.x, L.y, d) for L in layouts]
    devs = [metrics.DeviceLayout.from_host(L) for L in layouts]
    mean_v = max(1, sum(sizes) // len(sizes))
    try:
        for v in range(12):
            say(f"[node variants] d={d} variant {v}")
            for L, D, w in zip(layouts, devs, want):
                _lib.check(lib.rb_tune_set(2, 0, L.n_nodes, v), "rb_tune_set")
                assert metrics.node_occlusion(D.x, D.y, d) == w, (v, L.n_nodes)
            _lib.check(lib.rb_tune_set(2, 1, mean_v, v), "rb_tune_set")
            B = Batch(layouts)
            B.evaluate()
            assert list(B.results()["node_occlusion"]) == want, v
    finally:
        empty = tmp_path / "tune.txt"
        empty.write_text("")
        _lib.check(lib.rb_tune_load(str(empty).encode()), "rb_tune_load")   # built-in defaults


@pytest.mark.parametrize("E", [769, 4095, 4096, 8192])
def test_every_variant_at_record_segment_ends(torch_mod, E, tmp_path):
    """A row tile of 3 rows per thread (768 edges) does not divide the
    4096-record segment of a layout: the last tile's rows past the segment
    must be padding, in single-layout, pruned and batched sweeps alike."""
    from paper_2411_09809_amd import _lib, metrics
    from paper_2411_09809_amd.batch import Batch
    lib = _lib.lib()
    layouts = [gen.uniform_layout(max(200, E // 3), E, extent=2000, seed=E + k) for k in range(3)]
    want = [oracle.crossing_angle(L.x, L.y, L.src, L.dst, IDEAL) for L in layouts]
    D = metrics.DeviceLayout.from_host(layouts[0])
    try:
        for v in range(4):
            say(f"[segment-end] E={E} variant {v}")
            for kind in (1, 3):
                _lib.check(lib.rb_tune_set(kind, 0, E, v), "rb_tune_set")
            r = metrics.crossing_angle(D.x, D.y, D.src, D.dst, IDEAL)
            p = metrics.crossing_angle_pruned(D.x, D.y, D.src, D.dst, IDEAL)
            for got in (r, p):
                assert got[1] == want[0][1]
                assert got[0] == approx_eca(want[0][0], IDEAL)
            if v == 3:          # the 4-row sweep is not offered for batches
                assert lib.rb_tune_set(1, 1, E, v) == _lib.RB_EINVAL
                continue
            _lib.check(lib.rb_tune_set(1, 1, E, v), "rb_tune_set")
            B = Batch(layouts)
            B.evaluate()
            R = B.results()
            for i in range(3):
                assert R["edge_crossing"][i] == want[i][1], (v, i)
                assert R["crossing_angle"][i] == approx_eca(want[i][0], IDEAL)
    finally:
        empty = tmp_path / "tune.txt"
        empty.write_text("")
        _lib.check(lib.rb_tune_load(str(empty).encode()), "rb_tune_load")   # built-in defaults
