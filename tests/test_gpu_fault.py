"""Fault injection (RB_FAULT) on the GPU: a refused call leaves its outputs
untouched and the stream usable, an injected failure inside a graph capture
ends and discards the capture, and the same calls work once the variable is
unset."""
import numpy as np
import pytest

import oracle
from paper_2411_09809_amd import _lib, gen

pytestmark = pytest.mark.gpu


@pytest.fixture
def torch_mod(monkeypatch):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    monkeypatch.delenv("RB_FAULT", raising=False)
    return torch


def test_refused_launch_leaves_outputs_and_stream_intact(torch_mod, monkeypatch):
    torch = torch_mod
    from paper_2411_09809_amd import metrics
    L = gen.uniform_layout(800, 2000, extent=2048, seed=3)
    D = metrics.DeviceLayout.from_host(L)
    out = torch.full((3,), -5.0, dtype=torch.float64, device="cuda")
    ws = metrics.workspace(L.n_nodes, L.n_edges, "cuda")
    w, wb = metrics._ws_args(ws)
    p = out.data_ptr()
    args = (D.x.data_ptr(), D.y.data_ptr(), L.n_nodes, D.src.data_ptr(), D.dst.data_ptr(),
            L.n_edges, D.ideal_angle, p, p + 8, p + 16, w, wb,
            torch.cuda.current_stream().cuda_stream)
    monkeypatch.setenv("RB_FAULT", "launch")
    assert _lib.lib().rb_crossing_angle(*args) == _lib.RB_EHIP
    with pytest.raises(_lib.RBError):
        metrics.node_occlusion(D.x, D.y, 8.0)
    torch.cuda.synchronize()
    assert (out.cpu() == -5.0).all()
    monkeypatch.delenv("RB_FAULT")
    assert _lib.lib().rb_crossing_angle(*args) == _lib.RB_OK
    v = out.cpu()
    m, c, d = oracle.crossing_angle(L.x, L.y, L.src, L.dst, L.ideal_angle)
    assert int(v.view(torch.int64)[1]) == c and abs(float(v[0]) - m) <= 1e-5 * abs(m)
    assert metrics.node_occlusion(D.x, D.y, 8.0) == oracle.node_occlusion(L.x, L.y, 8.0)


def test_injected_capture_failure_then_capture(torch_mod, monkeypatch):
    torch = torch_mod
    from paper_2411_09809_amd.batch import Batch
    layouts = [gen.uniform_layout(300 + 50 * k, 700 + 100 * k, extent=1024, seed=40 + k)
               for k in range(6)]
    B = Batch(layouts)
    B.evaluate()
    eager = B.results()
    monkeypatch.setenv("RB_FAULT", "capture")
    with pytest.raises(_lib.RBError) as err:
        B.capture()
    assert err.value.status == _lib.RB_EHIP and "RB_FAULT=capture" in str(err.value)
    # the stream is not left capturing: eager work still runs
    monkeypatch.setenv("RB_FAULT", "launch")
    for t in (B.out_occlusion, B.out_crossings):
        t.fill_(-7)
    with pytest.raises(_lib.RBError):
        B.evaluate()
    torch.cuda.synchronize()
    assert (B.out_crossings.cpu() == -7).all()
    monkeypatch.delenv("RB_FAULT")
    B.evaluate()
    torch.cuda.synchronize()
    for k in eager:
        np.testing.assert_array_equal(B.results()[k], eager[k], err_msg=k)
    B.capture()
    for t in (B.out_occlusion, B.out_crossings):
        t.fill_(-7)
    B.replay()
    torch.cuda.synchronize()
    for k in eager:
        np.testing.assert_array_equal(B.results()[k], eager[k], err_msg=k)
    B.release_graph()


def test_validate_env_checks_the_layout_first(torch_mod, monkeypatch):
    """RB_VALIDATE=1: the workspace calls check the layout preconditions
    first and refuse a layout with a duplicate edge or a self-loop with
    RB_EDOMAIN; a valid layout gives the same results as without it."""
    torch = torch_mod
    from paper_2411_09809_amd import metrics
    L = gen.uniform_layout(500, 1200, extent=2048, seed=8)
    D = metrics.DeviceLayout.from_host(L)
    want = metrics.crossing_angle(D.x, D.y, D.src, D.dst)
    dup_src = torch.cat([D.src, D.dst[:1]]).contiguous()      # edge 0 again, reversed
    dup_dst = torch.cat([D.dst, D.src[:1]]).contiguous()
    loop_src = torch.cat([D.src, D.src[:1]]).contiguous()     # a self-loop
    monkeypatch.setenv("RB_VALIDATE", "1")
    assert metrics.crossing_angle(D.x, D.y, D.src, D.dst) == want
    assert metrics.node_occlusion(D.x, D.y, 8.0) == oracle.node_occlusion(L.x, L.y, 8.0)
    for s, d, text in ((dup_src, dup_dst, "duplicate edge"), (loop_src, dup_src, "self-loop")):
        with pytest.raises(_lib.RBError) as err:
            metrics.crossing_angle(D.x, D.y, s, d)
        assert err.value.status == _lib.RB_EDOMAIN and text in str(err.value)
        with pytest.raises(_lib.RBError):
            metrics.min_angle(D.x, D.y, s, d)
    xf = D.x.clone()
    xf[3] = 0.5                                               # not an integer
    with pytest.raises(_lib.RBError) as err:
        metrics.node_occlusion(xf, D.y, 8.0)
    assert "non-integer" in str(err.value)
    monkeypatch.setenv("RB_VALIDATE", "0")                    # off: no check, no error
    metrics.crossing_angle(D.x, D.y, dup_src, dup_dst)
