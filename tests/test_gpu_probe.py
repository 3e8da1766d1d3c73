"""The FP64 FMA probe used as the attainable VALU ceiling: a positive rate
no higher than the nominal issue peak (256 CUs x 64 lanes x 2.4 GHz), and
an error for arguments out of range."""
import ctypes as C

import pytest

from paper_2411_09809_amd import _lib

pytestmark = pytest.mark.gpu
NOMINAL = 256 * 64 * 2.4e9


def test_probe_rate_is_below_the_nominal_peak():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    R = _lib.lib()
    sink = torch.zeros(1, dtype=torch.float64, device="cuda")
    rate = C.c_double()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(R.rb_valu_probe(512, 3, C.byref(rate), C.c_void_p(sink.data_ptr()), stream), "probe")
    print("fp64 fma lane-ops/s", rate.value, rate.value / NOMINAL, flush=True)
    assert 0.2 * NOMINAL < rate.value <= 1.02 * NOMINAL
    assert float(sink.item()) == 0.0
    for iters, reps in ((0, 1), (1 << 25, 1), (4, 0), (4, 1001)):
        assert R.rb_valu_probe(iters, reps, C.byref(rate), C.c_void_p(sink.data_ptr()), stream) != 0


def test_timing_records_the_fused_adjoint_sweep():
    """rb_timing kind 4 holds one event pair per rb_loss_grad call (the fused
    forward + adjoint sweep only), and none for the plain crossing sweep."""
    import torch
    from paper_2411_09809_amd import gen, metrics, optim
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    R = _lib.lib()
    L = gen.uniform_layout(seed=0)
    D = metrics.DeviceLayout.from_host(L)
    optim.loss_grad(D.x, D.y, D.src, D.dst)
    torch.cuda.synchronize()
    R.rb_timing_reset()
    R.rb_timing_enable(1)
    try:
        for _ in range(3):
            optim.loss_grad(D.x, D.y, D.src, D.dst)
        metrics.crossing_angle(D.x, D.y, D.src, D.dst)
        torch.cuda.synchronize()
    finally:
        R.rb_timing_enable(0)
    ms, n = C.c_double(), C.c_int64()
    _lib.check(R.rb_timing_read(4, C.byref(ms), C.byref(n)), "timing")
    assert n.value == 3 and ms.value > 0.0
    _lib.check(R.rb_timing_read(0, C.byref(ms), C.byref(n)), "timing")
    assert n.value == 1
    R.rb_timing_reset()
