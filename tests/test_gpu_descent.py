"""The full-size descent workload against the oracle, step by step.

Random geometric graph, 20,000 nodes and about 60,000 edges on [0,2^16)^2,
100 steps of descent on w_a (1 - E_ca) + w_l M_l (step 2 grid units along
-g / max|g|, loss, gradient and exact crossing count evaluated on the
rounded layout each step).  The oracle evaluates the crossing count at every
one of the 100 integer layouts the GPU evaluated (counts bit for bit), and
the loss and analytic gradient at three of them (1e-5 relative; gradient
with the floor 1e-3 max|g_ref|).  Algorithms 4 and 5; the application is the
layout optimisation the paper's Conclusion names.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2411_09809_amd import gen

pytestmark = pytest.mark.gpu
IDEAL = gen.IDEAL_ANGLE
STEPS = 100


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def trajectory():
    import torch
    from paper_2411_09809_amd import metrics, optim
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    L = gen.geometric_layout(seed=0)
    say(f"[descent] rgg V={L.n_nodes} E={L.n_edges}: {STEPS} steps on the GPU")
    D = metrics.DeviceLayout.from_host(L)
    trace = []
    _, _, hist = optim.descend(D.x, D.y, D.src, D.dst, steps=STEPS, step_size=2.0, trace=trace)
    layouts = [(xi.cpu().numpy().astype(np.float64), yi.cpu().numpy().astype(np.float64))
               for xi, yi in trace]
    return L, layouts, hist


@pytest.mark.parametrize("block", range(4))
def test_every_step_count_equals_the_oracle(trajectory, block):
    L, layouts, hist = trajectory
    for k in range(block * STEPS // 4, (block + 1) * STEPS // 4):
        x, y = layouts[k]
        assert (x == np.round(x)).all() and x.min() >= 0 and x.max() < 1 << 16
        c, _ = oracle.edge_crossing(x, y, L.src, L.dst)
        assert hist[k][1] == c, (k, hist[k][1], c)
    say(f"[descent] steps {block * STEPS // 4}..{(block + 1) * STEPS // 4 - 1}: counts equal "
        f"the oracle (last {hist[k][1]})")


@pytest.mark.parametrize("k", [0, 50, STEPS - 1])
def test_loss_and_gradient_at_sampled_steps(trajectory, k):
    import torch
    from paper_2411_09809_amd import optim
    L, layouts, hist = trajectory
    x, y = layouts[k]
    S = oracle.crossing_pairs(x, y, L.src, L.dst)
    f_ref, gx_ref, gy_ref = oracle.loss_grad(x, y, L.src, L.dst, S, IDEAL, 1.0, 1.0)
    assert hist[k][0] == pytest.approx(f_ref, rel=1e-5)
    t = lambda a, dt: torch.as_tensor(a).to(device="cuda", dtype=dt).contiguous()
    f, gx, gy, cnt = optim.loss_grad(t(x, torch.float32), t(y, torch.float32),
                                     t(L.src, torch.int32), t(L.dst, torch.int32), IDEAL, 1.0, 1.0)
    assert int(cnt) == S.shape[0] and float(f) == pytest.approx(f_ref, rel=1e-5)
    cap = 1e-3 * max(np.abs(gx_ref).max(), np.abs(gy_ref).max())
    for g, ref in ((gx.cpu().numpy(), gx_ref), (gy.cpu().numpy(), gy_ref)):
        assert (np.abs(g - ref) <= 1e-5 * np.maximum(np.abs(ref), cap)).all()
    say(f"[descent] step {k}: loss {float(f):.12f} (oracle {f_ref:.12f}), |S| = {S.shape[0]}")


def test_the_loss_goes_down(trajectory):
    _, _, hist = trajectory
    assert len(hist) == STEPS
    assert min(h[0] for h in hist[1:]) < hist[0][0]


def test_checkpoint_and_resume(tmp_path):
    """A run saved after 4 steps and resumed to 7: the resumed run's first
    evaluated layout is the saved one (rounded), it takes the 3 remaining
    steps, and its exact counts are the oracle's."""
    import torch
    from paper_2411_09809_amd import metrics, optim
    L = gen.uniform_layout(600, 1500, extent=1 << 12, seed=17)
    D = metrics.DeviceLayout.from_host(L)
    f = str(tmp_path / "descent.npz")
    xa, ya, ha = optim.descend(D.x, D.y, D.src, D.dst, steps=4, step_size=4.0,
                               extent=1 << 12, checkpoint=f, checkpoint_every=2)
    z = np.load(f)
    assert int(z["step"]) == 4 and len(ha) == 4
    assert (np.clip(np.round(z["mx"]), 0, 4095) == xa.cpu().numpy()).all()
    assert (np.clip(np.round(z["my"]), 0, 4095) == ya.cpu().numpy()).all()
    trace = []
    xb, yb, hb = optim.descend(D.x, D.y, D.src, D.dst, steps=7, step_size=4.0, extent=1 << 12,
                               resume=f, trace=trace)
    assert len(hb) == 3 and len(trace) == 3
    assert torch.equal(trace[0][0], xa) and torch.equal(trace[0][1], ya)
    for (xi, yi), h in zip(trace, hb):
        c, _ = oracle.edge_crossing(xi.cpu().numpy(), yi.cpu().numpy(), L.src, L.dst)
        assert h[1] == c
