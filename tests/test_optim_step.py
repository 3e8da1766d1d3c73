"""The descent update of ``optim.descend`` on the CPU (pure torch; the loss
and gradient themselves need the GPU)."""
import pytest
import torch

from paper_2411_09809_amd import optim


def test_zero_gradient_leaves_the_layout_unchanged():
    """A stationary layout (no crossings, equal edge lengths: the straight
    grid drawing) has a zero gradient; the step must not divide 0 by 0."""
    mx = torch.tensor([0.0, 10.0, 20.0])
    my = torch.tensor([0.0, 0.0, 0.0])
    z = torch.zeros(3, dtype=torch.float64)
    optim.descent_step(mx, my, z.float(), z.float(), 2.0)
    assert torch.isfinite(mx).all() and torch.isfinite(my).all()
    assert mx.tolist() == [0.0, 10.0, 20.0] and my.tolist() == [0.0, 0.0, 0.0]
    optim.descent_step(mx[:0], my[:0], z[:0].float(), z[:0].float(), 2.0)


def test_step_moves_the_largest_component_by_step_size():
    mx = torch.tensor([5.0, 5.0])
    my = torch.tensor([5.0, 5.0])
    gx = torch.tensor([0.5, -2.0])
    gy = torch.tensor([1.0, 0.0])
    optim.descent_step(mx, my, gx, gy, 4.0)
    assert mx.tolist() == [4.0, 9.0] and my.tolist() == [3.0, 5.0]


def test_resume_from_a_file_of_another_size_is_refused(tmp_path):
    import numpy as np
    f = tmp_path / "ck.npz"
    np.savez(f, mx=np.zeros(5, np.float32), my=np.zeros(5, np.float32), step=np.int64(3))
    x = torch.zeros(7)
    e = torch.zeros(0, dtype=torch.int32)
    with pytest.raises(ValueError, match="5 nodes"):
        optim.descend(x, x, e, e, steps=4, resume=str(f))
