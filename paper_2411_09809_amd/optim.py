"""Layout optimisation with the readability loss (rb_loss_grad of rb.h).

``CrossingAngleLengthLoss`` is a ``torch.autograd.Function`` for
    L = w_angle (1 - E_ca) + w_length M_l + w_min_angle (1 - M_a)
(crossing set frozen at the evaluated layout): its forward and backward are
both computed by librb's kernels in one call.  ``descend`` runs gradient
descent on a float32 master copy of the coordinates, evaluating loss,
gradient and the exact crossing count on the rounded (integer) layout at
every step.
"""
from __future__ import annotations

import torch

from ._lib import check, lib
from .metrics import (IDEAL_ANGLE, _check_coords, _check_edges, _stream, _ws_args, grid_workspace,
                      workspace)


def loss_grad(x, y, src, dst, ideal_angle: float = IDEAL_ANGLE, w_angle: float = 1.0,
              w_length: float = 1.0, pruned: bool = False, w_min_angle: float = 0.0):
    """(loss, dL/dx, dL/dy, crossing count) as device tensors (float64,
    float64[V], float64[V], int64).  ``pruned`` uses rb_loss_grad_pruned,
    which skips the tiles of edges whose bounding boxes cannot meet;
    ``w_min_angle`` weighs the minimum-angle term 1 - M_a (0 skips it)."""
    _check_coords(x, y)
    _check_edges(x, src, dst)
    dev = x.device
    n = x.numel()
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    gx = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    gy = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = (grid_workspace if pruned else workspace)(n, src.numel(), dev)
    w, wb = _ws_args(ws)
    fn, name = ((lib().rb_loss_grad_pruned, "rb_loss_grad_pruned") if pruned
                else (lib().rb_loss_grad, "rb_loss_grad"))
    check(fn(x.data_ptr(), y.data_ptr(), n, src.data_ptr(), dst.data_ptr(), src.numel(),
             float(ideal_angle), float(w_angle), float(w_length), float(w_min_angle),
             loss.data_ptr(), gx.data_ptr(), gy.data_ptr(), cnt.data_ptr(), w, wb, _stream(dev)),
          name)
    return loss[0], gx[:n], gy[:n], cnt[0]


class CrossingAngleLengthLoss(torch.autograd.Function):
    """L(x, y) = w_angle (1 - E_ca) + w_length M_l + w_min_angle (1 - M_a) on
    integer-valued float32 coordinates; gradients come back in the
    coordinates' dtype."""

    @staticmethod
    def forward(ctx, x, y, src, dst, ideal_angle=IDEAL_ANGLE, w_angle=1.0, w_length=1.0,
                pruned=False, w_min_angle=0.0):
        loss, gx, gy, cnt = loss_grad(x, y, src, dst, ideal_angle, w_angle, w_length, pruned,
                                      w_min_angle)
        ctx.save_for_backward(gx, gy)
        ctx.dtype = x.dtype
        ctx.mark_non_differentiable(cnt)
        return loss, cnt

    @staticmethod
    def backward(ctx, g_loss, g_cnt):
        gx, gy = ctx.saved_tensors
        return ((g_loss * gx).to(ctx.dtype), (g_loss * gy).to(ctx.dtype), None, None, None, None,
                None, None, None)


def descent_step(mx, my, gx, gy, step_size: float):
    """One step of ``descend`` in place: the master coordinates move by
    ``step_size`` grid units along -g / max|g|; a zero gradient (a layout at
    a stationary point, e.g. no crossings and equal edge lengths) leaves them
    where they are.  No host synchronisation."""
    if gx.numel() == 0:
        return
    scale = torch.maximum(gx.abs().max(), gy.abs().max())
    step = torch.where(scale > 0, step_size / scale, 0.0)   # 1/0 = inf is not selected
    mx -= gx * step
    my -= gy * step


def descend(x, y, src, dst, steps: int = 100, step_size: float = 2.0,
            extent: int = 1 << 16, ideal_angle: float = IDEAL_ANGLE, w_angle: float = 1.0,
            w_length: float = 1.0, log=None, pruned: bool = False, w_min_angle: float = 0.0,
            trace: list | None = None, checkpoint: str | None = None,
            checkpoint_every: int = 10, resume: str | None = None):
    """Gradient descent on the readability loss.

    A float32 master copy of the coordinates moves by ``step_size`` grid
    units along -g / max|g| each step; loss, gradient and the exact crossing
    count are evaluated on the master rounded to integers and clamped to
    [0, extent).  Returns (x, y, history) with history = list of
    (loss, crossings, seconds) per step, seconds being the step's GPU time.
    The steps are enqueued without waiting for the GPU unless ``log`` is
    given (it is called with each step's entry as soon as it is known).
    With ``trace`` (a list), each step's evaluated integer layout is appended
    to it as a pair of device tensors.

    ``checkpoint`` (a file name) saves the master coordinates and the number
    of steps taken (numpy ``.npz``) every ``checkpoint_every`` steps and after
    the last; ``resume`` starts from such a file, taking the steps that
    remain of ``steps`` (the history then covers those steps only).  A run
    cut into pieces this way ends where the uninterrupted run ends: each
    step depends only on the master coordinates."""
    import os

    import numpy as np
    mx = x.detach().clone().to(torch.float32)
    my = y.detach().clone().to(torch.float32)
    first = 0
    if resume is not None:
        with np.load(resume) as z:
            if z["mx"].shape != tuple(mx.shape):
                raise ValueError(f"{resume}: {z['mx'].shape[0]} nodes, the layout has "
                                 f"{mx.shape[0]}")
            mx.copy_(torch.from_numpy(z["mx"]))
            my.copy_(torch.from_numpy(z["my"]))
            first = int(z["step"])

    def save(done):
        tmp = checkpoint + ".tmp.npz"
        np.savez(tmp, mx=mx.cpu().numpy(), my=my.cpu().numpy(), step=np.int64(done))
        os.replace(tmp, checkpoint)

    marks = [torch.cuda.Event(enable_timing=True)]
    marks[0].record()
    vals, hist = [], []
    for k in range(first, steps):
        xi = torch.clamp(torch.round(mx), 0, extent - 1).requires_grad_(True)
        yi = torch.clamp(torch.round(my), 0, extent - 1).requires_grad_(True)
        loss, cnt = CrossingAngleLengthLoss.apply(xi, yi, src, dst, ideal_angle, w_angle,
                                                  w_length, pruned, w_min_angle)
        loss.backward()
        with torch.no_grad():
            descent_step(mx, my, xi.grad, yi.grad, step_size)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        marks.append(ev)
        vals.append((loss.detach(), cnt))
        if trace is not None:
            trace.append((xi.detach(), yi.detach()))
        if log:
            ev.synchronize()
            hist.append((float(loss), int(cnt), marks[-2].elapsed_time(ev) * 1e-3))
            log(k, hist[-1])
        if checkpoint and ((k + 1) % checkpoint_every == 0 or k + 1 == steps):
            save(k + 1)
    if not log:
        marks[-1].synchronize()
        hist = [(float(l), int(c), marks[i].elapsed_time(marks[i + 1]) * 1e-3)
                for i, (l, c) in enumerate(vals)]
    return (torch.clamp(torch.round(mx), 0, extent - 1), torch.clamp(torch.round(my), 0, extent - 1),
            hist)
