"""Python entry points with the names of the C-ABI (include/rb.h).

Each function takes a layout as torch tensors on one AMD GPU -- ``x``, ``y``
float32 (integer-valued, |c| <= 2^20) and ``src``, ``dst`` int32 -- enqueues
the HIP kernels of librb on the current stream and returns Python numbers
(which waits for the stream), or device tensors with ``async_=True``.
PyTorch only provides device memory and the stream; all metric arithmetic
runs in librb's kernels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from ._lib import check, lib

IDEAL_ANGLE = 70.0 * math.pi / 180.0

# Workspaces are cached per (device, stream): calls enqueued on different
# streams may run at the same time and must not share scratch memory.
_ws_cache: dict[tuple, torch.Tensor] = {}


_WS_KEEP = 8       # cached workspaces per kind; the oldest goes first


def _ws_key(dev: torch.device) -> tuple:
    index = dev.index if dev.index is not None else torch.cuda.current_device()
    return index, torch.cuda.current_stream(torch.device("cuda", index)).cuda_stream


def _ws_get(cache: dict, key: tuple, need: int, dev: torch.device) -> torch.Tensor:
    # a workspace belongs to the memory pool of the stream it was made on, so
    # dropping one never hands its memory to work queued on another stream
    ws = cache.pop(key, None)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    cache[key] = ws                     # most recently used last
    while len(cache) > _WS_KEEP:
        cache.pop(next(iter(cache)))
    return ws


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def workspace(n_nodes: int, n_edges: int, device) -> torch.Tensor:
    """A cached device workspace large enough for this layout size."""
    need = int(lib().rb_workspace_size(int(n_nodes), int(n_edges)))
    if need == 0:
        raise ValueError(f"layout size out of range: {n_nodes} nodes, {n_edges} edges")
    dev = torch.device(device)
    return _ws_get(_ws_cache, _ws_key(dev), need, dev)


_grid_ws_cache: dict[tuple, torch.Tensor] = {}


def grid_workspace(n_nodes: int, n_edges: int, device) -> torch.Tensor:
    """A cached device workspace for the grid-pruned calls."""
    need = int(lib().rb_grid_workspace_size(int(n_nodes), int(n_edges)))
    if need == 0:
        raise ValueError(f"layout size out of range: {n_nodes} nodes, {n_edges} edges")
    dev = torch.device(device)
    return _ws_get(_grid_ws_cache, _ws_key(dev), need, dev)


def _ws_args(ws: torch.Tensor):
    p = ws.data_ptr()
    aligned = (p + 255) & ~255
    return aligned, ws.numel() - (aligned - p)


def _check_coords(x, y):
    for name, t in (("x", x), ("y", y)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
                and t.dim() == 1 and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous 1-D float32 GPU tensor")
    if x.shape != y.shape or x.device != y.device:
        raise ValueError("x and y must have the same shape and device")


def _check_edges(x, src, dst):
    for name, t in (("src", src), ("dst", dst)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32
                and t.dim() == 1 and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous 1-D int32 GPU tensor")
    if src.shape != dst.shape or src.device != x.device or dst.device != x.device:
        raise ValueError("src and dst must have the same shape and the device of x")


def _out(n, dtype, dev):
    return torch.zeros(n, dtype=dtype, device=dev)


def node_occlusion(x, y, diameter: float, *, async_: bool = False):
    """N_c: node pairs closer than ``diameter`` (Algorithm 1)."""
    _check_coords(x, y)
    out = _out(1, torch.int64, x.device)
    ws = workspace(x.numel(), 0, x.device)
    w, wb = _ws_args(ws)
    check(lib().rb_node_occlusion(_ptr(x), _ptr(y), x.numel(), float(diameter), _ptr(out), w, wb,
                                  _stream(x.device)), "rb_node_occlusion")
    return out if async_ else int(out.item())


def edge_crossing(x, y, src, dst, *, async_: bool = False):
    """(E_c, proper crossings) (Algorithm 4)."""
    _check_coords(x, y)
    _check_edges(x, src, dst)
    out = _out(2, torch.int64, x.device)
    ws = workspace(x.numel(), src.numel(), x.device)
    w, wb = _ws_args(ws)
    check(lib().rb_edge_crossing(_ptr(x), _ptr(y), x.numel(), _ptr(src), _ptr(dst), src.numel(),
                                 _ptr(out), _ptr(out) + 8, w, wb, _stream(x.device)),
          "rb_edge_crossing")
    if async_:
        return out
    c, p = out.tolist()
    return int(c), int(p)


def crossing_angle(x, y, src, dst, ideal_angle: float = IDEAL_ANGLE, *, async_: bool = False):
    """(E_ca, E_c, sum of |ideal - a|/ideal) (Algorithm 5)."""
    _check_coords(x, y)
    _check_edges(x, src, dst)
    out = _out(3, torch.float64, x.device)        # metric, count (int64 bits), dev sum
    ws = workspace(x.numel(), src.numel(), x.device)
    w, wb = _ws_args(ws)
    p = _ptr(out)
    check(lib().rb_crossing_angle(_ptr(x), _ptr(y), x.numel(), _ptr(src), _ptr(dst), src.numel(),
                                  float(ideal_angle), p, p + 8, p + 16, w, wb, _stream(x.device)),
          "rb_crossing_angle")
    if async_:
        return out
    vals = out.cpu()
    return float(vals[0]), int(vals.view(torch.int64)[1]), float(vals[2])


def crossing_angle_noalloc(x, y, src, dst, ideal_angle: float = IDEAL_ANGLE, *, out=None,
                           async_: bool = False):
    """``crossing_angle`` through the entry point that uses the library's
    static device scratch instead of a workspace (at most 1,000,000 edges).
    ``out`` (float64[3] on the layout's device) may be given so that the
    call allocates nothing; calls overlapping on one device race."""
    _check_coords(x, y)
    _check_edges(x, src, dst)
    if out is None:
        out = _out(3, torch.float64, x.device)
    elif not (out.dtype == torch.float64 and out.numel() >= 3 and out.device == x.device
              and out.is_contiguous()):
        raise ValueError("out must be a contiguous float64 tensor of 3 entries on x's device")
    p = _ptr(out)
    check(lib().rb_crossing_angle_noalloc(_ptr(x), _ptr(y), x.numel(), _ptr(src), _ptr(dst),
                                          src.numel(), float(ideal_angle), p, p + 8, p + 16,
                                          _stream(x.device)), "rb_crossing_angle_noalloc")
    if async_:
        return out
    vals = out.cpu()
    return float(vals[0]), int(vals.view(torch.int64)[1]), float(vals[2])


def min_angle(x, y, src, dst, *, async_: bool = False):
    """(M_a, sum of d_v, nodes of degree >= 1) (Algorithm 2)."""
    _check_coords(x, y)
    _check_edges(x, src, dst)
    out = _out(3, torch.float64, x.device)
    ws = workspace(x.numel(), src.numel(), x.device)
    w, wb = _ws_args(ws)
    p = _ptr(out)
    check(lib().rb_min_angle(_ptr(x), _ptr(y), x.numel(), _ptr(src), _ptr(dst), src.numel(),
                             p, p + 8, p + 16, w, wb, _stream(x.device)), "rb_min_angle")
    if async_:
        return out
    vals = out.cpu()
    return float(vals[0]), float(vals[1]), int(vals.view(torch.int64)[2])


def edge_length_variation(x, y, src, dst, *, async_: bool = False):
    """(M_l, mean edge length) (Algorithm 3)."""
    _check_coords(x, y)
    _check_edges(x, src, dst)
    out = _out(2, torch.float64, x.device)
    ws = workspace(x.numel(), src.numel(), x.device)
    w, wb = _ws_args(ws)
    p = _ptr(out)
    check(lib().rb_edge_length_variation(_ptr(x), _ptr(y), x.numel(), _ptr(src), _ptr(dst),
                                         src.numel(), p, p + 8, w, wb, _stream(x.device)),
          "rb_edge_length_variation")
    if async_:
        return out
    m, mu = out.tolist()
    return float(m), float(mu)


def node_occlusion_grid(x, y, diameter: float, *, async_: bool = False):
    """N_c by the grid method (Section 3.2.1): the brute-force count, with
    only pairs in the same or neighbouring cells tested."""
    _check_coords(x, y)
    out = _out(1, torch.int64, x.device)
    ws = grid_workspace(x.numel(), 0, x.device)
    w, wb = _ws_args(ws)
    check(lib().rb_node_occlusion_grid(_ptr(x), _ptr(y), x.numel(), float(diameter), _ptr(out), w,
                                       wb, _stream(x.device)), "rb_node_occlusion_grid")
    return out if async_ else int(out.item())


def crossing_angle_pruned(x, y, src, dst, ideal_angle: float = IDEAL_ANGLE, *,
                          async_: bool = False):
    """(E_ca, E_c, sum of |ideal - a|/ideal) as ``crossing_angle``, skipping
    tiles of edges whose bounding boxes cannot meet."""
    _check_coords(x, y)
    _check_edges(x, src, dst)
    out = _out(3, torch.float64, x.device)
    ws = grid_workspace(x.numel(), src.numel(), x.device)
    w, wb = _ws_args(ws)
    p = _ptr(out)
    check(lib().rb_crossing_angle_pruned(_ptr(x), _ptr(y), x.numel(), _ptr(src), _ptr(dst),
                                         src.numel(), float(ideal_angle), p, p + 8, p + 16, w,
                                         wb, _stream(x.device)), "rb_crossing_angle_pruned")
    if async_:
        return out
    vals = out.cpu()
    return float(vals[0]), int(vals.view(torch.int64)[1]), float(vals[2])


_strip_ws: dict[int, torch.Tensor] = {}


def enhanced_crossing(x, y, src, dst, width: int, horizontal: bool = False,
                      ideal_angle: float = IDEAL_ANGLE):
    """The strip approximation of Sections 3.2.2 / 3.2.3 with strips of
    integer ``width`` (vertical, or horizontal): (E_ca, crossing count, sum
    of |ideal - a|/ideal, number of strip pieces).  Synchronizes."""
    import ctypes as C
    _check_coords(x, y)
    _check_edges(x, src, dst)
    dev = x.device
    key = dev.index if dev.index is not None else torch.cuda.current_device()
    out = _out(3, torch.float64, dev)
    pieces = C.c_uint64()
    need = int(lib().rb_enhanced_workspace_size(src.numel(), 0))
    for _ in range(2):
        ws = _strip_ws.get(key)
        if ws is None or ws.numel() < need + 256:
            _strip_ws.pop(key, None)
            ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
            _strip_ws[key] = ws
        w, wb = _ws_args(ws)
        p = _ptr(out)
        rc = lib().rb_enhanced_crossing(_ptr(x), _ptr(y), x.numel(), _ptr(src), _ptr(dst),
                                        src.numel(), int(width), int(bool(horizontal)),
                                        float(ideal_angle), p, p + 8, p + 16, C.byref(pieces), w,
                                        wb, _stream(dev))
        if rc == 2 and pieces.value:            # workspace short for this many pieces
            need = int(lib().rb_enhanced_workspace_size(src.numel(), pieces.value))
            if need == 0:
                break
            continue
        break
    check(rc, "rb_enhanced_crossing")
    vals = out.cpu()
    return float(vals[0]), int(vals.view(torch.int64)[1]), float(vals[2]), int(pieces.value)


def crossing_angle_shard(x, y, src, dst, shard: int, n_shards: int,
                         ideal_angle: float = IDEAL_ANGLE):
    """(crossings, sum of |ideal - a|/ideal, row_begin, row_end) of shard k
    of n of the edge-pair sweep: pairs (e, f), row_begin <= e < row_end, e < f."""
    import ctypes as C
    _check_coords(x, y)
    _check_edges(x, src, dst)
    out = _out(2, torch.float64, x.device)
    ws = workspace(x.numel(), src.numel(), x.device)
    w, wb = _ws_args(ws)
    rb, re_ = C.c_int64(), C.c_int64()
    p = _ptr(out)
    check(lib().rb_crossing_angle_shard(_ptr(x), _ptr(y), x.numel(), _ptr(src), _ptr(dst),
                                        src.numel(), float(ideal_angle), int(shard), int(n_shards),
                                        p, p + 8, C.byref(rb), C.byref(re_), w, wb,
                                        _stream(x.device)), "rb_crossing_angle_shard")
    vals = out.cpu()
    return int(vals.view(torch.int64)[0]), float(vals[1]), rb.value, re_.value


def node_occlusion_shard(x, y, diameter: float, shard: int, n_shards: int):
    """(occluded pairs, row_begin, row_end) of shard k of n of the node-pair
    sweep: pairs (u, v), row_begin <= u < row_end, u < v."""
    import ctypes as C
    _check_coords(x, y)
    out = _out(1, torch.int64, x.device)
    ws = workspace(x.numel(), 0, x.device)
    w, wb = _ws_args(ws)
    rb, re_ = C.c_int64(), C.c_int64()
    check(lib().rb_node_occlusion_shard(_ptr(x), _ptr(y), x.numel(), float(diameter), int(shard),
                                        int(n_shards), _ptr(out), C.byref(rb), C.byref(re_), w,
                                        wb, _stream(x.device)), "rb_node_occlusion_shard")
    return int(out.item()), rb.value, re_.value


def validate_layout(x, y, src, dst) -> int:
    """Bit set of violated preconditions (0 when the layout is valid)."""
    import ctypes as C
    _check_coords(x, y)
    _check_edges(x, src, dst)
    ws = workspace(x.numel(), src.numel(), x.device)
    w, wb = _ws_args(ws)
    flags = C.c_int32(0)
    rc = lib().rb_validate_layout(_ptr(x), _ptr(y), x.numel(), _ptr(src), _ptr(dst), src.numel(),
                                  C.byref(flags), w, wb, _stream(x.device))
    if rc not in (0, 3):
        check(rc, "rb_validate_layout")
    return int(flags.value)


@dataclass
class DeviceLayout:
    """A layout resident in GPU memory."""
    x: torch.Tensor
    y: torch.Tensor
    src: torch.Tensor
    dst: torch.Tensor
    diameter: float = 8.0
    ideal_angle: float = IDEAL_ANGLE

    @classmethod
    def from_host(cls, L, device="cuda"):
        """Copy a ``gen.Layout`` (numpy arrays) to the GPU."""
        t = lambda a, dt: torch.as_tensor(a).to(device=device, dtype=dt).contiguous()
        return cls(t(L.x, torch.float32), t(L.y, torch.float32), t(L.src, torch.int32),
                   t(L.dst, torch.int32), float(L.diameter), float(L.ideal_angle))


_side_streams: dict[int, torch.cuda.Stream] = {}


def _side_stream(dev: torch.device) -> torch.cuda.Stream:
    index = dev.index if dev.index is not None else torch.cuda.current_device()
    st = _side_streams.get(index)
    if st is None:                      # default priority, like every stream here
        st = _side_streams[index] = torch.cuda.Stream(device=torch.device("cuda", index))
    return st


def evaluate_async(D: DeviceLayout):
    """All five metrics of one device layout, enqueued without a host wait:
    the edge-pair sweep on the current stream, and the node sweep, minimum
    angle and edge lengths on a second stream (its own workspace), so they
    run in the resources the edge sweep leaves idle.  The current stream
    waits for both.  Returns the device tensors of node_occlusion,
    crossing_angle, min_angle and edge_length_variation (``async_=True``)."""
    dev = D.x.device
    main = torch.cuda.current_stream(dev)
    side = _side_stream(dev)
    side.wait_stream(main)
    for t in (D.x, D.y, D.src, D.dst):  # read on the side stream too
        t.record_stream(side)
    with torch.cuda.stream(side):
        occ = node_occlusion(D.x, D.y, D.diameter, async_=True)
        ma = min_angle(D.x, D.y, D.src, D.dst, async_=True)
        ml = edge_length_variation(D.x, D.y, D.src, D.dst, async_=True)
    ang = crossing_angle(D.x, D.y, D.src, D.dst, D.ideal_angle, async_=True)
    main.wait_stream(side)
    for t in (occ, ma, ml):             # made on the side stream, read on this one
        t.record_stream(main)
    return occ, ang, ma, ml


def evaluate(D: DeviceLayout) -> dict:
    """All five metrics of one device layout (one pass of the hot path)."""
    occ, ang, ma, ml = evaluate_async(D)
    occ, ang, ma, ml = occ.cpu(), ang.cpu(), ma.cpu(), ml.cpu()
    return dict(node_occlusion=int(occ[0]), crossing_angle=float(ang[0]),
                edge_crossing=int(ang.view(torch.int64)[1]), crossing_dev_sum=float(ang[2]),
                min_angle=float(ma[0]), min_angle_sum_dv=float(ma[1]),
                min_angle_n_used=int(ma.view(torch.int64)[2]), edge_length_variation=float(ml[0]),
                mean_edge_length=float(ml[1]))
