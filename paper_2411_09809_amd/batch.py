"""Batched evaluation of many layouts (rb_batch_* of include/rb.h).

``Batch`` concatenates a list of layouts on the GPU, builds and uploads the
plan once, and then evaluates all five metrics of every layout with one
launch per all-pairs sweep -- eagerly, or by replaying a captured hipGraph.  Results are device tensors of one entry per layout.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import gen
from ._lib import check, lib
from .metrics import IDEAL_ANGLE


class Batch:
    def __init__(self, layouts, device="cuda", ideal_angle: float = IDEAL_ANGLE):
        x, y, src, dst, node_off, edge_off = gen.concat_layouts(layouts)
        dev = torch.device(device)
        self.device = dev
        self.n = len(layouts)
        self.ideal_angle = float(ideal_angle)
        self.node_off = np.ascontiguousarray(node_off, dtype=np.int64)
        self.edge_off = np.ascontiguousarray(edge_off, dtype=np.int64)
        self.diameters = np.ascontiguousarray([float(L.diameter) for L in layouts], dtype=np.float64)
        self.x = torch.as_tensor(x).to(dev).contiguous()
        self.y = torch.as_tensor(y).to(dev).contiguous()
        self.src = torch.as_tensor(src).to(dev).contiguous()
        self.dst = torch.as_tensor(dst).to(dev).contiguous()
        h = C.c_void_p()
        check(lib().rb_batch_create(self.n, self.node_off.ctypes.data, self.edge_off.ctypes.data,
                                    self.diameters.ctypes.data, C.byref(h)), "rb_batch_create")
        self._h = h
        self._graph = None
        need = int(lib().rb_batch_workspace_size(self._h))
        self._ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
        p = self._ws.data_ptr()
        self._w = (p + 255) & ~255
        self._wb = self._ws.numel() - (self._w - p)
        self.out_occlusion = torch.zeros(self.n, dtype=torch.int64, device=dev)
        self.out_crossings = torch.zeros(self.n, dtype=torch.int64, device=dev)
        self.out_crossing_angle = torch.zeros(self.n, dtype=torch.float64, device=dev)
        self.out_min_angle = torch.zeros(self.n, dtype=torch.float64, device=dev)
        self.out_elv = torch.zeros(self.n, dtype=torch.float64, device=dev)
        self._upload()

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def _upload(self):
        check(lib().rb_batch_upload(self._h, self._w, self._wb, self._stream()), "rb_batch_upload")

    def _args(self):
        return (self.x.data_ptr(), self.y.data_ptr(), self.src.data_ptr(), self.dst.data_ptr(),
                self.ideal_angle, self.out_occlusion.data_ptr(), self.out_crossings.data_ptr(),
                self.out_crossing_angle.data_ptr(), self.out_min_angle.data_ptr(),
                self.out_elv.data_ptr(), self._w, self._wb)

    def evaluate(self):
        """Enqueue one evaluation of every layout; results land in out_*."""
        check(lib().rb_batch_evaluate(self._h, *self._args(), self._stream()), "rb_batch_evaluate")

    def capture(self):
        """Capture ``evaluate`` into a hipGraph (kept by this object)."""
        self.release_graph()
        g = C.c_void_p()
        check(lib().rb_batch_graph_create(self._h, *self._args(), C.byref(g)),
              "rb_batch_graph_create")
        self._graph = g

    def replay(self):
        """Launch the captured graph on the current stream."""
        if self._graph is None:
            raise RuntimeError("capture() first")
        check(lib().rb_graph_launch(self._graph, self._stream()), "rb_graph_launch")

    def autotune(self, repeats: int = 3) -> float:
        """Time the sweep variants on this batch and keep the fastest."""
        ms = C.c_double()
        check(lib().rb_batch_autotune(self._h, self.x.data_ptr(), self.y.data_ptr(),
                                      self.src.data_ptr(), self.dst.data_ptr(), self.ideal_angle,
                                      int(repeats), C.byref(ms), self._w, self._wb,
                                      self._stream()), "rb_batch_autotune")
        if self._graph is not None:
            self.capture()              # the plan's tables were re-uploaded
        return float(ms.value)

    def variants(self) -> dict:
        v = [C.c_int() for _ in range(4)]
        check(lib().rb_batch_variants(self._h, *[C.byref(a) for a in v]), "rb_batch_variants")
        return dict(cross_rows=v[0].value, cross_waves=v[1].value, occl_rows=v[2].value,
                    occl_waves=v[3].value)

    def results(self) -> dict:
        """The out_* tensors as numpy arrays (waits for the stream)."""
        return dict(node_occlusion=self.out_occlusion.cpu().numpy(),
                    edge_crossing=self.out_crossings.cpu().numpy(),
                    crossing_angle=self.out_crossing_angle.cpu().numpy(),
                    min_angle=self.out_min_angle.cpu().numpy(),
                    edge_length_variation=self.out_elv.cpu().numpy())

    def layout_views(self, i: int):
        """Device views of layout i (for single-layout calls)."""
        a, b = int(self.node_off[i]), int(self.node_off[i + 1])
        c, d = int(self.edge_off[i]), int(self.edge_off[i + 1])
        return self.x[a:b], self.y[a:b], self.src[c:d], self.dst[c:d], float(self.diameters[i])

    def release_graph(self):
        if self._graph is not None:
            lib().rb_graph_destroy(self._graph)
            self._graph = None

    def __del__(self):
        try:
            self.release_graph()
            if getattr(self, "_h", None):
                lib().rb_batch_destroy(self._h)
                self._h = None
        except Exception:
            pass
