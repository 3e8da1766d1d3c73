"""ctypes loader for ``librb.so`` (the C-ABI of include/rb.h).

Argument marshalling only.  The library must have been built with
``python -m paper_2411_09809_amd.build`` (or ``__graft_entry__.build()``);
there is no fallback: a missing library raises ``RBError``.  The environment
variable RB_LIBRARY may name another build of it.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# RB_LIBRARY names another build of the same library (the host-sanitized one
# of the CPU tests); by default the in-tree librb.so
LIB_PATH = os.environ.get("RB_LIBRARY") or os.path.join(HERE, "librb.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "rb.h")

RB_OK, RB_EINVAL, RB_EWORKSPACE, RB_EDOMAIN, RB_EHIP, RB_ENOMEM = range(6)
STATUS_NAMES = {0: "RB_OK", 1: "RB_EINVAL", 2: "RB_EWORKSPACE", 3: "RB_EDOMAIN", 4: "RB_EHIP",
                5: "RB_ENOMEM"}


class RBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_vp, _i64, _f64, _sz = C.c_void_p, C.c_int64, C.c_double, C.c_size_t

_SIGS = {
    "rb_version": ([], C.c_char_p),
    "rb_last_error": ([], C.c_char_p),
    "rb_workspace_size": ([_i64, _i64], _sz),
    "rb_node_occlusion": ([_vp, _vp, _i64, _f64, _vp, _vp, _sz, _vp], C.c_int),
    "rb_edge_crossing": ([_vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _sz, _vp], C.c_int),
    "rb_crossing_angle": ([_vp, _vp, _i64, _vp, _vp, _i64, _f64, _vp, _vp, _vp, _vp, _sz, _vp],
                          C.c_int),
    "rb_crossing_angle_noalloc": ([_vp, _vp, _i64, _vp, _vp, _i64, _f64, _vp, _vp, _vp, _vp],
                                  C.c_int),
    "rb_min_angle": ([_vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _sz, _vp], C.c_int),
    "rb_edge_length_variation": ([_vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _sz, _vp],
                                 C.c_int),
    "rb_validate_layout": ([_vp, _vp, _i64, _vp, _vp, _i64, C.POINTER(C.c_int32), _vp, _sz, _vp],
                           C.c_int),
    "rb_grid_workspace_size": ([_i64, _i64], _sz),
    "rb_node_occlusion_grid": ([_vp, _vp, _i64, _f64, _vp, _vp, _sz, _vp], C.c_int),
    "rb_crossing_angle_pruned": ([_vp, _vp, _i64, _vp, _vp, _i64, _f64, _vp, _vp, _vp, _vp, _sz,
                                  _vp], C.c_int),
    "rb_loss_grad_pruned": ([_vp, _vp, _i64, _vp, _vp, _i64, _f64, _f64, _f64, _f64, _vp, _vp,
                             _vp, _vp, _vp, _sz, _vp], C.c_int),
    "rb_enhanced_workspace_size": ([_i64, C.c_uint64], _sz),
    "rb_enhanced_crossing": ([_vp, _vp, _i64, _vp, _vp, _i64, _i64, C.c_int, _f64, _vp, _vp, _vp,
                              C.POINTER(C.c_uint64), _vp, _sz, _vp], C.c_int),
    "rb_crossing_angle_shard": ([_vp, _vp, _i64, _vp, _vp, _i64, _f64, _i64, _i64, _vp, _vp,
                                 C.POINTER(C.c_int64), C.POINTER(C.c_int64), _vp, _sz, _vp],
                                C.c_int),
    "rb_node_occlusion_shard": ([_vp, _vp, _i64, _f64, _i64, _i64, _vp, C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int64), _vp, _sz, _vp], C.c_int),
    "rb_loss_grad": ([_vp, _vp, _i64, _vp, _vp, _i64, _f64, _f64, _f64, _f64, _vp, _vp, _vp, _vp,
                      _vp, _sz, _vp], C.c_int),
    "rb_autotune": ([_vp, _vp, _i64, _vp, _vp, _i64, _f64, _f64, C.c_int, C.POINTER(C.c_double),
                     _vp, _sz, _vp], C.c_int),
    "rb_valu_probe": ([C.c_int, C.c_int, C.POINTER(C.c_double), _vp, _vp], C.c_int),
    "rb_tune_set": ([C.c_int, C.c_int, _i64, C.c_int], C.c_int),
    "rb_tune_query": ([C.c_int, C.c_int, _i64, C.POINTER(C.c_int), C.POINTER(C.c_int),
                       C.POINTER(C.c_int)], C.c_int),
    "rb_tune_save": ([C.c_char_p], C.c_int),
    "rb_tune_load": ([C.c_char_p], C.c_int),
    "rb_batch_create": ([_i64, _vp, _vp, _vp, C.POINTER(C.c_void_p)], C.c_int),
    "rb_batch_workspace_size": ([_vp], _sz),
    "rb_batch_upload": ([_vp, _vp, _sz, _vp], C.c_int),
    "rb_batch_evaluate": ([_vp, _vp, _vp, _vp, _vp, _f64, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp],
                          C.c_int),
    "rb_batch_autotune": ([_vp, _vp, _vp, _vp, _vp, _f64, C.c_int, C.POINTER(C.c_double), _vp,
                           _sz, _vp], C.c_int),
    "rb_batch_variants": ([_vp] + [C.POINTER(C.c_int)] * 4, C.c_int),
    "rb_batch_destroy": ([_vp], None),
    "rb_batch_graph_create": ([_vp, _vp, _vp, _vp, _vp, _f64, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                               C.POINTER(C.c_void_p)], C.c_int),
    "rb_graph_launch": ([_vp, _vp], C.c_int),
    "rb_graph_destroy": ([_vp], None),
    "rb_timing_enable": ([C.c_int], C.c_int),
    "rb_timing_reset": ([], C.c_int),
    "rb_timing_read": ([C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
}


def header_symbols() -> list[str]:
    """Names of the functions declared in include/rb.h."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rb_[a-z_0-9]+)\s*\(", text)))


def lib():
    """Load librb.so once; raise RBError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RBError(RB_EHIP, f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_2411_09809_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(status: int, what: str):
    if status != RB_OK:
        raise RBError(status, f"{what}: {lib().rb_last_error().decode()}")
