"""Python access to the CPU oracle (``oracle/liboracle.so``).

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  The product package never imports this module.

Each function takes the arrays of one layout (any numeric dtype for the
coordinates; they are passed as float64 holding integers) and returns Python
numbers.  The library is built on first use if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None
_i64 = C.c_int64
_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u64p = C.POINTER(C.c_uint64)


class OracleError(RuntimeError):
    pass


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.oracle_node_occlusion.argtypes = [_dp, _dp, _i64, C.c_double, _u64p]
        L.oracle_edge_crossing.argtypes = [_dp, _dp, _i64, _i32p, _i32p, _i64, _u64p, _u64p]
        L.oracle_crossing_angle.argtypes = [_dp, _dp, _i64, _i32p, _i32p, _i64, C.c_double,
                                            _dp, _u64p, _dp]
        L.oracle_crossings_of_edges.argtypes = [_dp, _dp, _i64, _i32p, _i32p, _i64, C.c_double,
                                                _i64p, _i64, _u64p, _dp]
        L.oracle_min_angle.argtypes = [_dp, _dp, _i64, _i32p, _i32p, _i64, _dp, _dp, _u64p]
        L.oracle_edge_length_variation.argtypes = [_dp, _dp, _i64, _i32p, _i32p, _i64, _dp, _dp]
        L.oracle_segment_pair.argtypes = [_dp, C.c_double, C.POINTER(C.c_int), _dp]
        L.oracle_crossing_angle_rows.argtypes = [_dp, _dp, _i64, _i32p, _i32p, _i64, C.c_double,
                                                 _i64, _i64, _u64p, _u64p, _dp]
        L.oracle_node_occlusion_rows.argtypes = [_dp, _dp, _i64, C.c_double, _i64, _i64, _u64p]
        L.oracle_enhanced_crossing.argtypes = [_dp, _dp, _i64, _i32p, _i32p, _i64, _i64, C.c_int,
                                               C.c_double, _u64p, _dp]
        L.oracle_min_angle_term.argtypes = [_dp, _dp, _i64, _i32p, _i32p, _i64, C.c_double, _dp,
                                             _dp, _dp]
        L.oracle_crossing_pairs.argtypes = [_dp, _dp, _i64, _i32p, _i32p, _i64, _i64p, _i64, _i64p]
        L.oracle_loss.argtypes = [_dp, _dp, _i64, _i32p, _i32p, _i64, _i64p, _i64, C.c_double,
                                  C.c_double, C.c_double, _dp]
        L.oracle_loss_grad.argtypes = [_dp, _dp, _i64, _i32p, _i32p, _i64, _i64p, _i64,
                                       C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _p(a, t):
    return a.ctypes.data_as(t)


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def _unpack(L):
    x, y, s, d = _f64(L.x), _f64(L.y), _i32(L.src), _i32(L.dst)
    return x, y, s, d


def node_occlusion(x, y, diameter: float) -> int:
    x, y = _f64(x), _f64(y)
    out = C.c_uint64()
    _check(lib().oracle_node_occlusion(_p(x, _dp), _p(y, _dp), x.shape[0],
                                       float(diameter), C.byref(out)), "node_occlusion")
    return int(out.value)


def edge_crossing(x, y, src, dst) -> tuple[int, int]:
    """(closed crossing count, proper crossing count)."""
    x, y, s, d = _f64(x), _f64(y), _i32(src), _i32(dst)
    c, p = C.c_uint64(), C.c_uint64()
    _check(lib().oracle_edge_crossing(_p(x, _dp), _p(y, _dp), x.shape[0], _p(s, _i32p),
                                      _p(d, _i32p), s.shape[0], C.byref(c), C.byref(p)),
           "edge_crossing")
    return int(c.value), int(p.value)


def crossing_angle(x, y, src, dst, ideal_angle: float) -> tuple[float, int, float]:
    """(metric E_ca, crossing count, sum of |ideal - a| / ideal)."""
    x, y, s, d = _f64(x), _f64(y), _i32(src), _i32(dst)
    met, cnt, sm = C.c_double(), C.c_uint64(), C.c_double()
    _check(lib().oracle_crossing_angle(_p(x, _dp), _p(y, _dp), x.shape[0], _p(s, _i32p),
                                       _p(d, _i32p), s.shape[0], float(ideal_angle),
                                       C.byref(met), C.byref(cnt), C.byref(sm)),
           "crossing_angle")
    return float(met.value), int(cnt.value), float(sm.value)


def crossings_of_edges(x, y, src, dst, ideal_angle: float, which):
    """Per listed edge: (number of crossing edges, sum of |ideal - a|)."""
    x, y, s, d = _f64(x), _f64(y), _i32(src), _i32(dst)
    w = np.ascontiguousarray(np.asarray(which, dtype=np.int64))
    cnt = np.zeros(w.shape[0], dtype=np.uint64)
    dev = np.zeros(w.shape[0], dtype=np.float64)
    _check(lib().oracle_crossings_of_edges(_p(x, _dp), _p(y, _dp), x.shape[0], _p(s, _i32p),
                                           _p(d, _i32p), s.shape[0], float(ideal_angle),
                                           _p(w, _i64p), w.shape[0], _p(cnt, _u64p),
                                           _p(dev, _dp)), "crossings_of_edges")
    return cnt, dev


def min_angle(x, y, src, dst) -> tuple[float, float, int]:
    """(metric M_a, sum of d_v, number of vertices with degree >= 1)."""
    x, y, s, d = _f64(x), _f64(y), _i32(src), _i32(dst)
    met, sdv, used = C.c_double(), C.c_double(), C.c_uint64()
    _check(lib().oracle_min_angle(_p(x, _dp), _p(y, _dp), x.shape[0], _p(s, _i32p),
                                  _p(d, _i32p), s.shape[0], C.byref(met), C.byref(sdv),
                                  C.byref(used)), "min_angle")
    return float(met.value), float(sdv.value), int(used.value)


def edge_length_variation(x, y, src, dst) -> tuple[float, float]:
    """(metric M_l, mean edge length)."""
    x, y, s, d = _f64(x), _f64(y), _i32(src), _i32(dst)
    met, mu = C.c_double(), C.c_double()
    _check(lib().oracle_edge_length_variation(_p(x, _dp), _p(y, _dp), x.shape[0],
                                              _p(s, _i32p), _p(d, _i32p), s.shape[0],
                                              C.byref(met), C.byref(mu)),
           "edge_length_variation")
    return float(met.value), float(mu.value)


def segment_pair(p, ideal_angle: float = 1.2217304763960306) -> tuple[int, float]:
    """Crossing kind (0 none, 1 touching/overlapping, 2 proper) and the acute
    line angle of two segments p = (x0,y0,x1,y1, x2,y2,x3,y3)."""
    a = _f64(p)
    kind, ang = C.c_int(), C.c_double()
    _check(lib().oracle_segment_pair(_p(a, _dp), float(ideal_angle), C.byref(kind),
                                     C.byref(ang)), "segment_pair")
    return int(kind.value), float(ang.value)


def crossing_angle_rows(x, y, src, dst, ideal_angle: float, r0: int, r1: int,
                        proper: bool = False):
    """(crossings, sum of |ideal - a|/ideal) over pairs (e, f), r0 <= e < r1,
    e < f; with ``proper``, (crossings, proper crossings, sum)."""
    x, y, s, d = _f64(x), _f64(y), _i32(src), _i32(dst)
    cnt, prop, dev = C.c_uint64(), C.c_uint64(), C.c_double()
    _check(lib().oracle_crossing_angle_rows(_p(x, _dp), _p(y, _dp), x.shape[0], _p(s, _i32p),
                                            _p(d, _i32p), s.shape[0], float(ideal_angle),
                                            int(r0), int(r1), C.byref(cnt), C.byref(prop),
                                            C.byref(dev)),
           "crossing_angle_rows")
    if proper:
        return int(cnt.value), int(prop.value), float(dev.value)
    return int(cnt.value), float(dev.value)


def node_occlusion_rows(x, y, diameter: float, r0: int, r1: int) -> int:
    """Occluded pairs (u, v), r0 <= u < r1, u < v."""
    x, y = _f64(x), _f64(y)
    out = C.c_uint64()
    _check(lib().oracle_node_occlusion_rows(_p(x, _dp), _p(y, _dp), x.shape[0], float(diameter),
                                            int(r0), int(r1), C.byref(out)), "node_occlusion_rows")
    return int(out.value)


def enhanced_crossing(x, y, src, dst, width: int, horizontal: bool, ideal_angle: float):
    """(count, sum of |ideal - a|/ideal) of the strip method of Sections 3.2.2
    and 3.2.3 (strips of integer width, vertical or horizontal)."""
    x, y, s, d = _f64(x), _f64(y), _i32(src), _i32(dst)
    cnt, dev = C.c_uint64(), C.c_double()
    _check(lib().oracle_enhanced_crossing(_p(x, _dp), _p(y, _dp), x.shape[0], _p(s, _i32p),
                                          _p(d, _i32p), s.shape[0], int(width), int(horizontal),
                                          float(ideal_angle), C.byref(cnt), C.byref(dev)),
           "enhanced_crossing")
    return int(cnt.value), float(dev.value)


def crossing_pairs(x, y, src, dst) -> np.ndarray:
    """The crossing set S as an (|S|, 2) array of edge indices e < f."""
    x, y, s, d = _f64(x), _f64(y), _i32(src), _i32(dst)
    n = C.c_int64()
    _check(lib().oracle_crossing_pairs(_p(x, _dp), _p(y, _dp), x.shape[0], _p(s, _i32p),
                                       _p(d, _i32p), s.shape[0], None, 0, C.byref(n)),
           "crossing_pairs")
    out = np.zeros((max(n.value, 1), 2), dtype=np.int64)
    _check(lib().oracle_crossing_pairs(_p(x, _dp), _p(y, _dp), x.shape[0], _p(s, _i32p),
                                       _p(d, _i32p), s.shape[0], _p(out, _i64p), n.value,
                                       C.byref(n)), "crossing_pairs")
    return out[:n.value]


def min_angle_term(x, y, src, dst, w_min_angle=1.0, grad=False):
    """w_m (1 - M_a) at (possibly non-integer) coordinates; with grad, also
    its gradient (dT/dx, dT/dy)."""
    x, y, s, d = _f64(x), _f64(y), _i32(src), _i32(dst)
    out = C.c_double()
    gx = np.zeros(x.shape[0]) if grad else None
    gy = np.zeros(x.shape[0]) if grad else None
    _check(lib().oracle_min_angle_term(_p(x, _dp), _p(y, _dp), x.shape[0], _p(s, _i32p),
                                       _p(d, _i32p), s.shape[0], float(w_min_angle),
                                       C.byref(out), _p(gx, _dp) if grad else None,
                                       _p(gy, _dp) if grad else None), "min_angle_term")
    return (float(out.value), gx, gy) if grad else float(out.value)


def loss(x, y, src, dst, pairs, ideal_angle, w_angle=1.0, w_length=1.0,
         w_min_angle=0.0) -> float:
    """w_a (1 - E_ca) + w_l M_l + w_m (1 - M_a) at (possibly non-integer)
    coordinates, with the crossing set frozen to ``pairs``."""
    x, y, s, d = _f64(x), _f64(y), _i32(src), _i32(dst)
    P = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    out = C.c_double()
    _check(lib().oracle_loss(_p(x, _dp), _p(y, _dp), x.shape[0], _p(s, _i32p), _p(d, _i32p),
                             s.shape[0], _p(P, _i64p), P.shape[0], float(ideal_angle),
                             float(w_angle), float(w_length), C.byref(out)), "loss")
    f = float(out.value)
    if w_min_angle:
        f += min_angle_term(x, y, s, d, w_min_angle)
    return f


def loss_grad(x, y, src, dst, pairs, ideal_angle, w_angle=1.0, w_length=1.0, w_min_angle=0.0):
    """(loss, dL/dx, dL/dy) -- the analytic gradient of ``loss``."""
    x, y, s, d = _f64(x), _f64(y), _i32(src), _i32(dst)
    P = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    gx = np.zeros(x.shape[0])
    gy = np.zeros(x.shape[0])
    out = C.c_double()
    _check(lib().oracle_loss_grad(_p(x, _dp), _p(y, _dp), x.shape[0], _p(s, _i32p),
                                  _p(d, _i32p), s.shape[0], _p(P, _i64p), P.shape[0],
                                  float(ideal_angle), float(w_angle), float(w_length),
                                  C.byref(out), _p(gx, _dp), _p(gy, _dp)), "loss_grad")
    f = float(out.value)
    if w_min_angle:
        t, tx, ty = min_angle_term(x, y, s, d, w_min_angle, grad=True)
        f, gx, gy = f + t, gx + tx, gy + ty
    return f, gx, gy


def all_metrics(L) -> dict:
    """The five metrics of one layout (``paper_2411_09809_amd.gen.Layout``)."""
    x, y, s, d = _unpack(L)
    closed, proper = edge_crossing(x, y, s, d)
    eca, cnt, devsum = crossing_angle(x, y, s, d, L.ideal_angle)
    ma, sdv, used = min_angle(x, y, s, d)
    ml, mu = edge_length_variation(x, y, s, d)
    return dict(node_occlusion=node_occlusion(x, y, L.diameter), edge_crossing=closed,
                proper_crossing=proper, crossing_angle=eca, crossing_dev_sum=devsum,
                min_angle=ma, min_angle_sum_dv=sdv, min_angle_n_used=used,
                edge_length_variation=ml, mean_edge_length=mu)
