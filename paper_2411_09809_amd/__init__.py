"""Exact readability metrics of graph layouts on AMD MI355X (gfx950).

The five metrics of arXiv 2411.09809 (node occlusion, minimum angle, edge
length variation, edge crossing, crossing angle) computed by hand-written HIP
kernels in ``librb.so`` behind the C-ABI of ``include/rb.h``.

Submodules: ``gen`` (seeded synthetic layouts), ``metrics`` (torch-facing
entry points, imported lazily), ``build`` (compiles librb.so).
"""
_LAZY = {"node_occlusion", "edge_crossing", "crossing_angle", "min_angle",
         "edge_length_variation", "validate_layout", "evaluate", "DeviceLayout", "workspace",
         "IDEAL_ANGLE"}


def __getattr__(name):
    if name in _LAZY:
        from . import metrics
        return getattr(metrics, name)
    raise AttributeError(name)
