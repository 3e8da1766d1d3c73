"""The C-ABI library without a GPU: it loads, exports every function that
include/rb.h declares, and rejects bad arguments before touching the GPU."""
import ctypes as C
import os
import subprocess

import pytest

from paper_2411_09809_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _lib.header_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(names) <= exported


def test_header_compiles_as_c():
    src = '#include "rb.h"\nint main(void){return (int)rb_workspace_size(1,1) < 0;}\n'
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c",
                        "-I", os.path.join(ROOT, "include"), "-"], input=src, text=True,
                       capture_output=True)
    assert r.returncode == 0, r.stderr


def test_version_and_workspace(L):
    assert L.rb_version().decode().startswith("rb ")
    a = L.rb_workspace_size(1000, 2000)
    b = L.rb_workspace_size(50000, 149994)
    assert a > 0 and b > a and a % 256 == 0 and b % 256 == 0
    assert L.rb_workspace_size(0, 0) > 0
    assert L.rb_workspace_size(-1, 5) == 0
    assert L.rb_workspace_size(10, 1 << 31) == 0
    # from 2^20 edges on, room for the hub sort: degrees, keys and values twice
    below, at = L.rb_workspace_size(1000, (1 << 20) - 1), L.rb_workspace_size(1000, 1 << 20)
    assert at - below >= 1000 * 4 + 16 * (1 << 20)


def _err(L):
    return L.rb_last_error().decode()


def test_argument_errors_need_no_gpu(L):
    fake = 0x1000                     # never dereferenced: checks fail first
    ws_need = L.rb_workspace_size(10, 5)
    # NULL out pointer
    assert L.rb_edge_crossing(fake, fake, 10, fake, fake, 5, None, None, fake * 256, ws_need,
                              None) == _lib.RB_EINVAL
    assert "out_count" in _err(L)
    # NULL coordinates
    assert L.rb_node_occlusion(None, None, 10, 8.0, fake, fake * 256, ws_need,
                               None) == _lib.RB_EINVAL
    # bad diameter and ideal angle
    assert L.rb_node_occlusion(fake, fake, 10, -1.0, fake, fake * 256, ws_need,
                               None) == _lib.RB_EINVAL
    assert L.rb_node_occlusion(fake, fake, 10, float("inf"), fake, fake * 256, ws_need,
                               None) == _lib.RB_EINVAL
    assert L.rb_crossing_angle(fake, fake, 10, fake, fake, 5, 2.0, fake, None, None, fake * 256,
                               ws_need, None) == _lib.RB_EINVAL
    assert "ideal_angle" in _err(L)
    # negative sizes
    assert L.rb_min_angle(fake, fake, -3, fake, fake, 5, fake, None, None, fake * 256, ws_need,
                          None) == _lib.RB_EINVAL
    # edges without nodes
    assert L.rb_edge_length_variation(fake, fake, 1, fake, fake, 5, fake, None, fake * 256,
                                      ws_need, None) == _lib.RB_EINVAL
    # workspace: NULL, misaligned, too small
    assert L.rb_edge_crossing(fake, fake, 10, fake, fake, 5, fake, None, None, ws_need,
                              None) == _lib.RB_EWORKSPACE
    assert L.rb_edge_crossing(fake, fake, 10, fake, fake, 5, fake, None, fake * 256 + 8, ws_need,
                              None) == _lib.RB_EWORKSPACE
    assert L.rb_edge_crossing(fake, fake, 10, fake, fake, 5, fake, None, fake * 256, ws_need - 1,
                              None) == _lib.RB_EWORKSPACE
    assert "needed" in _err(L)
    assert L.rb_timing_read(7, None, None) == _lib.RB_EINVAL
    assert L.rb_timing_read(5, None, None) == _lib.RB_EINVAL
    # kind 4 (the fused forward + adjoint sweep) exists; nothing is recorded yet
    import ctypes as C
    ms, n = C.c_double(-1.0), C.c_int64(-1)
    assert L.rb_timing_reset() == 0
    assert L.rb_timing_read(4, C.byref(ms), C.byref(n)) == 0
    assert ms.value == 0.0 and n.value == 0
    # the FMA probe checks its arguments before touching the device
    rate = C.c_double()
    assert L.rb_valu_probe(0, 1, C.byref(rate), fake, None) == _lib.RB_EINVAL
    assert L.rb_valu_probe(16, 1, None, fake, None) == _lib.RB_EINVAL
    assert L.rb_valu_probe(16, 1, C.byref(rate), None, None) == _lib.RB_EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "librb.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(_lib.RBError):
        _lib.lib()


def test_argument_errors_of_the_other_entry_points_need_no_gpu(L):
    fake = 0x1000                     # never dereferenced: checks fail first
    ws = fake * 256
    need = L.rb_workspace_size(10, 5)
    gneed = L.rb_grid_workspace_size(10, 5)
    ideal = 1.2217304763960306
    nan = float("nan")
    # loss and gradient: weights must be finite, the ideal angle in (0, pi/2]
    for fn in (L.rb_loss_grad, L.rb_loss_grad_pruned):
        ws_bytes = need if fn is L.rb_loss_grad else gneed
        assert fn(fake, fake, 10, fake, fake, 5, ideal, 1.0, 1.0, nan, fake, fake, fake, None,
                  ws, ws_bytes, None) == _lib.RB_EINVAL
        assert "finite" in _err(L)
        assert fn(fake, fake, 10, fake, fake, 5, 0.0, 1.0, 1.0, 0.0, fake, fake, fake, None,
                  ws, ws_bytes, None) == _lib.RB_EINVAL
        assert fn(fake, fake, 10, fake, fake, 5, ideal, 1.0, 1.0, 0.0, None, fake, fake, None,
                  ws, ws_bytes, None) == _lib.RB_EINVAL
    # the pruned edge sweep indexes its unit list in 32 bits
    big = (1 << 24) + 1
    assert L.rb_loss_grad_pruned(fake, fake, 10, fake, fake, big, ideal, 1.0, 1.0, 0.0, fake,
                                 fake, fake, None, ws, gneed, None) == _lib.RB_EINVAL
    assert "2^24" in _err(L)
    # shards: 0 <= shard < n_shards
    lo, hi = C.c_int64(), C.c_int64()
    assert L.rb_crossing_angle_shard(fake, fake, 10, fake, fake, 5, ideal, 3, 3, fake, None,
                                     C.byref(lo), C.byref(hi), ws, need,
                                     None) == _lib.RB_EINVAL
    assert "shard" in _err(L)
    assert L.rb_node_occlusion_shard(fake, fake, 10, 8.0, -1, 2, fake, C.byref(lo), C.byref(hi),
                                     ws, need, None) == _lib.RB_EINVAL
    # grid paths: a workspace shorter than rb_grid_workspace_size
    assert L.rb_node_occlusion_grid(fake, fake, 10, 8.0, fake, ws, gneed - 256,
                                    None) == _lib.RB_EWORKSPACE
    assert L.rb_crossing_angle_pruned(fake, fake, 10, fake, fake, 5, ideal, fake, None, None, ws,
                                      gneed - 256, None) == _lib.RB_EWORKSPACE
    # strips: integer width in [1, 2^22]
    pieces = C.c_uint64(7)
    assert L.rb_enhanced_crossing(fake, fake, 10, fake, fake, 5, 0, 0, ideal, fake, None, None,
                                  C.byref(pieces), ws, L.rb_enhanced_workspace_size(5, 0),
                                  None) == _lib.RB_EINVAL
    assert "width" in _err(L)


def test_built_in_tuning_defaults(L, tmp_path):
    """The defaults a table returns to on a load of an empty file: crossing
    sweeps 2 rows / 7 waves, but 3 rows / 5 waves for the crossing + angle
    sweep of a single layout from 2^21 edges; the node sweep of a single layout
    2 rows / 8 waves in chunks split 8 ways below 2^13 nodes, 4 rows / 8 waves
    split 8 ways below 2^14 and 4 ways below 2^16, 4 rows / 8 waves in whole
    chunks from there (a batch: 4 rows / 8 waves, whole chunks, below a mean
    of 2^19 nodes); the pruned sweep 1-row tiles below 2^17 edges and 2-row
    tiles from there."""
    import ctypes as C
    empty = tmp_path / "tune.txt"
    empty.write_text("")
    assert L.rb_tune_load(str(empty).encode()) == 0

    def q(kind, n, batch=0):
        rows, waves, split = C.c_int(), C.c_int(), C.c_int()
        assert L.rb_tune_query(kind, batch, n, C.byref(rows), C.byref(waves),
                               C.byref(split)) == 0
        return (rows.value, waves.value) if kind != 2 else (rows.value, waves.value, split.value)

    for n in (2_000, 149_994, 3_000_000):
        assert q(0, n) == (2, 7) and q(1, n, batch=1) == (2, 7)
    assert q(1, 149_994) == (2, 7) and q(1, (1 << 21) - 1) == (2, 7)
    assert q(1, 1 << 21) == (3, 5) and q(1, 3_000_000) == (3, 5)
    assert q(2, 1_000) == (2, 8, 8) and q(2, (1 << 13) - 1) == (2, 8, 8)
    assert q(2, 1 << 13) == (4, 8, 8) and q(2, 20_000) == (4, 8, 4)
    assert q(2, (1 << 15) - 1) == (4, 8, 4) and q(2, 50_000) == (4, 8, 4)
    assert q(2, (1 << 16) - 1) == (4, 8, 4) and q(2, 1 << 16) == (4, 8, 1)
    assert q(2, 1_000_000) == (4, 8, 1)
    assert q(2, 50_000, batch=1) == (4, 8, 1) and q(2, 1 << 19, batch=1) == (8, 5, 1)
    assert q(3, (1 << 17) - 1) == (1, 8) and q(3, 1 << 17) == (2, 7)


def test_static_scratch_limit_needs_no_gpu(L):
    fake = 0x1000                     # never dereferenced: checks fail first
    assert L.rb_crossing_angle_noalloc(fake, fake, 10, fake, fake, 1_000_001, 1.2, fake, None,
                                       None, None) == _lib.RB_EINVAL
    assert "static scratch" in _err(L)
    assert L.rb_crossing_angle_noalloc(fake, fake, 10, fake, fake, 5, 1.2, None, None, None,
                                       None) == _lib.RB_EINVAL
    assert "out_metric" in _err(L)
    assert L.rb_crossing_angle_noalloc(fake, fake, 10, fake, fake, 5, 0.0, fake, None, None,
                                       None) == _lib.RB_EINVAL


def test_batched_crossing_sweep_does_not_offer_four_rows(L, tmp_path):
    """The 4-row variant (index 3) of the edge sweep is refused for batches
    (its batch form would spill registers in every block) and accepted for
    single layouts; a tuning file that names it for a batch is ignored."""
    import ctypes as C
    empty = tmp_path / "tune.txt"
    empty.write_text("")
    try:
        assert L.rb_tune_set(1, 1, 1000, 3) == _lib.RB_EINVAL
        assert "not offered" in _err(L)
        assert L.rb_tune_set(0, 1, 1000, 3) == _lib.RB_EINVAL
        assert L.rb_tune_set(1, 0, 1000, 3) == _lib.RB_OK
        assert L.rb_tune_set(1, 1, 1000, 2) == _lib.RB_OK
        f = tmp_path / "t.txt"
        f.write_text("1 1 9 3\n1 1 10 2\n")
        assert L.rb_tune_load(str(f).encode()) == 0
        rows, waves = C.c_int(), C.c_int()
        assert L.rb_tune_query(1, 1, 1000, C.byref(rows), C.byref(waves), None) == 0
        assert (rows.value, waves.value) == (2, 7)            # class 9: default kept
        assert L.rb_tune_query(1, 1, 1500, C.byref(rows), C.byref(waves), None) == 0
        assert (rows.value, waves.value) == (3, 5)            # class 10: loaded
    finally:
        assert L.rb_tune_load(str(empty).encode()) == 0

