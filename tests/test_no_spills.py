"""No kernel of the library spills registers to scratch memory.

A spill turns every register the compiler could not hold into a store and a
reload per unit of work (scratch traffic that the sweeps' roofline does not
count), and it tends to creep in when a sweep variant gains a few live
values.  This reads the code-object metadata of the built objects (the
device half of each ``_build/*.hip.o``) and checks each kernel's private
segment size.  CPU only: it needs the build, not a GPU.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2411_09809_amd import build

LLVM = "/opt/rocm/llvm/bin"
TOOLS = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]


def _kernels(obj, tmp):
    """(kernel name, private segment bytes) of one object's gfx950 code."""
    fat = os.path.join(tmp, os.path.basename(obj) + ".fatbin")
    co = os.path.join(tmp, os.path.basename(obj) + ".co")
    subprocess.run([TOOLS[0], f"--dump-section=.hip_fatbin={fat}", obj,
                    os.path.join(tmp, "stripped.o")], check=True, capture_output=True)
    subprocess.run([TOOLS[1], "--unbundle", "--type=o",
                    f"--targets=hipv4-amdgcn-amd-amdhsa--{build.ARCH}", f"--input={fat}",
                    f"--output={co}"], check=True, capture_output=True)
    notes = subprocess.run([TOOLS[2], "--notes", co], check=True, capture_output=True,
                           text=True).stdout
    out, name = [], None
    for line in notes.splitlines():
        m = re.match(r"\s+\.name:\s+(\S+)", line)
        if m:
            name = m.group(1)
        m = re.match(r"\s+\.private_segment_fixed_size:\s+(\d+)", line)
        if m and name is not None:
            out.append((name, int(m.group(1))))
            name = None
    return out


def test_no_kernel_uses_scratch(tmp_path):
    if not all(os.path.exists(t) for t in TOOLS):
        pytest.skip("ROCm LLVM tools not found")
    objs = sorted(os.path.join(build.OBJ, f) for f in os.listdir(build.OBJ)
                  if f.endswith(".hip.o")) if os.path.isdir(build.OBJ) else []
    if not objs:
        pytest.fail("no built objects: run paper_2411_09809_amd.build.build() first")
    seen, spilled = 0, []
    for obj in objs:
        with open(obj, "rb") as fh:
            if b"__CLANG_OFFLOAD_BUNDLE__" not in fh.read():
                continue                          # host-only source (no kernels)
        ks = _kernels(obj, str(tmp_path))
        seen += len(ks)
        spilled += [(os.path.basename(obj), n, b) for n, b in ks if b]
    assert seen >= 50, seen                       # every sweep, pass and reduction
    assert not spilled, spilled
    shutil.rmtree(tmp_path, ignore_errors=True)
