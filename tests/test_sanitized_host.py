"""The host code of librb under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds the host-sanitized library (paper_2411_09809_amd.build.build_sanitized:
the same sources, host code instrumented, device code not) and runs the
no-GPU tests of the C ABI -- symbol exports, argument errors, workspace
checks, the tuning table and its files, fault injection -- against it in a
subprocess with the sanitizer runtime preloaded.  Any sanitizer report ends
that process with an error.  No GPU is used.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def san_env():
    sys.path.insert(0, ROOT)
    from paper_2411_09809_amd import build
    lib = build.build_sanitized()
    env = dict(os.environ)
    env.update(RB_LIBRARY=lib, LD_PRELOAD=build.sanitizer_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("RB_FAULT", None)
    return env, lib


def test_sanitized_library_is_the_one_loaded(san_env):
    env, lib = san_env
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2411_09809_amd import _lib\n"
            "_lib.lib()\n"
            "maps = open('/proc/self/maps').read()\n"
            "print('librb_san' in maps, 'libclang_rt.asan' in maps)\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split() == ["True", "True"], r.stdout


def test_abi_and_fault_paths_under_sanitizers(san_env):
    env, _ = san_env
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", "test_abi.py"),
                        os.path.join(ROOT, "tests", "test_fault.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
