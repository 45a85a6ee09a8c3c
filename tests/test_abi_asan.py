"""The C ABI's host-side validation under AddressSanitizer: the ABI tests
(tests/test_abi_cpu.py, which never reach a device) run in a child process
against the host-instrumented build of the library with the sanitizer
runtime preloaded; any heap or stack error in the host code aborts the
child.  CPU only."""

from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_tests_under_host_asan():
    sys.path.insert(0, ROOT)
    from paper_1403_6968_amd import build_asan, build_lib
    rt = build_asan.asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime next to hipcc")
    srcs = [os.path.join(build_lib.CSRC, f) for f in os.listdir(build_lib.CSRC)] + \
        [os.path.join(ROOT, "include", "linview.h")]
    if not os.path.exists(build_asan.LIB) or os.path.getmtime(build_asan.LIB) < max(map(os.path.getmtime, srcs)):
        build_asan.build()
    env = dict(os.environ)
    env.update({"LINVIEW_LIBRARY": build_asan.LIB, "LD_PRELOAD": rt,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
                "HIP_VISIBLE_DEVICES": "", "PYTHONPATH": ROOT})
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=600)
    tail = "\n".join(p.stdout.splitlines()[-30:])
    assert p.returncode == 0, f"ABI tests under AddressSanitizer failed:\n{tail}"
    assert "AddressSanitizer" not in p.stdout, tail
    assert " passed" in tail
