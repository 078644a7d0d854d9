"""The CPU reference, the property checker and the input generator under
AddressSanitizer and UndefinedBehaviorSanitizer (host code only, no GPU).

Sanitizer copies of the three host libraries are built (``*_san.so``), and
the CPU tests that exercise them run again in a child process that loads
those copies (KBISIM_SANITIZE=1) with the ASan runtime preloaded.  Any
out-of-bounds access, use after free or undefined behaviour aborts the child.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

import pytest

import graphgen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    gcc = shutil.which("gcc")
    if not gcc:
        return None
    path = subprocess.run([gcc, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(900)
def test_cpu_suite_under_asan_and_ubsan():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no ASan runtime next to gcc")
    graphgen.build(force=False, sanitize=True)
    oracle.build(force=False, sanitize=True)
    env = dict(os.environ)
    env.update(KBISIM_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:detect_odr_violation=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS=env.get("OMP_NUM_THREADS", "4"))
    probe = ("import graphgen, oracle\n"
             "g = graphgen.tiny(seed=1, n=500, m=2000)\n"
             "oracle.refine(g, 2); oracle.check_step(g, *oracle.refine(g, 2)[0])\n"
             "maps = open('/proc/self/maps').read()\n"
             "print(all(x in maps for x in ('liboracle_san.so', 'libstepcheck_san.so', 'libgraphgen_san.so',\n"
             "                                'libasan')))\n")
    res = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True)
    assert res.returncode == 0 and res.stdout.strip() == "True", (res.stdout + res.stderr)[-2000:]
    tests = ["tests/test_oracle.py", "tests/test_stepcheck.py", "tests/test_summary_oracle.py",
             "tests/test_serve_scheduler.py"]
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                          "-o", "addopts="] + tests, cwd=ROOT, env=env, capture_output=True, text=True)
    tail = (res.stdout + res.stderr)[-4000:]
    assert res.returncode == 0, tail
    assert "passed" in res.stdout and "error" not in res.stdout.lower().split("passed")[-1], tail
