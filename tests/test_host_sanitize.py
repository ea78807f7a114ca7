"""The library's host code under AddressSanitizer + UndefinedBehaviorSanitizer
and ThreadSanitizer, on the CPU.

The host sources (network builder, orders, plan compiler, batch planner, C
ABI) are compiled with g++ and the sanitizer, with the device entry points
replaced by "no device" stubs (tests/sanitize/device_stubs.cpp), and loaded
into a Python process that builds, orders (16 host threads, 128 line-graph
restarts per network) and batch-plans the 5-regular p=2 batching batches —
where heap-corruption aborts were once seen on the GPU machine — and more. Any
sanitizer report fails the test.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1709_03636_amd", "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("build.cpp", "order.cpp", "plan.cpp", "api.cpp", "bplan.cpp")] + \
          [os.path.join(ROOT, "tests", "sanitize", "device_stubs.cpp")]
REPORTS = ("ERROR: AddressSanitizer", "WARNING: ThreadSanitizer", "runtime error:", "ERROR: LeakSanitizer")

pytestmark = pytest.mark.slow


def _build(out_dir, flags):
    os.makedirs(out_dir, exist_ok=True)

    def one(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC",
                        "-I" + os.path.join(ROOT, "include")] + flags + ["-c", src, "-o", obj], check=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(one, SOURCES))
    lib = os.path.join(out_dir, "libqtn_host.so")
    subprocess.run(["g++", "-shared"] + flags + objs + ["-o", lib], check=True)
    return lib


def _runtime(name):
    return subprocess.run(["g++", "-print-file-name=" + name], capture_output=True, text=True, check=True).stdout.strip()


def _plan(lib, preload, cases, extra_env):
    env = dict(os.environ, QTN_LIB=lib, LD_PRELOAD=preload, **extra_env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize", "plan_grid.py")] + cases,
                       capture_output=True, text=True, env=env, timeout=900)
    text = r.stdout + r.stderr
    assert r.returncode == 0, text[-4000:]
    assert r.stdout.strip().endswith("ok"), text[-4000:]
    for rep in REPORTS:
        assert rep not in text, text[-4000:]
    return r.stdout


def test_planning_under_address_and_undefined_sanitizers(tmp_path):
    lib = _build(str(tmp_path / "asan"), ["-fsanitize=address,undefined"])
    out = _plan(lib, _runtime("libasan.so"), ["5,50,2", "5,100,2", "4,50,2", "3,60,2"],
                {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
                 "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    assert out.count("\n") >= 8


def test_threaded_planning_under_thread_sanitizer(tmp_path):
    lib = _build(str(tmp_path / "tsan"), ["-fsanitize=thread"])
    _plan(lib, _runtime("libtsan.so"), ["5,50,2"], {"TSAN_OPTIONS": "halt_on_error=1:report_signal_unsafe=0"})
