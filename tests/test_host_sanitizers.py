"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The FP64 oracle (oracle/stl_oracle.c) and the plan compiler
(paper_2501_04194_amd/csrc/stl_compile.cpp: validation of the node array,
lowering, slot allocation, the longest-first order) are rebuilt with
gcc -fsanitize=address,undefined and driven from a child Python process that
preloads the ASan runtime: the oracle through its pin tests, the plan
compiler through the host tests of the C ABI (accepted formulas and every
error path).  A sanitizer report ends the child with a non-zero status."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
         "-fPIC", "-shared"]


@pytest.fixture(scope="module")
def sanitized():
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("gcc is not installed")
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's ASan runtime is not installed")
    d = tempfile.mkdtemp(prefix="stl_san_")
    oracle_lib = os.path.join(d, "liboracle_san.so")
    plan_lib = os.path.join(d, "libstlplan_san.so")
    subprocess.check_call(["gcc"] + FLAGS + ["-fopenmp", "-o", oracle_lib, os.path.join(ROOT, "oracle", "stl_oracle.c"),
                                             "-lm"])
    subprocess.check_call(["g++", "-std=c++17"] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-o", plan_lib,
                                                           os.path.join(ROOT, "paper_2501_04194_amd", "csrc",
                                                                        "stl_compile.cpp")])
    yield {"asan": asan, "oracle": oracle_lib, "plan": plan_lib}
    shutil.rmtree(d, ignore_errors=True)


def _child(args, san, extra_env):
    env = dict(os.environ, LD_PRELOAD=san["asan"], ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2", **extra_env)
    r = subprocess.run([sys.executable] + args, env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out
    assert r.returncode == 0, out
    return out


def test_oracle_pins_under_sanitizers(sanitized):
    out = _child(["-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu", "tests/test_oracle_pins.py"],
                 sanitized, {"STL_ORACLE_LIB": sanitized["oracle"]})
    assert " passed" in out


PLAN_CHILD = r"""
import ctypes, os, sys
sys.path.insert(0, "tests")
from paper_2501_04194_amd import stl
stl._lib = stl._bind(ctypes.CDLL(os.environ["STL_PLAN_LIB"]))
import test_lib_host as T
names = ["test_compile_accepts_benchmark_formulas", "test_compile_error_paths",
         "test_nary_more_than_four_children_compiles", "test_lpt_order", "test_param_vector_layout",
         "test_compile_coefficient_budget"]
for n in names:
    getattr(T, n)()
    print("ok", n)
print("PLAN-COMPILER-OK")
"""


def test_plan_compiler_under_sanitizers(sanitized):
    out = _child(["-c", PLAN_CHILD], sanitized, {"STL_PLAN_LIB": sanitized["plan"]})
    assert "PLAN-COMPILER-OK" in out
