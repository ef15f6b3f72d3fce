"""CPU: the oracle's C loops and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer.

* oracle/ref.c is rebuilt with gcc's sanitizers and every oracle pin (tests/test_oracle_pins.py)
  runs against it in a child process (ORACLE_LIBRARY selects the build, the gcc runtimes are
  preloaded into the uninstrumented interpreter);
* libspx is rebuilt with the sanitizers on its host code only (device code is unchanged) and the
  C-ABI checks (tests/test_abi_cpu.py: exports, status strings, every argument error path of
  conversion, products, export, batches and the server) run against it with clang's runtime
  preloaded.
Leak detection is off: the interpreter and the HIP runtime keep allocations until exit."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True,
                       check=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip("gcc has no %s" % name)
    return p


def _run_child(args, env_extra):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider"] + args,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                           "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-fopenmp", "-shared",
                           "-std=c11", os.path.join(ROOT, "oracle", "ref.c"), "-o", lib, "-lm"])
    pre = _gcc_runtime("libasan.so") + ":" + _gcc_runtime("libubsan.so")
    out = _run_child([os.path.join("tests", "test_oracle_pins.py")],
                     {"ORACLE_LIBRARY": lib, "LD_PRELOAD": pre})
    assert " passed" in out


def test_abi_host_code_under_asan_ubsan(tmp_path):
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts:
        pytest.skip("no clang AddressSanitizer runtime")
    sys.path.insert(0, ROOT)
    from paper_2502_19284_amd import build as spx_build
    lib = spx_build.build(lib=str(tmp_path / "libspx_san.so"),
                          extra_flags=["-Xarch_host", "-fsanitize=address", "-Xarch_host",
                                       "-fsanitize=undefined", "-Xarch_host",
                                       "-fno-omit-frame-pointer"])
    nm = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan" in nm and "__ubsan" in nm   # the host code is instrumented
    out = _run_child([os.path.join("tests", "test_abi_cpu.py")],
                     {"SPX_LIBRARY": lib, "LD_PRELOAD": rts[-1]})
    assert " passed" in out
