"""AddressSanitizer and UndefinedBehaviorSanitizer runs of the CPU code.

The oracle's C part and the HIP library's host code (argument validation,
the exports, the host steps of the ladder initialisation) are built with
clang's sanitizers (the library's device code is compiled as usual) and
exercised by a selection of the CPU tests in a child process that preloads
clang's shared sanitizer runtime; any report fails the run (reports of
undefined behaviour are fatal).  A planted out-of-bounds read in a small
probe library, run the same way, shows that the runtime is live.
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"


def _runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/"
                             "libclang_rt.asan-x86_64.so"))
    if not found or not os.path.exists(CLANG):
        pytest.skip("clang sanitizer runtime not installed")
    return found[-1]


def _env(rt, **extra):
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               LD_LIBRARY_PATH="/opt/rocm/llvm/lib:" +
               env.get("LD_LIBRARY_PATH", ""), **extra)
    return env


def test_sanitizer_runtime_reports_a_planted_error(tmp_path):
    rt = _runtime()
    src = tmp_path / "probe.c"
    src.write_text(textwrap.dedent("""
        #include <stdlib.h>
        double probe(int i) {
          double* a = (double*)malloc(4 * sizeof(double));
          for (int k = 0; k < 4; ++k) a[k] = k;
          double v = a[i];   /* i = 4: one past the end */
          free(a);
          return v;
        }
    """))
    lib = tmp_path / "libprobe.so"
    subprocess.run([CLANG, "-O1", "-g", "-fsanitize=address,undefined",
                    "-shared-libsan", "-fPIC", "-shared", str(src), "-o",
                    str(lib)], check=True)
    code = ("import ctypes; L = ctypes.CDLL(%r); "
            "L.probe.restype = ctypes.c_double; print(L.probe(4))" % str(lib))
    r = subprocess.run([sys.executable, "-c", code], env=_env(rt),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr


@pytest.mark.slow
def test_cpu_code_under_sanitizers(tmp_path):
    rt = _runtime()
    sys.path.insert(0, ROOT)
    import oracle
    from paper_1507_03703_amd import build as hip_build
    olib = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    blib = hip_build.build_sanitized(str(tmp_path / "libbpmf_san.so"))
    tests = ["tests/test_abi.py", "tests/test_protocol_host.py",
             "tests/test_oracle_interp.py", "tests/test_oracle_forcefield.py",
             "tests/test_oracle_sampling.py", "tests/test_oracle_pairs.py"]
    # the child checks that the sanitized builds are the ones it loaded
    check = ("import oracle, paper_1507_03703_amd as p; oracle.lib(); "
             "p.library(); m = open('/proc/self/maps').read(); "
             "assert %r in m and %r in m, 'sanitized builds not loaded'"
             % (olib, blib))
    env = _env(rt, BPMF_ORACLE_LIB=olib, BPMF_LIB=blib)
    r = subprocess.run([sys.executable, "-c", check], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p",
                        "no:cacheprovider", "-m", "not gpu", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=1500)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for marker in ("AddressSanitizer", "runtime error:",
                   "LeakSanitizer", "UndefinedBehaviorSanitizer"):
        assert marker not in out, out[-4000:]
