"""The host code of libqtt under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is built a second time with the host pass instrumented
(_build/san/libqtt.so; the device code is compiled as usual) and the CPU ABI
tests -- argument validation, workspace planning of every entry point, shape
errors, rank-bound queries -- run against it in a child process with the
sanitizer runtime preloaded.  Any report fails the test.  No GPU is used.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sanitized_library():
    from paper_2602_20226_amd import build as B
    srcs = B.sources() + [os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC) if f.endswith((".hpp", ".h"))]
    srcs.append(os.path.join(ROOT, "include", "qtt.h"))
    newest = max(os.path.getmtime(p) for p in srcs)
    if not os.path.exists(B.SAN_LIB) or os.path.getmtime(B.SAN_LIB) < newest:
        B.build_sanitized(verbose=False)
    return B.SAN_LIB, B.sanitizer_runtime()


@pytest.mark.timeout(900)
def test_host_code_clean_under_address_and_ub_sanitizers():
    try:
        lib, rt = _sanitized_library()
    except (FileNotFoundError, RuntimeError) as e:
        pytest.skip(f"sanitizer build unavailable here: {e}")
    nm = subprocess.run(["nm", "-D", lib], capture_output=True, text=True)
    assert "__asan" in nm.stdout and "__ubsan" in nm.stdout, "library is not instrumented"
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "QTT_LIBRARY": lib,
    })
    probe = ("import os, paper_2602_20226_amd.qtt as Q; L = Q.load_library(); "
             "maps = open('/proc/self/maps').read(); "
             "assert Q.LIB_PATH == os.environ['QTT_LIBRARY'] and 'libclang_rt.asan' in maps; print('instrumented')")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "instrumented" in r.stdout, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_abi.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
