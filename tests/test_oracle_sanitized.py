"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C source is compiled with gcc's -fsanitize=address,undefined (every report is
fatal) into a temporary library, and the oracle's pin tests run against it in a child
process with the ASan runtime preloaded: an out-of-bounds access, a use after free, a
signed overflow or a misaligned load anywhere the pins drive the oracle ends the run.  A
tiny program with a planted heap overflow first shows that the sanitizer build reports.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.c")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _runtime(name):
    out = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    path = os.path.realpath(out)
    return path if os.path.isabs(out) and os.path.exists(path) else None


def _env(lib):
    asan = _runtime("libasan.so")
    pre = os.environ.get("LD_PRELOAD", "")
    return dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan + (":" + pre if pre else ""),
                ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


@pytest.fixture(scope="module")
def sanitizer():
    if _runtime("libasan.so") is None or _runtime("libubsan.so") is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    return True


def test_sanitizer_build_reports_a_planted_overflow(sanitizer, tmp_path):
    src = tmp_path / "overflow.c"
    src.write_text("#include <stdlib.h>\nint main(void) { volatile int* a = malloc(4 * sizeof(int));"
                   " a[4] = 1; int r = a[0]; free((void*)a); return r; }\n")
    exe = tmp_path / "overflow"
    subprocess.check_call(["gcc"] + SAN + ["-o", str(exe), str(src)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode != 0 and ("heap-buffer-overflow" in r.stderr or "runtime error:" in r.stderr)


def test_oracle_pins_under_sanitizers(sanitizer, tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc"] + SAN + ["-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE", "-o", lib,
                                           SRC, "-lm"])
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=_env(lib), capture_output=True, text=True, timeout=900)
    tail = r.stdout[-3000:] + r.stderr[-3000:]
    print(r.stdout[-400:])
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail
    assert " passed" in r.stdout
