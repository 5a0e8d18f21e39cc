"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): the pins of test_oracle_pins.py run again in a child process
against a sanitizer build of oracle.c, and a planted out-of-bounds read in
a small C file built with the same flags shows that the checking build
reports such mistakes."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("no ASan runtime for gcc")
    return path


def _san_env(lib):
    env = dict(os.environ)
    env.update({"LD_PRELOAD": _asan_runtime(), "ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "print_stacktrace=1",
                "MMM_ORACLE_LIB": lib, "OMP_NUM_THREADS": "4"})
    return env


def test_sanitizer_build_reports_a_planted_overflow(tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build

    src = tmp_path / "planted.c"
    src.write_text("#include <stdlib.h>\n"
                   "int main(void) { volatile double* a = malloc(4 * sizeof(double));\n"
                   "  double s = 0.0; for (int i = 0; i <= 4; ++i) s = s + a[i]; free((void*)a); return s > 1; }\n")
    exe = tmp_path / "planted"
    subprocess.run(["gcc", *build.SAN_FLAGS, "-o", str(exe), str(src)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    # either sanitizer may stop the run first: UBSan (a load with no room for
    # the object) or ASan (heap-buffer-overflow)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr or "runtime error: load of address" in r.stderr, r.stderr[-2000:]


def test_oracle_pins_under_asan_and_ubsan():
    sys.path.insert(0, ROOT)
    from oracle import build

    lib = build.build(sanitize=True)
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-x", "-q",
                        "-p", "no:cacheprovider"], capture_output=True, text=True, env=_san_env(lib), cwd=ROOT,
                       timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
