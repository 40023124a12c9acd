"""AddressSanitizer / UndefinedBehaviorSanitizer build of the oracle's C core
(test infrastructure: the C core is what the GPU path is checked against).
oracle/sanitize_driver.c runs every entry point on patches whose arrays have
exactly their documented sizes (spherical and cartesian, 8 and 9 variables,
every limiter, odd and one-cell interiors); the build must run clean.  A
planted heap overrun and a planted signed overflow must be caught, so the
check cannot pass on an uninstrumented build.  (It found ora_rhs
reading face fluxes through a NULL buffer that its contract allowed.)"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-ffp-contract=off"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")


def _build(tmp_path, sources, name, flags=FLAGS):
    exe = str(tmp_path / name)
    subprocess.run(["gcc"] + flags + sources + ["-lm", "-o", exe], check=True, capture_output=True, text=True)
    return exe


def test_oracle_core_runs_clean_under_asan_and_ubsan(tmp_path):
    exe = _build(tmp_path, [os.path.join(ROOT, "oracle", "oracle.c"),
                            os.path.join(ROOT, "oracle", "sanitize_driver.c")], "ora_san")
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-4000:]


def test_the_sanitizers_catch_planted_errors(tmp_path):
    """An overrun of a heap array (AddressSanitizer alone) and a signed
    overflow (UndefinedBehaviorSanitizer alone) fail their runs."""
    src = tmp_path / "overrun.c"
    src.write_text("#include <stdlib.h>\nint main(void) { double *a = malloc(4 * sizeof(double));\n"
                   "  a[0] = 1.0; volatile int i = 4; double x = a[i]; free(a); return x > 0; }\n")
    exe = _build(tmp_path, [str(src)], "overrun", ["-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer"])
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=60)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
    src = tmp_path / "overflow.c"
    src.write_text("int main(void) { volatile int i = 2147483647; int j = i + 1; return j == 0; }\n")
    exe = _build(tmp_path, [str(src)], "overflow", ["-O1", "-g", "-fsanitize=undefined", "-fno-sanitize-recover=all"])
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=60)
    assert r.returncode != 0 and "signed integer overflow" in r.stderr
