"""The library's host runtime under AddressSanitizer and
UndefinedBehaviorSanitizer on a real device: paper_2211_12867_amd/icarus_san
(built by build.py from the library's sources and csrc/sanitize_driver.cpp,
host code instrumented, device code as usual) calls every C-ABI entry point
through a refined cone-CME run with two members, the tracer and combined
criterion, user-flag and plain regrids, checkpoint and restore, learned flags
with the judge, training and inference, and the error paths.  It must exit 0
with no sanitizer report (leaks of the HIP and HSA runtimes themselves are
suppressed; the library's own are not)."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2211_12867_amd", "icarus_san")


@pytest.mark.skipif(not os.path.exists(EXE), reason="icarus_san not built (paper_2211_12867_amd/build.py)")
def test_host_runtime_runs_clean_under_sanitizers(tmp_path):
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\nleak:libdrm\nleak:librocprofiler\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               LSAN_OPTIONS="suppressions=%s:print_suppressions=0" % supp, UBSAN_OPTIONS="print_stacktrace=1")
    print("running", EXE, flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, env=env, timeout=240)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout[-2000:], r.stderr[-6000:])
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
