"""Sanitizer builds of the library's host-side event-file code (csrc/lhe.cpp,
pure C++): compiled with g++ under AddressSanitizer + UndefinedBehaviorSanitizer
and, separately, ThreadSanitizer (the parse runs in parallel threads), linked
to a driver (tests/sanitize/lhe_driver.cpp) that reads, sorts, exports,
appends weights, writes, re-reads, and feeds the parser damaged copies.  Any
memory error, undefined behaviour or data race aborts the driver.  CPU only."""
import os
import shutil
import subprocess

import pytest

from synth import lhe as slhe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "paper_2510_05100_amd", "csrc", "lhe.cpp"),
       os.path.join(ROOT, "tests", "sanitize", "lhe_driver.cpp")]
FLAGS = {
    "address,undefined": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
    "thread": ["-fsanitize=thread"],
}


@pytest.mark.parametrize("kind", list(FLAGS))
def test_lhe_code_under_sanitizers(kind, tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = tmp_path / "lhe_driver"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-pthread"] + FLAGS[kind] + SRC + ["-o", str(exe)]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-3000:]
    text, _ = slhe.lhe_text(n_per_process=(300, 250, 200, 50))
    src = tmp_path / "in.lhe"
    src.write_text(text)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", TSAN_OPTIONS="halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe), str(src), str(tmp_path / "out.lhe")], capture_output=True, text=True,
                         timeout=300, env=env)
    print(run.stdout, run.stderr[-2000:])
    assert run.returncode == 0, run.stderr[-4000:]
    assert "failures 0" in run.stdout
