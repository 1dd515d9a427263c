"""Sanitizer builds of the library's host code, run on the CPU.

- The event-file code (csrc/lhe.cpp, pure C++) with g++ under AddressSanitizer
  + UndefinedBehaviorSanitizer and, separately, ThreadSanitizer (the parse
  runs in parallel threads), linked to tests/sanitize/lhe_driver.cpp, which
  reads, sorts, exports, appends weights, writes, re-reads, and feeds the
  parser damaged copies.
- The whole library, its host-logic units instrumented (ASan + UBSan), linked
  to tests/sanitize/abi_driver.cpp (card and process parsing, the
  reweighting-card parser on damaged cards, the training order, the
  checkpoint reader).
Any memory error, undefined behaviour, leak or data race fails the test."""
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


def test_library_host_code_under_asan_ubsan(tmp_path):
    """The whole library (the units with host logic -- the C ABI, the
    surrogate's host side, the event files -- instrumented with
    AddressSanitizer and UndefinedBehaviorSanitizer, the kernel units as usual)
    linked to tests/sanitize/abi_driver.cpp, which runs the host-side paths
    without a GPU: process and SLHA parsing in rwgt_create (failing cleanly
    where it needs the device), the reweighting-card parser on valid and
    damaged cards, the training order and the checkpoint reader."""
    import concurrent.futures as cf
    from paper_2510_05100_amd import build as b
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/lib/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("hipcc / clang++ not available")
    flags = ["--offload-arch=gfx950", "-O3", "-Xarch_host", "-g", "-std=c++17", "-fPIC", "-I" + b.CSRC,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]
    srcs = [os.path.join(b.CSRC, s) for s in b.SOURCES] + [os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp")]

    host_units = ("rwgt_abi.cpp", "mlp_abi.cpp", "mlp_train.cpp", "lhe.cpp", "abi_driver.cpp")

    def compile_one(src):
        obj = tmp_path / (os.path.basename(src) + ".o")
        # instrument the units with host logic; the kernel units (launch wrappers and the host
        # instantiation of the generated code that counts its operations) build as usual
        f = flags if os.path.basename(src) in host_units else [x for x in flags if "sanitize" not in x and x != "-g"]
        f = [x for i, x in enumerate(f) if not (x == "-Xarch_host" and (i + 1 >= len(f) or f[i + 1] == "-Xarch_host"))]
        r = subprocess.run([hipcc] + f + ["-c", src, "-o", str(obj)], capture_output=True, text=True, timeout=900)
        assert r.returncode == 0, r.stderr[-3000:]
        return str(obj)
    with cf.ThreadPoolExecutor(min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = tmp_path / "abi_driver"
    link = [clang, "-fsanitize=address,undefined"] + objs + ["-o", str(exe), "-L/opt/rocm/lib", "-lamdhip64",
                                                             "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(link, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    print(run.stdout, run.stderr[-2000:])
    assert run.returncode == 0, run.stderr[-4000:]
    assert "failures 0" in run.stdout
