"""Build librwgt.so in-tree for gfx950: generate the per-process headers, then
compile every translation unit with hipcc in parallel and link.  With
check=True, the bounds-checked variant librwgt_check.so (-DRWGT_CHECK: every
global-memory index of the device kernels compared with its array's extent)
from the same sources, into its own object folder.

    python -m paper_2510_05100_amd.build [--jobs N] [--verbose] [--check]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librwgt.so")
OBJ_CHECK = os.path.join(HERE, "_build_check")
LIB_CHECK = os.path.join(HERE, "librwgt_check.so")
ARCH = "gfx950"

SOURCES = ["kernels.hip", "proc_ee_mumu.hip", "proc_uu_eeg.hip", "proc_gg_ttgg.hip", "proc_gg_tttt.hip", "batch.hip", "mlp.hip", "mlp_abi.cpp", "mlp_train.cpp", "rwgt_abi.cpp", "lhe.cpp"]

# -packed-fp32-ops: no v_pk_{add,mul,fma}_f32 in generated code.
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-I" + CSRC,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _newest_input(src):
    paths = [os.path.join(CSRC, src)]
    for root, _, files in os.walk(CSRC):
        paths += [os.path.join(root, f) for f in files if f.endswith(".h")]
    paths.append(os.path.join(os.path.dirname(CSRC), "..", "include", "rwgt.h"))
    return max(os.path.getmtime(p) for p in paths if os.path.exists(p))


def _compile(src, verbose, incremental=False, check=False):
    obj = os.path.join(OBJ_CHECK if check else OBJ, os.path.splitext(src)[0] + ".o")
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > _newest_input(src):
        return obj
    cmd = [hipcc()] + HIP_FLAGS + (["-DRWGT_CHECK"] if check else []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    t0 = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        errors = "\n".join(ln for ln in res.stderr.splitlines() if " error:" in ln or ln.startswith("error"))
        raise RuntimeError(f"hipcc failed for {src}:\n{errors}\n{res.stderr[-2000:]}")
    if verbose:
        print(f"  {src}: {time.time() - t0:.1f}s", flush=True)
    return obj


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False, check: bool = False) -> str:
    """Compile every source (or, with incremental=True, those whose inputs
    changed) and link librwgt.so (check=True: librwgt_check.so)."""
    from .procgen.__main__ import main as procgen_main
    procgen_main(os.path.join(CSRC, "generated"))
    lib = LIB_CHECK if check else LIB
    os.makedirs(OBJ_CHECK if check else OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, incremental, check), SOURCES))
    tmp = lib + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-4000:]}")
    os.replace(tmp, lib)
    return lib


def build_all(jobs: int | None = None, verbose: bool = False) -> tuple:
    """Both libraries (librwgt.so and librwgt_check.so), their translation
    units compiled in one pool, longest first."""
    from .procgen.__main__ import main as procgen_main
    procgen_main(os.path.join(CSRC, "generated"))
    os.makedirs(OBJ, exist_ok=True)
    os.makedirs(OBJ_CHECK, exist_ok=True)
    slow = ["proc_gg_ttgg.hip", "proc_gg_tttt.hip", "mlp.hip"]             # the longest compiles start first
    order = slow + [s for s in SOURCES if s not in slow]
    tasks = [(s, c) for s in order for c in (False, True)]
    jobs = jobs or (os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda t: _compile(t[0], verbose, False, t[1]), tasks))
    out = []
    for check in (False, True):
        lib = LIB_CHECK if check else LIB
        mine = [o for (s, c), o in zip(tasks, objs) if c == check]
        tmp = lib + ".tmp"
        cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + mine
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed:\n{res.stderr[-4000:]}")
        os.replace(tmp, lib)
        out.append(lib)
    return tuple(out)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--incremental", action="store_true", help="recompile only changed translation units")
    ap.add_argument("--check", action="store_true", help="the bounds-checked library librwgt_check.so")
    a = ap.parse_args()
    t = time.time()
    print(build(a.jobs, a.verbose, a.incremental, a.check), f"({time.time() - t:.0f}s)")
    sys.exit(0)
