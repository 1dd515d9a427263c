"""Device bounds checks: the check build of the library (librwgt_check.so,
-DRWGT_CHECK) compares every global-memory index of the matrix-element,
ingest, cross-section, factored, running-alpha_s, non-finite-count, batched
and card-per-event kernels with its array's extent and counts the misses
instead of making the access.  tests/bounds_workload.py drives each of those
kernels with ragged sizes in a child process that loads the check build
(RWGT_LIBRARY=check); every step must report zero indices out of range, and
the checked FP64 g g -> t t~ g g |M|^2 must still match the oracle (1e-10).
The normal build compiles the checks away: there rwgt_bounds_check reports
enabled = 0 and no misses.
"""
import os
import subprocess
import sys

import pytest

from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_normal_build_reports_no_checks():
    import paper_2510_05100_amd as rw
    torch_cuda()
    assert rw.rwgt_bounds_check() == (False, 0)


def test_check_build_finds_no_index_out_of_range():
    lib = os.path.join(os.path.dirname(HERE), "paper_2510_05100_amd", "librwgt_check.so")
    if not os.path.exists(lib):
        pytest.fail("librwgt_check.so is missing: build it with `python -m paper_2510_05100_amd.build --check`")
    print("[case] bounds-checked library, every checked kernel", flush=True)
    env = dict(os.environ, RWGT_LIBRARY="check")
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "bounds_workload.py")], env=env,
                       capture_output=True, text=True, timeout=240)
    print(r.stdout[-4000:])
    print(r.stderr[-2000:])
    assert r.returncode == 0, "bounds check found indices out of range (or the child failed)"
    assert "bounds check clean" in r.stdout
