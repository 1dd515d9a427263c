"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/rwgt.h, and rejects bad arguments before touching a
device."""
import ctypes
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2510_05100_amd", "librwgt.so")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rwgt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rwgt_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("librwgt.so not built (python -m paper_2510_05100_amd.build)")
    from paper_2510_05100_amd import _abi
    return _abi.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("rwgt_create", "rwgt_eval", "rwgt_destroy", "rwgt_me2", "rwgt_param_layout", "rwgt_set_stream"):
        assert must in names


def test_every_declared_symbol_exported(lib):
    from paper_2510_05100_amd import _abi
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _abi.SIGNATURES, name


def test_check_build_exports_the_same_symbols(lib):
    """The bounds-checked build (librwgt_check.so) exports the same boundary;
    the normal build reports the checks compiled away (enabled 0, no misses,
    without touching a device) and rejects NULL arguments."""
    path = os.path.join(ROOT, "paper_2510_05100_amd", "librwgt_check.so")
    if not os.path.exists(path):
        pytest.skip("librwgt_check.so not built (python -m paper_2510_05100_amd.build --check)")
    chk = ctypes.CDLL(path)
    for name in declared_functions():
        assert hasattr(chk, name), name
    en, n = ctypes.c_int32(-1), ctypes.c_uint64(7)
    assert lib.rwgt_bounds_check(ctypes.byref(en), ctypes.byref(n)) == 0
    assert (en.value, n.value) == (0, 0)
    assert lib.rwgt_bounds_check(None, ctypes.byref(n)) == -1


def test_create_rejects_bad_arguments(lib):
    from paper_2510_05100_amd import _abi
    out = ctypes.c_void_p()
    card = synth.ORIG_QCD.slha().encode()
    assert lib.rwgt_create(None, card, 0, ctypes.byref(out)) == -1
    assert lib.rwgt_create(b"g g > t t~ g g", card, 7, ctypes.byref(out)) == -1
    assert lib.rwgt_create(b"g g > t t~", card, 0, ctypes.byref(out)) == -2
    assert b"unsupported process" in lib.rwgt_create_error()
    assert lib.rwgt_create(b"g g > t t~ g g", b"BLOCK MASS\n 6 173\n", 0, ctypes.byref(out)) == -3
    assert b"SMINPUTS 3" in lib.rwgt_create_error()
    assert lib.rwgt_create(b"g g > t t~ g g", b"6 173\n", 0, ctypes.byref(out)) == -3
    assert lib.rwgt_create(b"e+ e- > mu+ mu-", b"BLOCK SMINPUTS\n 1 x\n", 0, ctypes.byref(out)) == -3
    assert out.value is None
    with pytest.raises(_abi.RwgtError, match="EPROCESS"):
        _abi.rwgt_create("u u~ > mu+ mu-", card.decode())
    lib.rwgt_destroy(None)                      # NULL is a no-op
    assert lib.rwgt_last_error(None) == b"context is NULL"


def test_null_context_calls(lib):
    assert lib.rwgt_eval(None, None, 0, None, None, 1, None) == -1
    assert lib.rwgt_me2(None, None, 0, None, 1, None) == -1
    assert lib.rwgt_set_stream(None, None) == -1
    n = ctypes.c_int32()
    assert lib.rwgt_param_layout(None, ctypes.byref(n), None) == -1


def test_generated_process_constants():
    # the process compiler reproduces the diagram, flow and helicity counts
    from paper_2510_05100_amd.procgen import diagrams, emit
    for name, text, ndiag, namp, ncol, ngood in [
        ("ee_mumu", "e+ e- > mu+ mu-", 2, 2, 1, 4),
        ("uu_eeg", "u u~ > e+ e- g", 4, 4, 1, 8),
        ("gg_ttgg", "g g > t t~ g g", 123, 159, 24, 64),
    ]:
        d = diagrams.build(diagrams.parse(name, text))
        assert (d.n_diagrams, len(d.terms), len(d.basis)) == (ndiag, namp, ncol)
        assert len(emit.good_helicities(d)) == ngood


def test_procgen_colour_matrix_matches_bruteforce():
    # symbolic Fierz reduction (device side) against the oracle's brute force
    import numpy as np
    from oracle import colour as oc
    from paper_2510_05100_amd.procgen import diagrams, emit
    d = diagrams.build(diagrams.parse("gg_ttgg", "g g > t t~ g g"))
    num, den = emit.colour_matrix_ints(d)
    assert den == 54
    sym = np.array(num, dtype=float) / den
    brute = oc.colour_matrix(4).real          # same basis order: permutations of the 4 gluon slots
    np.testing.assert_allclose(sym, brute, atol=1e-12)
    for name, text, want in [("ee_mumu", "e+ e- > mu+ mu-", [[1]]), ("uu_eeg", "u u~ > e+ e- g", [[4]])]:
        num, den = emit.colour_matrix_ints(diagrams.build(diagrams.parse(name, text)))
        assert np.allclose(np.array(num) / den, want)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: any other --gpus exits with status 2 and a
    message, before generating events or touching a device."""
    import subprocess
    import sys
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU only" in res.stderr and res.stdout == ""


def test_train_order_is_a_permutation_per_epoch(lib):
    """rwgt_train_order: every (seed, epoch) gives a bijection of [0, n), for n
    just above a power of four (the cycle walk then rejects most of the
    Feistel word space) and for the 4e6-pair training grid; another epoch or
    seed gives another order; a window equals the same slice of the whole."""
    import numpy as np
    from paper_2510_05100_amd import _abi
    for n in (1, 2, 3, 17, 4097, 65537):
        for epoch in (0, 5):
            o = _abi.rwgt_train_order(11, epoch, n)
            np.testing.assert_array_equal(np.sort(o), np.arange(n))
    full = _abi.rwgt_train_order(1, 0, 4_000_000)
    np.testing.assert_array_equal(np.sort(full), np.arange(4_000_000))
    assert not np.array_equal(full[:1000], _abi.rwgt_train_order(1, 1, 4_000_000, 0, 1000))
    assert not np.array_equal(full[:1000], _abi.rwgt_train_order(2, 0, 4_000_000, 0, 1000))
    np.testing.assert_array_equal(_abi.rwgt_train_order(1, 0, 4_000_000, 123_456, 4096), full[123_456:127_552])
    # a shuffle, not a shift: consecutive positions land far apart in the grid
    assert np.median(np.abs(np.diff(full[:4096]))) > 1e5
    assert lib.rwgt_train_order(1, 0, 10, 5, 6, None) == -1
    with pytest.raises(_abi.RwgtError):
        _abi.rwgt_train_order(1, 0, 10, 5, 6)


def test_checkpoint_reader_rejects_bad_files(lib, tmp_path):
    """rwgt_mlp_checkpoint_info reads on the host only: a missing file is
    EINVAL, a file without the magic, a truncated one and one with a flipped
    byte are ECARD, with a message naming the cause."""
    from paper_2510_05100_amd import _abi
    with pytest.raises(_abi.RwgtError, match="EINVAL"):
        _abi.rwgt_mlp_checkpoint_info(str(tmp_path / "missing.ckpt"))
    junk = tmp_path / "junk.ckpt"
    junk.write_bytes(b"not a checkpoint at all, just text")
    with pytest.raises(_abi.RwgtError, match="not a surrogate checkpoint"):
        _abi.rwgt_mlp_checkpoint_info(str(junk))
    fake = tmp_path / "fake.ckpt"
    fake.write_bytes(b"RWGTMLP\0" + bytes(200))
    with pytest.raises(_abi.RwgtError, match="hash mismatch"):
        _abi.rwgt_mlp_checkpoint_info(str(fake))
    with pytest.raises(_abi.RwgtError, match="ECARD"):
        _abi.rwgt_mlp_load(str(fake))
    assert lib.rwgt_mlp_load(None, None) == -1
