"""Event files on the host (no GPU): the library's LHE reader, process sort,
momentum export and writer, and the reweighting-card parser, against the
plain reader in oracle/lhe.py and against the known contents of seeded files
(synth/lhe.py writes them from known momenta and weights).  All of this is
parsing and copying: every comparison is exact."""
import numpy as np
import pytest

import synth
from oracle import lhe as olhe
from synth import lhe as slhe

PROC = {"ee_mumu": "e+ e- > mu+ mu-", "uu_eeg": "u u~ > e+ e- g", "gg_ttgg": "g g > t t~ g g"}


def _rw():
    import paper_2510_05100_amd as rw
    try:
        rw.load()
    except OSError as ex:                     # the library is not built
        pytest.skip(str(ex))
    return rw


def _canonical(mom, process):
    """Momenta with the slots of identical particles put in a fixed order (the
    two incoming or the two final gluons of g g > t t~ g g can be matched
    either way; |M|^2 is symmetric under their exchange)."""
    mom = np.array(mom, dtype=np.float64)
    rows = mom.reshape((-1,) + mom.shape[-2:])
    sl = olhe.slots(process)
    for key in set(sl):
        pos = [i for i, k in enumerate(sl) if k == key]
        if len(pos) < 2:
            continue
        for r in rows:
            sub = r[pos].copy()
            r[pos] = sub[np.lexsort(sub.T[::-1])]
    return rows.reshape(mom.shape)


@pytest.fixture(scope="module")
def sample(tmp_path_factory):
    text, truth = slhe.lhe_text()
    path = tmp_path_factory.mktemp("lhe") / "in.lhe"
    path.write_text(text)
    return path, text, truth


def test_oracle_reader_reproduces_the_written_contents(sample):
    """Pin of the oracle reader: the generator's own momenta and weights."""
    _, text, truth = sample
    ev = olhe.read(text)
    assert len(ev) == len(truth)
    for e, (key, p, xw) in zip(ev, truth):
        assert e["info"][0] == xw
        if key in PROC:
            np.testing.assert_array_equal(_canonical(olhe.momenta(e, PROC[key]), PROC[key]),
                                          _canonical(p, PROC[key]))
        else:
            assert all(olhe.match(e, pr) is None for pr in PROC.values())


def test_library_reader_sort_and_momenta(sample):
    rw = _rw()
    path, text, truth = sample
    ev = olhe.read(text)
    lhe = rw.rwgt_lhe_read(path)
    try:
        assert rw.rwgt_lhe_num_events(lhe) == len(truth)
        for i in (0, 1, len(ev) // 2, len(ev) - 1):
            nup, idp, info = rw.rwgt_lhe_event_info(lhe, i)
            assert (nup, idp, info) == (ev[i]["nup"], ev[i]["idprup"], ev[i]["info"])
        allidx = np.arange(len(ev))
        np.testing.assert_array_equal(rw.rwgt_lhe_info(lhe, allidx), np.array([e["info"] for e in ev]))
        for key, proc in PROC.items():
            idx = rw.rwgt_lhe_select(lhe, proc)
            want = [i for i, t in enumerate(truth) if t[0] == key]
            np.testing.assert_array_equal(idx, want)
            mom, w = rw.rwgt_lhe_momenta(lhe, proc, idx)
            np.testing.assert_array_equal(_canonical(mom, proc),
                                          _canonical(np.stack([truth[i][1] for i in want]), proc))
            np.testing.assert_array_equal(w, [truth[i][2] for i in want])
            # the same matching rule on both sides: identical slots agree too
            np.testing.assert_array_equal(mom, np.array([olhe.momenta(ev[i], proc) for i in want]))
        assert rw.rwgt_lhe_select(lhe, "d d~ > e+ e-").size == 10
    finally:
        rw.rwgt_lhe_destroy(lhe)


def test_parallel_parse_of_a_larger_file(tmp_path):
    rw = _rw()
    text, truth = slhe.lhe_text(n_per_process=(3000, 2000, 600, 400), seed=4100, previous_rwgt=False)
    path = tmp_path / "big.lhe"
    path.write_text(text)
    lhe = rw.rwgt_lhe_read(path)
    try:
        assert rw.rwgt_lhe_num_events(lhe) == 6000
        for key, proc in PROC.items():
            idx = rw.rwgt_lhe_select(lhe, proc)
            want = [i for i, t in enumerate(truth) if t[0] == key]
            np.testing.assert_array_equal(idx, want)
            mom, _ = rw.rwgt_lhe_momenta(lhe, proc, idx)
            np.testing.assert_array_equal(_canonical(mom, proc),
                                          _canonical(np.stack([truth[i][1] for i in want]), proc))
    finally:
        rw.rwgt_lhe_destroy(lhe)


def test_write_adds_weights_and_keeps_everything_else(sample, tmp_path):
    rw = _rw()
    path, text, truth = sample
    lhe = rw.rwgt_lhe_read(path)
    rng = np.random.default_rng(9)
    added = {}
    try:
        ee = rw.rwgt_lhe_select(lhe, PROC["ee_mumu"])
        uu = rw.rwgt_lhe_select(lhe, PROC["uu_eeg"])
        a, b = rng.uniform(0, 3, ee.size), rng.uniform(0, 3, uu.size) * 1e-7
        rw.rwgt_lhe_add_weights(lhe, "set_1", "set MASS 23 91.5", ee, a)
        rw.rwgt_lhe_add_weights(lhe, "set_1", "set MASS 23 91.5", uu, b)
        rw.rwgt_lhe_add_weights(lhe, "set_2", "set SMINPUTS 3 0.13", uu, -b)
        for i, v in zip(ee, a):
            added.setdefault(int(i), {})["set_1"] = v
        for i, v in zip(uu, b):
            added.setdefault(int(i), {})["set_1"] = v
            added[int(i)]["set_2"] = -v
        out = tmp_path / "out.lhe"
        rw.rwgt_lhe_write(lhe, out)
        with pytest.raises(rw.RwgtError, match="EINVAL"):
            rw.rwgt_lhe_add_weights(lhe, "bad'id", "", ee[:1], a[:1])
    finally:
        rw.rwgt_lhe_destroy(lhe)
    new = out.read_text()
    old_ev, new_ev = olhe.read(text), olhe.read(new)
    assert len(new_ev) == len(old_ev)
    for i, (o, n) in enumerate(zip(old_ev, new_ev)):
        assert (n["nup"], n["idprup"], n["info"], n["particles"]) == (o["nup"], o["idprup"], o["info"], o["particles"])
        want = dict(o["weights"])
        want.update({"set_1": 0.0, "set_2": 0.0})
        want.update(added.get(i, {}))
        assert n["weights"] == want          # 17 significant digits: exact
    hw = olhe.header_weights(new)
    assert hw["set_1"] == "set MASS 23 91.5" and hw["set_2"] == "set SMINPUTS 3 0.13" and "old_1" in hw
    # the file read back by the library gives the same momenta
    lhe = rw.rwgt_lhe_read(out)
    try:
        idx = rw.rwgt_lhe_select(lhe, PROC["gg_ttgg"])
        mom, _ = rw.rwgt_lhe_momenta(lhe, PROC["gg_ttgg"], idx)
        np.testing.assert_array_equal(_canonical(mom, PROC["gg_ttgg"]),
                                      _canonical(np.stack([t[1] for t in truth if t[0] == "gg_ttgg"]),
                                                 PROC["gg_ttgg"]))
    finally:
        rw.rwgt_lhe_destroy(lhe)


def test_malformed_files_and_bad_requests(sample):
    rw = _rw()
    _, text, _ = sample
    first = text.index("<event")
    line_end = text.index("\n", text.index("\n", first) + 1)       # the event line of the first event
    broken = text[:line_end + 1] + " 11 -1 0 0 0 0 garbage 0 0 1 0 0 9\n" + text[line_end + 1:]
    with pytest.raises(rw.RwgtError, match="ECARD.*event 0"):
        rw.rwgt_lhe_parse(broken)
    with pytest.raises(rw.RwgtError, match="ECARD.*unterminated"):
        rw.rwgt_lhe_parse(text[:text.rindex("</event>")])
    with pytest.raises(rw.RwgtError, match="ECARD"):
        rw.rwgt_lhe_parse("<LesHouchesEvents>\n</LesHouchesEvents>\n")
    lhe = rw.rwgt_lhe_parse(text)
    try:
        with pytest.raises(rw.RwgtError, match="EPROCESS"):
            rw.rwgt_lhe_select(lhe, "x y > z")
        other = rw.rwgt_lhe_select(lhe, "d d~ > e+ e-")
        with pytest.raises(rw.RwgtError, match="EPROCESS"):
            rw.rwgt_lhe_momenta(lhe, PROC["ee_mumu"], other[:1])
        with pytest.raises(rw.RwgtError, match="EINVAL"):
            rw.rwgt_lhe_momenta(lhe, PROC["ee_mumu"], [10 ** 6])
    finally:
        rw.rwgt_lhe_destroy(lhe)


def test_reweight_card():
    rw = _rw()
    card = """# a reweighting card
change backend hip
change fptype m
launch --rwgt_name=mz_up
set MASS 23 91.5      # Z mass
set decay 23 2.6
launch rwgt_name=alpha_s
set SMINPUTS 3 0.130
set MASS 6 180.0
launch
set RWGTEW 1 0.2312
"""
    orig = synth.ORIG_EW
    sets, names, fp = rw.rwgt_reweight_card(PROC["uu_eeg"], orig.slha(), card)
    assert names == ["mz_up", "alpha_s", "rwgt_3"] and fp == "m"
    # the paper's m keeps FP64 amplitudes: it runs as FP64, never on single-precision amplitudes
    from paper_2510_05100_amd import lhe as rlhe
    assert rlhe.FPTYPE["m"] == rw.RWGT_FP64 and rlhe.FPTYPE["d"] == rw.RWGT_FP64
    base = orig.row("uu_eeg")
    want = np.tile(base, (3, 1))
    want[0, 3], want[0, 4] = 91.5, 2.6
    want[1, 1] = 0.130                         # MASS 6 is not a u u~ > e+ e- g parameter
    want[2, 2] = 0.2312
    np.testing.assert_array_equal(sets, want)
    # g g > t t~ g g keeps the top mass column: the second set changes it
    sets, _, _ = rw.rwgt_reweight_card(PROC["gg_ttgg"], orig.slha(), card)
    np.testing.assert_array_equal(sets[:, 0], [0.118, 0.130, 0.118])
    np.testing.assert_array_equal(sets[:, 1], [173.0, 180.0, 173.0])
    for bad, code in (("set MASS 23 91\n", "ECARD"), ("launch\nset MASS 23 x\n", "ECARD"),
                      ("launch\nset mz 91\n", "ECARD"), ("frobnicate\n", "ECARD")):
        with pytest.raises(rw.RwgtError, match=code):
            rw.rwgt_reweight_card(PROC["ee_mumu"], orig.slha(), bad)
    with pytest.raises(rw.RwgtError, match="EPROCESS"):
        rw.rwgt_reweight_card("d d~ > e+ e-", orig.slha(), "launch\n")
