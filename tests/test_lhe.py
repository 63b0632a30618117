"""Les Houches event files through libmgrw's reader and writer (host code,
no GPU): synthetic files written by tests/lhe_fixture.py, read back in the
process's particle order and partonic frame, written again with new weights."""
import os
import re

import numpy as np
import pytest

from paper_2312_07440_amd import binding as bd
from synth import generate_events
from lhe_fixture import write_lhe


@pytest.fixture(autouse=True)
def need_lib():
    if not os.path.exists(bd.LIB_PATH):
        pytest.skip("libmgrw.so not built")


def test_events_back_in_process_order_and_cm_frame(tmp_path):
    mom = generate_events("gg_ttgg", 40)
    w = np.random.default_rng(1).uniform(0.5, 2.0, 40)
    path = tmp_path / "a.lhe"
    write_lhe(path, "gg_ttgg", mom, w)
    f = bd.LHEFile(path)
    assert len(f) == 40
    got, gw = f.events("gg_ttgg")
    assert np.array_equal(gw, w)
    # gluons are identical particles: compare the two final gluons as a set
    assert np.max(np.abs(got[:4] - mom[:4])) < 1e-9
    g_got = np.sort(got[4:, 0], axis=0)
    g_ref = np.sort(mom[4:, 0], axis=0)
    assert np.max(np.abs(g_got - g_ref)) < 1e-9
    assert np.max(np.abs(got.sum(axis=0)[1:] - 2 * got[:2].sum(axis=0)[1:])) < 1e-8   # conservation


def test_write_adds_only_the_weights(tmp_path):
    mom = generate_events("gg_ttg", 12)
    w = np.ones(12)
    src, dst = tmp_path / "in.lhe", tmp_path / "out.lhe"
    write_lhe(src, "gg_ttg", mom, w)
    f = bd.LHEFile(src)
    wn = np.random.default_rng(2).normal(size=(3, 12)) * 1e-3
    ids = ["k0", "k1", "k2"]
    f.write(dst, wn, ids)
    text = dst.read_text()
    # every weight appears with its id, exactly (17 significant digits round-trip)
    got = re.findall(r"<wgt id='(k\d)'> (\S+) </wgt>", text)
    assert len(got) == 36
    vals = np.array([float(v) for _, v in got]).reshape(12, 3).T
    assert np.array_equal(vals, wn)
    assert [i for i, _ in got[:3]] == ids
    assert "<initrwgt>" in text and "<weight id='k1'>" in text
    # removing the added lines gives back the input byte for byte
    stripped = re.sub(r"<rwgt>\n(<wgt id='k\d'> \S+ </wgt>\n)+</rwgt>\n", "", text)
    stripped = re.sub(r"<initrwgt>\n(<weight id='k\d'> </weight>\n)+</initrwgt>\n", "", stripped)
    assert stripped == src.read_text()


def test_existing_rwgt_block_is_extended(tmp_path):
    mom = generate_events("gg_tt", 5)
    src, dst = tmp_path / "in.lhe", tmp_path / "out.lhe"
    write_lhe(src, "gg_tt", mom, np.ones(5), rwgt_block=True)
    f = bd.LHEFile(src)
    f.write(dst, np.full((1, 5), 0.25), ["new"])
    text = dst.read_text()
    assert text.count("<rwgt>") == 5
    assert text.count("<wgt id='old'> 1.5 </wgt>\n<wgt id='new'> 2.50000000000000000e-01 </wgt>\n</rwgt>") == 5


def test_photon_events(tmp_path):
    mom = generate_events("ee_5a", 7)
    path = tmp_path / "a.lhe"
    write_lhe(path, "ee_5a", mom, np.ones(7))
    got, _ = bd.LHEFile(path).events("ee_5a")
    assert np.max(np.abs(got[:2] - mom[:2])) < 1e-9
    assert np.max(np.abs(np.sort(got[2:, 0], axis=0) - np.sort(mom[2:, 0], axis=0))) < 1e-9


def test_errors(tmp_path):
    with pytest.raises(bd.MgrwError, match="cannot open"):
        bd.LHEFile(tmp_path / "missing.lhe")
    mom = generate_events("gg_ttg", 3)
    path = tmp_path / "a.lhe"
    write_lhe(path, "gg_ttg", mom, np.ones(3))
    with pytest.raises(bd.MgrwError, match="does not belong|does not match"):
        bd.LHEFile(path).events("gg_ttgg")
    text = path.read_text()
    cut = tmp_path / "cut.lhe"
    cut.write_text(text[: text.rindex("</event>")])
    with pytest.raises(bd.MgrwError, match="ends inside an event"):
        bd.LHEFile(cut)
    bad = tmp_path / "bad.lhe"
    bad.write_text(text.replace("<event>\n 6 1", "<event>\n 0 1", 1))
    with pytest.raises(bd.MgrwError, match="particle count"):
        bd.LHEFile(bad)
    f = bd.LHEFile(path)
    with pytest.raises(bd.MgrwError, match="ids"):
        f.write(tmp_path / "o.lhe", np.ones((1, 3)), ["a'b"])
    assert not (tmp_path / "o.lhe").exists()
