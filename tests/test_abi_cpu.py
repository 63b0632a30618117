"""The C ABI library loads and exports every symbol include/mgrw.h declares;
argument validation that needs no device (no kernel is launched)."""
import ctypes
import os
import re
import struct

import pytest

from paper_2312_07440_amd import binding as bd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "mgrw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mgrw_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("mgrw_create_process", "mgrw_set_params", "mgrw_eval_me", "mgrw_reweight",
              "mgrw_destroy_process", "mgrw_last_error", "mgrw_process_info"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    if not os.path.exists(bd.LIB_PATH):
        pytest.skip("libmgrw.so not built")
    lib = ctypes.CDLL(bd.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s), s


@pytest.fixture
def L():
    if not os.path.exists(bd.LIB_PATH):
        pytest.skip("libmgrw.so not built")
    return bd.lib()


def test_create_validates_arguments(L):
    h = ctypes.c_void_p()
    base = bd.make_params()
    assert L.mgrw_create_process(99, 0, ctypes.byref(base), ctypes.byref(h)) == bd.ERR_ARG
    assert L.mgrw_create_process(bd.GG_TT, 7, ctypes.byref(base), ctypes.byref(h)) == bd.ERR_ARG
    assert L.mgrw_create_process(bd.GG_TT, 0, None, ctypes.byref(h)) == bd.ERR_ARG
    assert L.mgrw_create_process(bd.EE_MUMU, bd.MIXED, ctypes.byref(base), ctypes.byref(h)) == bd.ERR_UNSUPPORTED
    bad = bd.make_params(wt=1.0)
    assert L.mgrw_create_process(bd.GG_TT, 0, ctypes.byref(bad), ctypes.byref(h)) == bd.ERR_ARG
    assert b"width" in L.mgrw_last_error()
    nan = bd.make_params(alphas=float("nan"))
    assert L.mgrw_create_process(bd.GG_TT, 0, ctypes.byref(nan), ctypes.byref(h)) == bd.ERR_ARG


def test_set_params_and_state_errors(L):
    p = bd.Process("gg_ttgg", "mixed")
    assert (p.n_ext, p.n_flows, p.n_hel, p.n_diagrams) == (6, 24, 64, 123)
    with pytest.raises(bd.MgrwError) as e:
        p.set_params([{"mt": 172.0}])           # external mass change
    assert e.value.status == bd.ERR_ARG
    arr = (bd.Params * 1)(bd.make_params())
    assert L.mgrw_set_params(p._h, arr, 0) == bd.ERR_ARG
    assert L.mgrw_set_params(p._h, arr, 65) == bd.ERR_ARG
    # no points yet: reweight and eval_me(point >= 0) are state errors (no launch)
    assert L.mgrw_reweight(p._h, None, None, 10, None, None, None) == bd.ERR_STATE
    assert L.mgrw_eval_me(p._h, None, 10, 0, None, None) == bd.ERR_STATE
    p.set_params([{"kappa_ttg": 0.9}, {"kappa_ttg": 1.1}])
    assert L.mgrw_eval_me(p._h, None, 10, 2, None, None) == bd.ERR_ARG
    assert L.mgrw_eval_me(p._h, None, 10, -2, None, None) == bd.ERR_ARG
    assert L.mgrw_reweight(p._h, None, None, -1, None, None, None) == bd.ERR_ARG
    # n = 0 is accepted and launches nothing
    assert L.mgrw_reweight(p._h, None, None, 0, None, None, None) == bd.OK
    p.close()


def test_photon_process_info_and_option_errors(L):
    p = bd.Process("ee_5a", "mixed", {"alpha": 1 / 132.5})
    assert (p.n_ext, p.n_flows, p.n_hel, p.n_diagrams) == (7, 1, 128, 120)
    with pytest.raises(bd.MgrwError):
        p.set_rescue_threshold(1e-3)
    with pytest.raises(bd.MgrwError):
        p.set_params([{"alpha": -1.0}])
    with pytest.raises(bd.MgrwError):
        p.kernel_time_ms()                      # timing is off


def test_colour_mfma_option_only_for_the_split_process(L):
    with pytest.raises(bd.MgrwError, match="matrix-core"):
        bd.Process("gg_ttgg", "mixed").set_colour_mfma(True)
    bd.Process("gg_ttggg", "mixed").set_colour_mfma(True)
    bd.Process("gg_ttgg", "mixed").set_colour_mfma(False)


def test_unsupported_precisions_and_processes(L):
    h = ctypes.c_void_p()
    base = bd.make_params()
    assert L.mgrw_create_process(bd.EE_MUMU, bd.MIXED, ctypes.byref(base), ctypes.byref(h)) == bd.ERR_UNSUPPORTED
    # g g -> t tbar g g g runs in both precisions; its FP64 re-evaluation is a
    # mixed-precision option
    assert L.mgrw_create_process(bd.GG_TTGGG, bd.FP64, ctypes.byref(base), ctypes.byref(h)) == bd.OK
    assert L.mgrw_set_option(h, 2, 3000) == bd.ERR_UNSUPPORTED
    L.mgrw_destroy_process(h)
    assert L.mgrw_create_process(bd.GG_TTGGG, bd.MIXED, ctypes.byref(base), ctypes.byref(h)) == bd.OK
    assert L.mgrw_set_option(h, 2, 3000) == bd.OK
    L.mgrw_destroy_process(h)
    assert L.mgrw_create_process(bd.EE_5A + 1, bd.FP64, ctypes.byref(base), ctypes.byref(h)) == bd.ERR_ARG
    assert L.mgrw_create_process(bd.EE_5A, bd.FP64, ctypes.byref(base), ctypes.byref(h)) == bd.OK
    L.mgrw_destroy_process(h)


def test_surrogate_checkpoint_errors(L, tmp_path):
    """Checkpoint files are checked in full before the device is touched."""
    p = bd.Process("gg_ttg", "mixed")
    assert L.mgrw_surrogate_save(p._h, str(tmp_path / "x.sur").encode()) == bd.ERR_STATE   # no network
    assert L.mgrw_surrogate_load(p._h, str(tmp_path / "missing.sur").encode()) == bd.ERR_ARG
    n = bd.SURROGATE_N_PARAMS
    good_head = b"MGRWSUR1" + struct.pack("<II", n, 0)
    cases = {
        "magic.sur": b"MGRWSUR2" + struct.pack("<II", n, 0) + bytes(4 * n),
        "count.sur": b"MGRWSUR1" + struct.pack("<II", n - 1, 0) + bytes(4 * (n - 1)),
        "short.sur": good_head + bytes(4 * n - 4),
        "long.sur": good_head + bytes(4 * n + 4),
        "empty.sur": b"",
    }
    for name, data in cases.items():
        f = tmp_path / name
        f.write_bytes(data)
        assert L.mgrw_surrogate_load(p._h, str(f).encode()) == bd.ERR_ARG, name
        assert b"checkpoint" in L.mgrw_last_error(), name
    assert L.mgrw_surrogate_load(None, str(tmp_path / "magic.sur").encode()) == bd.ERR_ARG
    assert L.mgrw_surrogate_load(p._h, None) == bd.ERR_ARG
    p.close()


def test_host_reweight_argument_errors(L):
    """mgrw_reweight_host checks its arguments before touching the device."""
    p = bd.Process("gg_ttg", "mixed")
    assert L.mgrw_reweight_host(p._h, None, None, 10, None, None, 0) == bd.ERR_STATE   # no points
    p.set_params([{"kappa_ttg": 1.1}])
    assert L.mgrw_reweight_host(p._h, None, None, -1, None, None, 0) == bd.ERR_ARG
    assert L.mgrw_reweight_host(p._h, None, None, 10, None, None, -5) == bd.ERR_ARG
    assert L.mgrw_reweight_host(p._h, None, None, 10, None, None, 0) == bd.ERR_ARG     # null arrays
    assert L.mgrw_reweight_host(p._h, None, None, 0, None, None, 0) == bd.OK           # nothing to do
    assert L.mgrw_reweight_host(None, None, None, 0, None, None, 0) == bd.ERR_ARG
    p.close()


def test_surrogate_needs_unit_base_kappa(L):
    """The network's prediction vanishes at kappa = 1 by construction, so a
    base point with another kappa is refused before the device is touched."""
    p = bd.Process("gg_ttgg", "mixed", {"kappa_ttg": 1.2})
    p.set_params([{"kappa_ttg": 0.9}, {"kappa_ttg": 1.1}])
    cfg = bd.TrainConfig(2, 1024, 1e-3, 0.7, 1)
    assert L.mgrw_surrogate_train(p._h, None, 10, ctypes.byref(cfg), None, None) == bd.ERR_UNSUPPORTED
    assert b"kappa_ttg = 1" in L.mgrw_last_error()
    st = (ctypes.c_double * 10)()
    assert L.mgrw_reweight_surrogate(p._h, None, None, 10, 0.01, 1, 0.01, None, st, None, None) == bd.ERR_UNSUPPORTED
    p.close()


def test_get_option_and_default_rescue_thresholds(L):
    """Options read back as set; the FP64 re-evaluation thresholds default to
    3e-3 (g g -> t tbar g g), 1e-3 (g g -> t tbar g g g) and off in FP64."""
    v = ctypes.c_int64()
    for proc, prec, want in (("gg_ttgg", "mixed", 3000), ("gg_ttggg", "mixed", 1000), ("gg_ttgg", "fp64", 0),
                             ("gg_tt", "mixed", 3000)):
        p = bd.Process(proc, prec)
        assert L.mgrw_get_option(p._h, 2, ctypes.byref(v)) == bd.OK
        assert v.value == want
        p.close()
    p = bd.Process("gg_ttgg", "mixed")
    assert L.mgrw_set_option(p._h, 2, 500) == bd.OK
    assert p.rescue_threshold == pytest.approx(5e-4)
    assert L.mgrw_get_option(p._h, 1, ctypes.byref(v)) == bd.OK and v.value == 0
    assert L.mgrw_get_option(p._h, 5, ctypes.byref(v)) == bd.OK and v.value == 53   # surrogate inputs
    assert L.mgrw_set_option(p._h, 5, 25) == bd.OK
    assert L.mgrw_get_option(p._h, 5, ctypes.byref(v)) == bd.OK and v.value == 25
    assert L.mgrw_set_option(p._h, 5, 30) == bd.ERR_ARG
    assert L.mgrw_get_option(p._h, 99, ctypes.byref(v)) == bd.ERR_ARG
    assert L.mgrw_get_option(p._h, 2, None) == bd.ERR_ARG
    assert L.mgrw_get_option(None, 2, ctypes.byref(v)) == bd.ERR_ARG
    p.close()


def test_noalloc_argument_errors(L):
    """mgrw_reweight_noalloc checks its arguments like mgrw_reweight, before
    touching the device, and refuses the split program."""
    assert L.mgrw_reweight_noalloc(None, None, None, 10, None, None, None) == bd.ERR_ARG
    p = bd.Process("gg_ttgg", "mixed")
    assert L.mgrw_reweight_noalloc(p._h, None, None, 10, None, None, None) == bd.ERR_STATE
    p.set_params([{"kappa_ttg": 1.1}])
    assert L.mgrw_reweight_noalloc(p._h, None, None, -1, None, None, None) == bd.ERR_ARG
    assert L.mgrw_reweight_noalloc(p._h, None, None, 0, None, None, None) == bd.OK
    p.close()
    q = bd.Process("gg_ttggg", "mixed")
    q.set_params([{"kappa_ttg": 1.1}])
    assert L.mgrw_reweight_noalloc(q._h, None, None, 10, None, None, None) == bd.ERR_UNSUPPORTED
    assert b"g g -> t tbar g g g" in L.mgrw_last_error()
    q.close()
