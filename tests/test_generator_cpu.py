"""Process generator and host-executed amplitude programs (no GPU).

The generated per-helicity programs (Feynman diagrams, colour coefficients,
shared currents) are compiled for the host in double precision and compared
with the oracle's independent recursion; the colour matrices of the generator
(index-loop counting) are compared with the oracle's Fierz recursion.
"""
import ctypes
import json
import os

import numpy as np
import pytest

import oracle
from paper_2312_07440_amd import build as B
from paper_2312_07440_amd.gen import process as P
from synth import generate_events, kappa_points

ALS, MT = 0.118, 173.0


def hostlib():
    if not os.path.exists(B.HOSTLIB):
        pytest.skip("host validation library not built (run __graft_entry__.build())")
    return ctypes.CDLL(B.HOSTLIB)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def test_diagram_and_flow_counts():
    assert [P.n_diagrams(n) for n in (2, 3, 4, 5)] == [3, 16, 123, 1240]
    assert [len(P.flows(n)) for n in (2, 3, 4, 5)] == [2, 6, 24, 120]
    # pure-gluon trees with m leaves (four-gluon vertex counted once)
    assert [len(P.trees((1 << m) - 1, False)) for m in (1, 2, 3, 4, 5)] == [1, 1, 4, 25, 220]


@pytest.mark.parametrize("ng", [2, 3, 4])
def test_colour_coefficients_are_signs(ng):
    for seq in P.diagrams(ng):
        col = P.diagram_colour(seq)
        assert col, seq
        assert all(c in (1, -1) for c in col.values())


@pytest.mark.parametrize("ng", [2, 3, 4])
def test_generator_colour_matrix_matches_oracle(ng):
    assert P.colour_matrix_loops(ng) == oracle.colour_matrix(ng)


@pytest.mark.parametrize("name,ng,n", [("gg_tt", 2, 64), ("gg_ttg", 3, 32), ("gg_ttgg", 4, 6)])
def test_host_program_matches_oracle(name, ng, n):
    lib = hostlib()
    mom = np.ascontiguousarray(generate_events(name, n))
    kap = [1.0] + list(kappa_points(3))
    gs = np.sqrt(4 * np.pi * ALS)
    pts = np.array([[gs, k] for k in kap]).ravel()
    me = np.zeros((len(kap), n))
    assert lib.mgrw_host_qcd_me(ng, _dp(mom), ctypes.c_int64(n), ctypes.c_double(MT), _dp(pts), len(kap),
                                _dp(me)) == 0
    ref = oracle.qcd_me(ng, mom, [(ALS, MT, k) for k in kap])
    assert np.max(np.abs(me / ref - 1)) < 1e-12


def test_host_ee_mumu_matches_oracle():
    lib = hostlib()
    mom = np.ascontiguousarray(generate_events("ee_mumu", 256))
    ew = [(1 / 132.5, 0.2312, 91.1876, 2.4952), (1 / 132.5, 0.2312, 95.0, 2.4952)]
    p6 = []
    for a, sw2, mz, wz in ew:
        e2 = 4 * np.pi * a
        p6 += [e2, e2 / (sw2 * (1 - sw2)), -0.5 + sw2, sw2, mz * mz, mz * wz]
    p6 = np.array(p6)
    me = np.zeros((2, 256))
    assert lib.mgrw_host_ee_mumu_me(_dp(mom), ctypes.c_int64(256), _dp(p6), 2, _dp(me)) == 0
    assert np.max(np.abs(me / oracle.ee_mumu_me(mom, ew) - 1)) < 1e-12


def test_flop_counts_recorded():
    path = os.path.join(B.GEN, "flops.json")
    if not os.path.exists(path):
        pytest.skip("not built")
    f = json.load(open(path))
    assert set(f) >= {"gg_tt", "gg_ttg", "gg_ttgg"}
    assert f["gg_tt"]["per_helicity_flops"] < f["gg_ttg"]["per_helicity_flops"] < f["gg_ttgg"]["per_helicity_flops"]
    # symmetric colour sum of K flows: row i costs 2(1 + 2(K-1-i)) + 4 flops -> 2K^2 + 4K
    for name, K in (("gg_tt", 2), ("gg_ttg", 6), ("gg_ttgg", 24)):
        assert f[name]["colour_sum_flops"] == 2 * K * K + 4 * K
