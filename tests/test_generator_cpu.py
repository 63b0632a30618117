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


@pytest.mark.parametrize("ng", [2, 3, 4, 5])
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


@pytest.mark.parametrize("name,ng,n", [("gg_tt", 2, 64), ("gg_ttg", 3, 32), ("gg_ttgg", 4, 6)])
def test_host_kappa_polynomial_matches_oracle(name, ng, n):
    """The kappa-polynomial evaluation (amplitudes split by the number of
    top-gluon vertices, one program at unit couplings) against the oracle at
    points that vary both alpha_s and kappa."""
    lib = hostlib()
    mom = np.ascontiguousarray(generate_events(name, n))
    kap = [1.0, 0.0, 2.5] + list(kappa_points(3))
    als = [ALS, ALS, 0.09, 0.118, 0.13, 0.2]
    pts = np.array([[np.sqrt(4 * np.pi * a), k] for a, k in zip(als, kap)]).ravel()
    me = np.zeros((len(kap), n))
    assert lib.mgrw_host_qcd_me_kpoly(ng, _dp(mom), ctypes.c_int64(n), ctypes.c_double(MT), _dp(pts), len(kap),
                                      _dp(me)) == 0
    ref = oracle.qcd_me(ng, mom, [(a, MT, k) for a, k in zip(als, kap)])
    assert np.all(me[1] == 0) and np.all(ref[1] == 0)      # every diagram has a top-gluon vertex
    ok = np.arange(len(kap)) != 1
    assert np.max(np.abs(me[ok] / ref[ok] - 1)) < 1e-12


@pytest.mark.parametrize("ng,name", [(2, "gg_tt"), (3, "gg_ttg")])
def test_oracle_me_is_polynomial_in_kappa(ng, name):
    """|M|^2 is a polynomial in kappa with powers 2..2 ng only: fitted through
    2 ng - 1 points it predicts the oracle elsewhere."""
    mom = np.ascontiguousarray(generate_events(name, 8))
    fit = np.linspace(0.5, 1.5, 2 * ng - 1)
    test = [0.3, 1.9, -0.7]
    me = oracle.qcd_me(ng, mom, [(ALS, MT, k) for k in list(fit) + test])
    V = np.array([[k ** p for p in range(2, 2 * ng + 1)] for k in fit])
    coef = np.linalg.solve(V, me[:len(fit)])
    pred = np.array([[k ** p for p in range(2, 2 * ng + 1)] for k in test]) @ coef
    assert np.max(np.abs(pred / me[len(fit):] - 1)) < 1e-9


def test_kappa_polynomial_flop_counts_recorded():
    path = os.path.join(B.GEN, "flops.json")
    if not os.path.exists(path):
        pytest.skip("not built")
    f = json.load(open(path))
    for name, ng, K in (("gg_tt", 2, 2), ("gg_ttg", 3, 6), ("gg_ttgg", 4, 24)):
        kf = f[name]["kpoly_per_helicity_flops"]
        # more than one plain program (ng colour products, ng(ng+1)/2 dot products)
        assert f[name]["per_helicity_flops"] < kf < 2 * f[name]["per_helicity_flops"] + ng * 4 * K * K


def test_host_photon_recursion_matches_oracle():
    """The subset recursion of e+ e- -> 5 photons (Weyl spinors, 64 live
    helicity configurations) against the oracle's explicit sum over the 120
    diagrams and all 128 configurations."""
    from synth import alpha_points
    lib = hostlib()
    n = 24
    mom = np.ascontiguousarray(generate_events("ee_5a", n))
    al = np.array([1 / 132.5] + list(alpha_points(3)))
    me = np.zeros((len(al), n))
    assert lib.mgrw_host_ee5a_me(_dp(mom), ctypes.c_int64(n), _dp(al), len(al), _dp(me)) == 0
    ref = oracle.ee_photons_me(mom, al)
    assert np.max(np.abs(me / ref - 1)) < 1e-12


def test_colour_matrix_bf16_split_is_exact():
    """The matrix-core colour sum of g g -> t tbar g g g uses the integer colour
    numerators as the sum of two bfloat16 matrices; the split must be exact
    and the padding zero."""
    from fractions import Fraction
    cf = P.colour_matrix_loops(5)
    den = 1
    for row in cf:
        for x in row:
            den = den * x.denominator // np.gcd(den, x.denominator)
    num = [[int(x * den) for x in row] for row in cf]
    hi, lo = P.bf16_split_table(num, 128)
    for r in (0, 7, 119, 120, 127):
        for c in (0, 5, 119, 120, 127):
            v = num[r][c] if r < 120 and c < 120 else 0
            assert P.bf16_value(hi[r * 128 + c]) + P.bf16_value(lo[r * 128 + c]) == v
    assert max(abs(x) for row in num for x in row) < 1 << 16
    assert Fraction(num[0][0], den) == cf[0][0]


def test_host_gg_ttggg_whole_and_split_programs_match_oracle():
    """g g -> t tbar g g g: the whole generated program and its double-
    precision cut into (closing-group chunk x colour-flow range) functions,
    where a diagram with terms in several ranges is evaluated once per range
    and adds only that range's terms, against the oracle's recursion at
    kappa = 1 and kappa != 1."""
    lib = hostlib()
    n = 2
    mom = np.ascontiguousarray(generate_events("gg_ttggg", n, first_event=77))
    kap = [1.0, 0.83, 1.17]
    gs = np.sqrt(4 * np.pi * ALS)
    pts = np.array([[gs, k] for k in kap]).ravel()
    whole = np.zeros((len(kap), n))
    split = np.zeros((len(kap), n))
    assert lib.mgrw_host_qcd_me(5, _dp(mom), ctypes.c_int64(n), ctypes.c_double(MT), _dp(pts), len(kap),
                                _dp(whole)) == 0
    assert lib.mgrw_host_qcd_me_split(5, _dp(mom), ctypes.c_int64(n), ctypes.c_double(MT), _dp(pts), len(kap),
                                      _dp(split)) == 0
    ref = oracle.qcd_me(5, mom, [(ALS, MT, k) for k in kap])
    assert np.max(np.abs(whole / ref - 1)) < 1e-12
    assert np.max(np.abs(split / ref - 1)) < 1e-12
