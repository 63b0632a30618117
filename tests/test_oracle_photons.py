"""Pins of the oracle's e+ e- -> n photons (massless QED, n! diagrams summed
explicitly), the process of the paper's own timing experiment (Sec. 3.3,
Table 1).

What fixes it independently of its code: the textbook two-photon result, the
closed form for three photons, soft-photon factorisation (n = 4, 5 onto
n - 1), the Ward identity for every photon, chirality zeros of the massless
electron line, rotation and boost invariance, Bose symmetry and the exact
alpha^n scaling.
"""
import itertools

import numpy as np
import pytest

import oracle
from synth import generate_events
from synth.phase_space import rambo_massive

ALPHA = 1 / 132.5
E2 = 4 * np.pi * ALPHA


def dot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def events(na, n, seed=77):
    return rambo_massive(n, seed, 1000.0, (0.0,) * na, pt_min=10.0, dr_min=0.4, n_massive_leading=0)


def test_two_photons_textbook():
    # spin-averaged e+ e- -> 2 photons, massless: 2 e^4 (u/t + t/u); 1/2! for the photons
    m = events(2, 16)
    me = oracle.ee_photons_me(m, [ALPHA])[0]
    t = -2 * dot(m[1], m[2])
    u = -2 * dot(m[1], m[3])
    assert np.max(np.abs(me / (E2 ** 2 * (u / t + t / u)) - 1)) < 1e-13


def test_three_photons_closed_form():
    # massless e+ e- -> 3 photons: spin average e^6 s sum_i a_i b_i (a_i^2 + b_i^2) / prod_j a_j b_j
    # with a_i = p(e+).k_i, b_i = p(e-).k_i (Berends et al., Phys. Lett. 103B (1981) 124); 1/3!
    m = events(3, 16)
    me = oracle.ee_photons_me(m, [ALPHA])[0]
    s = 2 * dot(m[0], m[1])
    a = np.array([dot(m[0], m[2 + i]) for i in range(3)])
    b = np.array([dot(m[1], m[2 + i]) for i in range(3)])
    f = s * np.sum(a * b * (a * a + b * b), axis=0) / np.prod(a * b, axis=0)
    assert np.max(np.abs(me / (E2 ** 3 * f / 6) - 1)) < 1e-12


def add_soft_photon(m, lam, seed):
    """(n-1)-photon event -> n photons with a soft one of energy ~lam, exactly
    on-shell and momentum conserving (boost to the rest frame, rescale)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.8, 0.8)
    phi = rng.uniform(0, 2 * np.pi)
    sn = np.sqrt(1 - c * c)
    k = lam * np.array([1.0, sn * np.cos(phi), sn * np.sin(phi), c])
    fin = np.concatenate([m[2:], k[None, :]], axis=0)
    P = fin.sum(axis=0)
    M = np.sqrt(dot(P, P))
    bvec = -P[1:] / P[0]
    b2 = bvec @ bvec
    g = 1 / np.sqrt(1 - b2)
    out = np.empty_like(fin)
    for i, q in enumerate(fin):
        bq = bvec @ q[1:]
        out[i, 0] = g * (q[0] + bq)
        out[i, 1:] = q[1:] + ((g - 1) * bq / b2 + g * q[0]) * bvec
    out *= (m[0, 0] + m[1, 0]) / M
    return np.concatenate([m[:2], out], axis=0)


@pytest.mark.parametrize("na", [4, 5])
def test_soft_photon_factorisation(na):
    # |M_n|^2 -> e^2 2 p0.p1 / (p0.k p1.k) |M_{n-1}|^2 as k -> 0 (eikonal factor);
    # with the 1/n! symmetry factors the ratio carries 1/n
    base = events(na - 1, 4, seed=31)
    for e in range(4):
        hard = base[:, :, e]
        soft = add_soft_photon(hard, 1e-2, seed=e)
        me_n = oracle.ee_photons_me(soft[:, :, None], [ALPHA])[0, 0]
        me_h = oracle.ee_photons_me(hard[:, :, None], [ALPHA])[0, 0]
        k = soft[-1]
        eik = E2 * 2 * dot(soft[0], soft[1]) / (dot(soft[0], k) * dot(soft[1], k))
        assert abs(me_n / (eik * me_h / na) - 1) < 2e-4


@pytest.mark.parametrize("na", [3, 5])
def test_ward_identity(na):
    # a polarisation replaced by the photon's momentum: the amplitude vanishes;
    # the scale is the largest amplitude of the event times the photon energy
    m = events(na, 3)
    for e in range(3):
        ev = np.ascontiguousarray(m[:, :, e])
        hels = [[1, -1, *hp] for hp in itertools.product((-1, 1), repeat=na)]
        scale = max(abs(oracle.ee_photons_amp(ev, h, ALPHA)) for h in hels)
        for hel in hels[::3]:
            for g in range(na):
                gauge = abs(oracle.ee_photons_amp(ev, hel, ALPHA, gauge_leg=g))
                assert gauge < 1e-13 * scale * ev[2 + g, 0]


def test_chirality_zeros():
    # a massless electron line conserves chirality: equal e+ and e- helicity labels give exactly 0
    ev = np.ascontiguousarray(events(5, 1)[:, :, 0])
    for h in itertools.product((-1, 1), repeat=7):
        a = oracle.ee_photons_amp(ev, list(h), ALPHA)
        if h[0] == h[1]:
            assert a == 0
        else:
            assert a != 0


def rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_rotation_and_boost_invariance():
    rng = np.random.default_rng(8)
    m = generate_events("ee_5a", 6)
    me = oracle.ee_photons_me(m, [ALPHA])[0]
    R = rotation(rng)
    mr = m.copy()
    mr[:, 1:, :] = np.einsum("ij,pje->pie", R, m[:, 1:, :])
    assert np.max(np.abs(oracle.ee_photons_me(mr, [ALPHA])[0] / me - 1)) < 1e-12
    beta = 0.6
    g = 1 / np.sqrt(1 - beta ** 2)
    mb = m.copy()
    mb[:, 0] = g * (m[:, 0] + beta * m[:, 3])
    mb[:, 3] = g * (m[:, 3] + beta * m[:, 0])
    assert np.max(np.abs(oracle.ee_photons_me(mb, [ALPHA])[0] / me - 1)) < 1e-11


def test_bose_symmetry():
    m = generate_events("ee_5a", 4)
    me = oracle.ee_photons_me(m, [ALPHA])[0]
    perm = [0, 1, 4, 2, 6, 3, 5]
    assert np.max(np.abs(oracle.ee_photons_me(np.ascontiguousarray(m[perm]), [ALPHA])[0] / me - 1)) < 1e-12
    ev = np.ascontiguousarray(m[:, :, 0])
    hel = [-1, 1, 1, -1, -1, 1, 1]
    a = oracle.ee_photons_amp(ev, hel, ALPHA)
    b = oracle.ee_photons_amp(np.ascontiguousarray(ev[perm]), [hel[i] for i in perm], ALPHA)
    assert abs(a - b) < 1e-12 * abs(a)


def test_alpha_power():
    m = generate_events("ee_5a", 8)
    al = [ALPHA, 0.9 * ALPHA, 1.37 * ALPHA]
    me = oracle.ee_photons_me(m, al)
    for k in (1, 2):
        assert np.max(np.abs(me[k] / me[0] / (al[k] / al[0]) ** 5 - 1)) < 1e-13
