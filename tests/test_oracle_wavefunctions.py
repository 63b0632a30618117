"""Pins of the oracle's external wavefunctions against the Dirac algebra.

The gamma matrices are built here independently of the oracle (chiral
representation); the checks are the Dirac equation, the spin sums
(completeness) and helicity eigenvalues -- none reuses the oracle's formulas.
"""
import numpy as np
import pytest

import oracle

I2 = np.eye(2)
SX = np.array([[0, 1], [1, 0]], dtype=complex)
SY = np.array([[0, -1j], [1j, 0]])
SZ = np.array([[1, 0], [0, -1]], dtype=complex)
Z2 = np.zeros((2, 2))
G0 = np.block([[Z2, I2], [I2, Z2]]).astype(complex)
GK = [np.block([[Z2, s], [-s, Z2]]) for s in (SX, SY, SZ)]
GAMMA = [G0] + GK
G5 = 1j * G0 @ GK[0] @ GK[1] @ GK[2]
METRIC = np.diag([1.0, -1.0, -1.0, -1.0])


def slash(p):
    return sum(METRIC[m, m] * GAMMA[m] * p[m] for m in range(4))


def random_momentum(rng, m):
    p3 = rng.normal(size=3) * rng.uniform(10, 800)
    e = np.sqrt(m * m + p3 @ p3)
    return np.concatenate([[e], p3])


def test_gamma_algebra_is_chiral_clifford():
    for a in range(4):
        for b in range(4):
            ac = GAMMA[a] @ GAMMA[b] + GAMMA[b] @ GAMMA[a]
            assert np.allclose(ac, 2 * METRIC[a, b] * np.eye(4))
    assert np.allclose(G5, np.diag([-1, -1, 1, 1]))


@pytest.mark.parametrize("m", [0.0, 173.0])
def test_dirac_equation(m):
    rng = np.random.default_rng(1)
    for _ in range(20):
        p = random_momentum(rng, m)
        scale = p[0]
        for lam in (-1, 1):
            u = oracle.wavefunction("u", p, m, lam)
            v = oracle.wavefunction("v", p, m, lam)
            ub = oracle.wavefunction("ubar", p, m, lam)
            vb = oracle.wavefunction("vbar", p, m, lam)
            assert np.abs((slash(p) - m * np.eye(4)) @ u).max() < 1e-12 * scale
            assert np.abs((slash(p) + m * np.eye(4)) @ v).max() < 1e-12 * scale
            assert np.abs(ub @ (slash(p) - m * np.eye(4))).max() < 1e-12 * scale
            assert np.abs(vb @ (slash(p) + m * np.eye(4))).max() < 1e-12 * scale
            # normalisation ubar u = 2m, vbar v = -2m
            assert abs(ub @ u - 2 * m) < 1e-12 * scale
            assert abs(vb @ v + 2 * m) < 1e-12 * scale


@pytest.mark.parametrize("m", [0.0, 173.0])
def test_spin_sums(m):
    rng = np.random.default_rng(2)
    for _ in range(20):
        p = random_momentum(rng, m)
        su = sum(np.outer(oracle.wavefunction("u", p, m, l), oracle.wavefunction("ubar", p, m, l))
                 for l in (-1, 1))
        sv = sum(np.outer(oracle.wavefunction("v", p, m, l), oracle.wavefunction("vbar", p, m, l))
                 for l in (-1, 1))
        assert np.abs(su - (slash(p) + m * np.eye(4))).max() < 1e-12 * p[0]
        assert np.abs(sv - (slash(p) - m * np.eye(4))).max() < 1e-12 * p[0]


def test_helicity_eigenvalues():
    """u(p, lam) has helicity lam/2; v(p, lam) describes an antiparticle of
    helicity lam/2, i.e. it is an eigenvector of the helicity operator with
    eigenvalue -lam/2."""
    rng = np.random.default_rng(3)
    for m in (0.0, 173.0):
        for _ in range(10):
            p = random_momentum(rng, m)
            n = p[1:] / np.linalg.norm(p[1:])
            sig = n[0] * SX + n[1] * SY + n[2] * SZ
            h = 0.5 * np.block([[sig, Z2], [Z2, sig]])
            for lam in (-1, 1):
                u = oracle.wavefunction("u", p, m, lam)
                v = oracle.wavefunction("v", p, m, lam)
                assert np.allclose(h @ u, 0.5 * lam * u, atol=1e-12 * p[0])
                assert np.allclose(h @ v, -0.5 * lam * v, atol=1e-12 * p[0])


def test_massless_chirality():
    """For m = 0, u(+) is right-handed and u(-) left-handed (gamma5 = diag(-1,-1,1,1))."""
    rng = np.random.default_rng(4)
    for _ in range(10):
        p = random_momentum(rng, 0.0)
        up = oracle.wavefunction("u", p, 0.0, 1)
        um = oracle.wavefunction("u", p, 0.0, -1)
        assert np.allclose(G5 @ up, up, atol=1e-12 * p[0])
        assert np.allclose(G5 @ um, -um, atol=1e-12 * p[0])


def test_polarisation_vectors():
    rng = np.random.default_rng(5)
    ks = [random_momentum(rng, 0.0) for _ in range(20)]
    ks += [np.array([300.0, 0, 0, 300.0]), np.array([300.0, 0, 0, -300.0])]
    for k in ks:
        eps = {l: oracle.wavefunction("eps", k, 0.0, l) for l in (-1, 1)}
        epss = {l: oracle.wavefunction("epsstar", k, 0.0, l) for l in (-1, 1)}
        proj = np.zeros((4, 4), dtype=complex)
        for l in (-1, 1):
            e = eps[l]
            assert abs(e[0]) < 1e-15                       # time component zero
            assert abs(e[1:] @ k[1:]) < 1e-12 * k[0]       # transverse
            assert np.allclose(epss[l], np.conj(e))
            assert abs(np.vdot(e[1:], e[1:]) - 1) < 1e-14  # unit norm
            proj += np.outer(e, np.conj(e))
        # sum over helicities = transverse projector delta_ij - k_i k_j / |k|^2
        kk = k[1:] / np.linalg.norm(k[1:])
        assert np.allclose(proj[1:, 1:].real, np.eye(3) - np.outer(kk, kk), atol=1e-14)
        assert np.allclose(proj[1:, 1:].imag, 0, atol=1e-14)
        # helicity: (S.k-hat) eps = lam eps with (S_i)_{jk} = -i eps_ijk
        lc = np.zeros((3, 3, 3))
        lc[0, 1, 2] = lc[1, 2, 0] = lc[2, 0, 1] = 1
        lc[0, 2, 1] = lc[2, 1, 0] = lc[1, 0, 2] = -1
        sk = -1j * np.einsum("ijk,i->jk", lc, kk)
        for l in (-1, 1):
            assert np.allclose(sk @ eps[l][1:], l * eps[l][1:], atol=1e-14)
