"""Pins of the seeded phase-space fixture that feeds both the HIP path and the
oracle (no GPU).

Every sample must be a valid partonic event in the centre-of-mass frame:
momentum conservation, on-shell external particles, beams along +-z with half
the CM energy each, and the workload's cuts (gluon p_T, Delta R between
final-state gluon pairs with pseudorapidity and the azimuth wrapped to pi; no
cut involving the tops).  The massless RAMBO core must be flat: the energy
fraction x = 2E/sqrt(s) of one particle of n-body massless phase space has the
density proportional to x (1 - x)^(n-3).  Samples are deterministic and do not
depend on their size (event e is a function of e alone).
"""
import numpy as np
import pytest
from scipy import stats

from synth import PROCESSES, generate_events, rambo_massive, uneven_batches

QCD_MASSES = {"gg_tt": (173.0, 173.0), "gg_ttg": (173.0, 173.0, 0.0), "gg_ttgg": (173.0, 173.0, 0.0, 0.0),
              "gg_ttggg": (173.0, 173.0, 0.0, 0.0, 0.0)}
N_SAMPLE = {"ee_mumu": 4000, "gg_tt": 4000, "gg_ttg": 3000, "gg_ttgg": 2000, "gg_ttggg": 1500, "ee_5a": 1500}


def outgoing_masses(proc):
    return {"ee_mumu": (0.0, 0.0), "ee_5a": (0.0,) * 5}.get(proc) or QCD_MASSES[proc]


def eta_phi(p):
    """Pseudorapidity and azimuth of momenta p[4, n] (computed here, not by the fixture)."""
    pabs = np.sqrt(p[1] ** 2 + p[2] ** 2 + p[3] ** 2)
    return np.arctanh(p[3] / pabs), np.arctan2(p[2], p[1])


def delta_r(a, b):
    ea, pa = eta_phi(a)
    eb, pb = eta_phi(b)
    dphi = np.mod(pa - pb + np.pi, 2 * np.pi) - np.pi
    return np.hypot(ea - eb, dphi)


@pytest.fixture(scope="module")
def samples():
    return {p: generate_events(p, N_SAMPLE[p]) for p in N_SAMPLE}


@pytest.mark.parametrize("proc", list(N_SAMPLE))
def test_momentum_conservation_and_frame(samples, proc):
    mom = samples[proc]
    assert mom.shape == (PROCESSES[proc].n_ext, 4, N_SAMPLE[proc]) and mom.flags.c_contiguous
    rs = mom[0, 0] + mom[1, 0]
    tot = mom[0] + mom[1] - mom[2:].sum(axis=0)
    assert np.max(np.abs(tot) / rs) <= 1e-12
    # beams along +z and -z with sqrt(s)/2 each
    assert np.array_equal(mom[0, 0], mom[1, 0]) and np.array_equal(mom[0, 3], mom[0, 0])
    assert np.array_equal(mom[1, 3], -mom[1, 0])
    assert np.all(mom[0, 1:3] == 0) and np.all(mom[1, 1:3] == 0)
    spec = PROCESSES[proc]
    if spec.sqrt_s is not None:
        assert np.allclose(rs, spec.sqrt_s, rtol=0, atol=1e-12 * spec.sqrt_s)


@pytest.mark.parametrize("proc", list(N_SAMPLE))
def test_external_particles_on_shell(samples, proc):
    mom = samples[proc]
    for i, m in enumerate((0.0, 0.0) + outgoing_masses(proc)):
        p = mom[i]
        m2 = p[0] ** 2 - p[1] ** 2 - p[2] ** 2 - p[3] ** 2
        assert np.max(np.abs(m2 - m * m) / p[0] ** 2) <= 1e-12, (proc, i)
        assert np.all(p[0] > 0)


@pytest.mark.parametrize("proc", ["gg_ttg", "gg_ttgg", "gg_ttggg"])
def test_gluon_cuts(samples, proc):
    """p_T > 20 GeV for every final-state gluon and Delta R > 0.4 for every
    final-state gluon pair (none for g g -> t tbar g)."""
    mom = samples[proc]
    spec = PROCESSES[proc]
    glu = list(range(4, spec.n_ext))
    for i in glu:
        assert np.all(np.hypot(mom[i, 1], mom[i, 2]) > 20.0)
    for a in glu:
        for b in glu:
            if a < b:
                assert np.all(delta_r(mom[a], mom[b]) > 0.4), (a, b)
    # the cuts are on gluons only: the tops are unconstrained
    dr_top = np.min([delta_r(mom[t], mom[g]) for t in (2, 3) for g in glu], axis=0)
    assert np.any(dr_top < 0.4)
    assert np.any(np.hypot(mom[2, 1], mom[2, 2]) < 20.0) or np.any(np.hypot(mom[3, 1], mom[3, 2]) < 20.0)


def test_cuts_are_binding():
    """Without the cuts the same generator produces gluons below 20 GeV and
    pairs closer than 0.4, so the acceptance test above is not vacuous."""
    spec = PROCESSES["gg_ttgg"]
    raw = rambo_massive(2000, spec.seed, spec.sqrt_s, spec.masses)
    pt = np.hypot(raw[4:, 1], raw[4:, 2])
    assert np.any(pt < 20.0)
    assert np.any(delta_r(raw[4], raw[5]) < 0.4)


def test_photon_cuts(samples):
    mom = samples["ee_5a"]
    for i in range(2, 7):
        assert np.all(np.hypot(mom[i, 1], mom[i, 2]) > 10.0)
        assert np.all(np.abs(eta_phi(mom[i])[0]) < 2.5)
        for j in range(i + 1, 7):
            assert np.all(delta_r(mom[i], mom[j]) > 0.4)


def test_two_body_distributions(samples):
    """g g -> t tbar: ln sqrt(s) uniform on [ln 350, ln 2000], cos(theta) and
    phi of the top uniform; e+ e- -> mu+ mu-: cos(theta) uniform at 200 GeV."""
    mom = samples["gg_tt"]
    rs = mom[0, 0] + mom[1, 0]
    u = (np.log(rs) - np.log(350.0)) / (np.log(2000.0) - np.log(350.0))
    assert u.min() > 0 and u.max() < 1
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    pabs = np.sqrt((mom[2, 1:] ** 2).sum(axis=0))
    assert stats.kstest((mom[2, 3] / pabs + 1) / 2, "uniform").pvalue > 1e-3
    phi = np.arctan2(mom[2, 2], mom[2, 1])
    assert stats.kstest((phi + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3
    ee = samples["ee_mumu"]
    c = ee[2, 3] / ee[2, 0]
    assert np.allclose(ee[2, 0], 100.0) and stats.kstest((c + 1) / 2, "uniform").pvalue > 1e-3


@pytest.mark.parametrize("nout", [3, 4, 5])
def test_massless_rambo_is_flat(nout):
    """Energy fraction of one particle of flat n-body massless phase space:
    density (n-1)(n-2) x (1-x)^(n-3) on [0, 1]; directions isotropic."""
    n = 20000
    p = rambo_massive(n, 4242, 1000.0, (0.0,) * nout)
    x = 2 * p[2, 0] / 1000.0
    k = nout
    # CDF of (k-1)(k-2) x (1-x)^(k-3)
    def cdf(t):
        from scipy.special import betainc
        return betainc(2, k - 2, t)
    assert stats.kstest(x, cdf).pvalue > 1e-3
    c = p[3, 3] / p[3, 0]
    assert stats.kstest((c + 1) / 2, "uniform").pvalue > 1e-3


def test_massive_rescaling_exact():
    """The massive rescaling keeps every 3-momentum direction and the total
    energy sqrt(s), so only |p| changes relative to the massless draw."""
    spec = PROCESSES["gg_ttg"]
    p0 = rambo_massive(500, 77, 1500.0, (0.0, 0.0, 0.0))
    p1 = rambo_massive(500, 77, 1500.0, (173.0, 173.0, 0.0))
    d0 = p0[2:, 1:] / np.sqrt((p0[2:, 1:] ** 2).sum(axis=1, keepdims=True))
    d1 = p1[2:, 1:] / np.sqrt((p1[2:, 1:] ** 2).sum(axis=1, keepdims=True))
    assert np.max(np.abs(d0 - d1)) < 1e-12
    ratio = np.sqrt((p1[2:, 1:] ** 2).sum(axis=1)) / np.sqrt((p0[2:, 1:] ** 2).sum(axis=1))
    assert np.max(np.abs(ratio - ratio[0])) < 1e-12          # one xi per event
    assert np.allclose(p1[2:, 0].sum(axis=0), 1500.0, rtol=1e-14)
    assert spec.masses[:2] == (173.0, 173.0)


@pytest.mark.parametrize("proc", ["ee_mumu", "gg_tt", "gg_ttgg", "gg_ttggg", "ee_5a"])
def test_deterministic_and_size_independent(proc):
    a = generate_events(proc, 300)
    b = generate_events(proc, 300)
    assert np.array_equal(a, b)
    assert np.array_equal(generate_events(proc, 100), a[:, :, :100])
    assert np.array_equal(generate_events(proc, 120, first_event=150), a[:, :, 150:270])
    # another seed gives another sample
    assert not np.array_equal(generate_events(proc, 50, seed=12345), a[:, :, :50])


def test_uneven_batches():
    sizes = uneven_batches("gg_ttggg")
    assert sum(sizes) == PROCESSES["gg_ttggg"].n_events
    assert all(65536 <= s <= 262144 for s in sizes[:-1]) and 0 < sizes[-1] <= 262144
    assert sizes == uneven_batches("gg_ttggg")
    small = uneven_batches("gg_ttggg", n=300000)
    assert sum(small) == 300000 and small[0] == sizes[0]


def test_three_body_dalitz_plot_is_flat():
    """Flat three-body massless phase space is uniform on the Dalitz triangle
    x1 + x2 >= 1 (x1, x2 <= 1): w = (x1 + x2 - 1)/x1 is uniform and x1^2 too."""
    p = rambo_massive(40000, 4242, 1000.0, (0.0,) * 3)
    x1, x2 = 2 * p[2, 0] / 1000.0, 2 * p[3, 0] / 1000.0
    assert stats.kstest((x1 + x2 - 1) / x1, "uniform").pvalue > 1e-3
    assert stats.kstest(x1 * x1, "uniform").pvalue > 1e-3


@pytest.mark.parametrize("proc", ["gg_ttgg", "gg_ttggg", "ee_5a"])
def test_rejection_replayed_with_independent_cuts(proc):
    """Event e is the first RAMBO attempt of e that passes the cuts, decided
    here with this test's own p_T, |eta| and Delta R code: a cut that is too
    strict or too loose picks another attempt."""
    import synth.phase_space as ps
    spec = PROCESSES[proc]
    n = 200
    got = generate_events(proc, n)
    first = 0 if proc == "ee_5a" else 2          # particles the cuts apply to (outgoing index)
    for e in range(n):
        ev = np.array([e], dtype=np.uint64)
        for attempt in range(10000):
            q = ps._rambo_attempt(spec.seed, ev, attempt, spec.sqrt_s, spec.masses)[:, :, 0]
            g = q[first:]
            ok = all(np.hypot(x[1], x[2]) > spec.pt_min for x in g)
            if spec.eta_max is not None:
                ok = ok and all(abs(eta_phi(x[:, None])[0][0]) < spec.eta_max for x in g)
            ok = ok and all(delta_r(g[a][:, None], g[b][:, None])[0] > spec.dr_min
                            for a in range(len(g)) for b in range(a + 1, len(g)))
            if ok:
                break
        assert np.array_equal(got[2:, :, e], q), (proc, e, attempt)
