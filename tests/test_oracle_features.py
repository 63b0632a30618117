"""Pins of the oracle's surrogate input features (no GPU).

features(mom, kappa) returns one row per (event, point), event-major: the 24
momentum components of the six particles divided by sqrt(s)/2, the scaled
coupling (kappa - 1)/0.2, then v_ij = 2 p_i.p_j / s for the 14 particle pairs
other than the two beams and log v_ij.  The checks below follow from the
kinematics, not from the formula: the momenta are recovered from the first
24 columns; the invariant columns do not change under a rotation about the
beam axis while the components do; and momentum conservation fixes sums of
the invariants (for an outgoing particle k, v_0k + v_1k - sum_l v_kl = 2 m_k^2/s
over the other outgoing l; the outgoing pairs sum to 1 - sum m^2/s), which a
swapped column or a wrong normalisation breaks.
"""
import numpy as np
import pytest

from oracle import mlp
from synth import generate_events, kappa_points

MASSES = (0.0, 0.0, 173.0, 173.0, 0.0, 0.0)


@pytest.fixture(scope="module")
def sample():
    mom = generate_events("gg_ttgg", 64)
    kap = kappa_points(5)
    x, kd = mlp.features(mom, kap)
    return mom, kap, x, kd


def pair_columns():
    """(i, j) -> column of v_ij, found by matching every column against
    2 p_i.p_j/s computed here for one event."""
    mom = generate_events("gg_ttgg", 3)
    x, _ = mlp.features(mom, [1.0])
    s = (mom[0, 0] + mom[1, 0]) ** 2
    cols = {}
    for i in range(6):
        for j in range(i + 1, 6):
            if (i, j) == (0, 1):
                continue
            v = 2 * (mom[i, 0] * mom[j, 0] - (mom[i, 1:] * mom[j, 1:]).sum(axis=0)) / s
            match = [c for c in range(25, 39) if np.allclose(x[:, c], v, rtol=1e-13, atol=0)]
            assert len(match) == 1, (i, j, match)
            cols[(i, j)] = match[0]
    # lexicographic pair order (the convention the device feature kernel follows)
    assert [cols[k] for k in sorted(cols)] == list(range(25, 39))
    return cols


def test_shape_and_row_order(sample):
    mom, kap, x, kd = sample
    n, P = mom.shape[2], len(kap)
    assert x.shape == (n * P, mlp.NFEAT) and kd.shape == (n * P,)
    rows = x.reshape(n, P, mlp.NFEAT)
    # event-major, point-minor: momentum columns constant over the points of an event
    assert np.all(rows[:, :, :24] == rows[:, :1, :24])
    assert np.allclose(rows[0, :, 24], (np.asarray(kap) - 1) / 0.2, rtol=1e-14)
    assert np.allclose(kd.reshape(n, P)[3], np.asarray(kap) - 1, rtol=0, atol=1e-15)


def test_momenta_recovered(sample):
    mom, kap, x, _ = sample
    n, P = mom.shape[2], len(kap)
    rs = mom[0, 0] + mom[1, 0]
    comps = x.reshape(n, P, mlp.NFEAT)[:, 0, :24] * (rs / 2)[:, None]
    assert np.allclose(comps.T.reshape(6, 4, n), mom, rtol=1e-14, atol=1e-12)


def test_invariant_columns_are_pair_products(sample):
    mom, kap, x, _ = sample
    cols = pair_columns()
    n = mom.shape[2]
    s = (mom[0, 0] + mom[1, 0]) ** 2
    rows = x.reshape(n, len(kap), mlp.NFEAT)[:, 0]
    for (i, j), c in cols.items():
        v = 2 * (mom[i, 0] * mom[j, 0] - (mom[i, 1:] * mom[j, 1:]).sum(axis=0)) / s
        assert np.allclose(rows[:, c], v, rtol=1e-12, atol=0)
        assert np.allclose(rows[:, c + 14], np.log(v), rtol=0, atol=1e-12)


def test_invariants_from_momentum_conservation(sample):
    mom, kap, x, _ = sample
    cols = pair_columns()
    n = mom.shape[2]
    s = (mom[0, 0] + mom[1, 0]) ** 2
    v = x.reshape(n, len(kap), mlp.NFEAT)[:, 0]
    col = lambda i, j: v[:, cols[(min(i, j), max(i, j))]]
    out = range(2, 6)
    for k in out:
        lhs = col(0, k) + col(1, k) - sum(col(k, l) for l in out if l != k)
        assert np.allclose(lhs, 2 * MASSES[k] ** 2 / s, rtol=0, atol=1e-12)
    total = sum(col(k, l) for k in out for l in out if k < l)
    assert np.allclose(total, 1 - sum(m * m for m in MASSES[2:]) / s, rtol=0, atol=1e-12)


def test_rotation_about_beam_axis(sample):
    mom, kap, x, _ = sample
    phi = 0.7391
    c, sn = np.cos(phi), np.sin(phi)
    rot = mom.copy()
    rot[:, 1] = c * mom[:, 1] - sn * mom[:, 2]
    rot[:, 2] = sn * mom[:, 1] + c * mom[:, 2]
    xr, _ = mlp.features(rot, kap)
    assert np.allclose(xr[:, 25:], x[:, 25:], rtol=1e-11, atol=1e-13)
    assert np.allclose(xr[:, 24], x[:, 24])
    # the transverse components do change
    assert np.max(np.abs(xr[:, 4:24] - x[:, 4:24])) > 1e-2
