"""Synthetic partonic events in the centre-of-mass frame.

Layout of every sample: a float64 array ``mom`` of shape (n_ext, 4, n), C
order, i.e. ``mom[(i*4 + mu)*n + e]`` is component mu = (E, px, py, pz), in
GeV, of external particle i in event e ("structure of arrays").  Particle order
follows the process name: (e+, e-, mu+, mu-) or (g, g, t, tbar, g, ...).  The
two incoming partons run along +z and -z with half the centre-of-mass energy
each.

Recipes (one per workload):

* ``ee_mumu``   sqrt(s) = 200 GeV; cos(theta) = 2u-1, phi = 2 pi u, theta being
                the angle between e+ and mu+.
* ``gg_tt``     ln sqrt(s) uniform in [ln 350, ln 2000] GeV; two-body massive
                final state with cos(theta), phi uniform; m_t = 173 GeV.
* ``gg_ttg``    sqrt(s) = 1.5 TeV, massive RAMBO, gluon pT > 20 GeV.
* ``gg_ttgg``   sqrt(s) = 1.5 TeV, massive RAMBO, gluon pT > 20 GeV and
                Delta R(g, g) > 0.4 (pseudorapidity, azimuth wrapped to pi).
* ``gg_ttggg``  sqrt(s) = 2 TeV, same cuts over all gluon pairs.
* ``ee_5a``     e+ e- -> 5 photons at sqrt(s) = 1 TeV, massless RAMBO, photon
                pT > 10 GeV, |eta| < 2.5 and Delta R(a, a) > 0.4 (the usual
                default photon cuts of LO generators).

RAMBO is the algorithm of Kleiss, Stirling and Ellis (Comput. Phys. Commun. 40
(1986) 359): isotropic massless momenta with energies -ln(u u'), boosted and
scaled to the centre-of-mass frame, followed by the standard massive
rescaling with the factor xi that solves sum_i sqrt(m_i^2 + xi^2 |p_i|^2) =
sqrt(s).  Events failing a cut are redrawn (attempt a uses draws a*64 + j), so
the momenta of event e do not depend on the sample size.  The phase-space
weight is not returned: the input event weight W of the reweighting is a
separate array.
"""
from dataclasses import dataclass

import numpy as np

from .rng import uniform

MT = 173.0

STREAM_PS = 0      # phase space
STREAM_KAPPA = 1   # parameter points
STREAM_AUDIT = 2   # surrogate audit selection
STREAM_MLP = 3     # surrogate initialisation / shuffling
STREAM_TRAIN = 4   # surrogate training events
STREAM_BATCH = 5   # uneven batch sizes


@dataclass(frozen=True)
class ProcessSpec:
    name: str
    config_id: int
    n_ext: int
    n_gluons: int        # gluons in the process, incoming included (0 for e+e-)
    masses: tuple        # outgoing masses in particle order
    sqrt_s: float        # fixed CM energy (None: drawn per event)
    n_events: int        # full sample size of the workload
    pt_min: float = 0.0
    dr_min: float = 0.0
    eta_max: float = None

    @property
    def seed(self):
        return 1000 * self.config_id


PROCESSES = {
    "ee_mumu": ProcessSpec("ee_mumu", 1, 4, 0, (0.0, 0.0), 200.0, 65536),
    "gg_tt": ProcessSpec("gg_tt", 2, 4, 2, (MT, MT), None, 1 << 20),
    "gg_ttg": ProcessSpec("gg_ttg", 3, 5, 3, (MT, MT, 0.0), 1500.0, 1 << 22, 20.0, 0.0),
    "gg_ttgg": ProcessSpec("gg_ttgg", 4, 6, 4, (MT, MT, 0.0, 0.0), 1500.0, 1 << 23, 20.0, 0.4),
    "gg_ttggg": ProcessSpec("gg_ttggg", 5, 7, 5, (MT, MT, 0.0, 0.0, 0.0), 2000.0, 1 << 20, 20.0, 0.4),
    "ee_5a": ProcessSpec("ee_5a", 6, 7, 0, (0.0,) * 5, 1000.0, 1 << 22, 10.0, 0.4, 2.5),
}


def _beams(sqrt_s):
    n = sqrt_s.shape[0]
    e = 0.5 * sqrt_s
    p1 = np.stack([e, np.zeros(n), np.zeros(n), e])
    p2 = np.stack([e, np.zeros(n), np.zeros(n), -e])
    return p1, p2


def ee_mumu(n, seed, first_event=0, sqrt_s=200.0):
    ev = np.arange(first_event, first_event + n, dtype=np.uint64)
    c = 2.0 * uniform(seed, STREAM_PS, ev, 0) - 1.0
    phi = 2.0 * np.pi * uniform(seed, STREAM_PS, ev, 1)
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    e = 0.5 * sqrt_s
    p1, p2 = _beams(np.full(n, sqrt_s))
    p3 = np.stack([np.full(n, e), e * s * np.cos(phi), e * s * np.sin(phi), e * c])
    p4 = np.stack([np.full(n, e), -p3[1], -p3[2], -p3[3]])
    return np.ascontiguousarray(np.stack([p1, p2, p3, p4]))


def gg_tt(n, seed, first_event=0, mt=MT, lo=350.0, hi=2000.0):
    ev = np.arange(first_event, first_event + n, dtype=np.uint64)
    rs = np.exp(np.log(lo) + uniform(seed, STREAM_PS, ev, 0) * (np.log(hi) - np.log(lo)))
    c = 2.0 * uniform(seed, STREAM_PS, ev, 1) - 1.0
    phi = 2.0 * np.pi * uniform(seed, STREAM_PS, ev, 2)
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    e = 0.5 * rs
    p = np.sqrt(e * e - mt * mt)
    p1, p2 = _beams(rs)
    p3 = np.stack([e, p * s * np.cos(phi), p * s * np.sin(phi), p * c])
    p4 = np.stack([e, -p3[1], -p3[2], -p3[3]])
    return np.ascontiguousarray(np.stack([p1, p2, p3, p4]))


def _rambo_attempt(seed, ev, attempt, sqrt_s, masses):
    """One RAMBO draw per event in `ev`; returns (n_out, 4, len(ev))."""
    nout = len(masses)
    base = np.uint64(attempt * 64)
    q = np.empty((nout, 4, len(ev)))
    for i in range(nout):
        d = base + np.uint64(4 * i)
        c = 2.0 * uniform(seed, STREAM_PS, ev, d) - 1.0
        phi = 2.0 * np.pi * uniform(seed, STREAM_PS, ev, d + np.uint64(1))
        q0 = -np.log(uniform(seed, STREAM_PS, ev, d + np.uint64(2)) *
                     uniform(seed, STREAM_PS, ev, d + np.uint64(3)))
        s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
        q[i] = np.stack([q0, q0 * s * np.cos(phi), q0 * s * np.sin(phi), q0 * c])
    Q = q.sum(axis=0)
    M = np.sqrt(Q[0] ** 2 - Q[1] ** 2 - Q[2] ** 2 - Q[3] ** 2)
    b = -Q[1:] / M
    x = sqrt_s / M
    gam = Q[0] / M
    a = 1.0 / (1.0 + gam)
    p = np.empty_like(q)
    for i in range(nout):
        bq = b[0] * q[i, 1] + b[1] * q[i, 2] + b[2] * q[i, 3]
        p[i, 0] = x * (gam * q[i, 0] + bq)
        p[i, 1:] = x * (q[i, 1:] + b * q[i, 0] + a * bq * b)
    # massive rescaling: solve sum_i sqrt(m_i^2 + xi^2 |p_i|^2) = sqrt(s)
    m2 = np.array(masses, dtype=np.float64) ** 2
    if np.any(m2 > 0):
        pp2 = (p[:, 1:] ** 2).sum(axis=1)               # |p_i|^2, (nout, n)
        xi = np.full(len(ev), np.sqrt(max(0.0, 1.0 - (sum(masses) / sqrt_s) ** 2)))
        for _ in range(60):
            e = np.sqrt(m2[:, None] + xi[None, :] ** 2 * pp2)
            f = e.sum(axis=0) - sqrt_s
            fp = (xi[None, :] * pp2 / e).sum(axis=0)
            step = f / fp
            xi = xi - step
            if np.all(np.abs(step) <= 1e-15 * xi):
                break
        e = np.sqrt(m2[:, None] + xi[None, :] ** 2 * pp2)
        p[:, 0] = e
        p[:, 1:] *= xi[None, None, :]
    return p


def _cuts(p_gluons, pt_min, dr_min, eta_max=None):
    """Acceptance mask for the outgoing massless partons p_gluons (ng, 4, n)."""
    ok = np.ones(p_gluons.shape[2], dtype=bool)
    if p_gluons.shape[0] == 0:
        return ok
    pt = np.hypot(p_gluons[:, 1], p_gluons[:, 2])
    ok &= np.all(pt > pt_min, axis=0)
    if eta_max is not None:
        pabs = np.sqrt(pt ** 2 + p_gluons[:, 3] ** 2)
        eta = 0.5 * np.log((pabs + p_gluons[:, 3]) / np.maximum(pabs - p_gluons[:, 3], 1e-300))
        ok &= np.all(np.abs(eta) < eta_max, axis=0)
    if dr_min > 0 and p_gluons.shape[0] > 1:
        pabs = np.sqrt(pt ** 2 + p_gluons[:, 3] ** 2)
        eta = 0.5 * np.log((pabs + p_gluons[:, 3]) / np.maximum(pabs - p_gluons[:, 3], 1e-300))
        phi = np.arctan2(p_gluons[:, 2], p_gluons[:, 1])
        ng = p_gluons.shape[0]
        for i in range(ng):
            for j in range(i + 1, ng):
                dphi = np.abs(phi[i] - phi[j])
                dphi = np.where(dphi > np.pi, 2.0 * np.pi - dphi, dphi)
                ok &= (eta[i] - eta[j]) ** 2 + dphi ** 2 > dr_min ** 2
    return ok


def rambo_massive(n, seed, sqrt_s, masses, pt_min=0.0, dr_min=0.0, first_event=0,
                  n_massive_leading=2, max_attempts=10000, eta_max=None):
    """Massive RAMBO in the CM frame with gluon cuts by rejection.

    `masses` are the outgoing masses; particles after the first
    `n_massive_leading` are the gluons the cuts apply to."""
    nout = len(masses)
    out = np.empty((2 + nout, 4, n))
    p1, p2 = _beams(np.full(n, float(sqrt_s)))
    out[0], out[1] = p1, p2
    pending = np.arange(n)
    for attempt in range(max_attempts):
        if pending.size == 0:
            break
        ev = (pending + first_event).astype(np.uint64)
        p = _rambo_attempt(seed, ev, attempt, float(sqrt_s), masses)
        ok = _cuts(p[n_massive_leading:], pt_min, dr_min, eta_max)
        acc = pending[ok]
        out[2:, :, acc] = p[:, :, ok]
        pending = pending[~ok]
    if pending.size:
        raise RuntimeError("phase-space rejection did not converge")
    return np.ascontiguousarray(out)


def generate_events(proc, n, first_event=0, seed=None):
    """Seeded sample of `n` events of process `proc` (a name in PROCESSES)."""
    spec = PROCESSES[proc]
    seed = spec.seed if seed is None else seed
    if proc == "ee_mumu":
        return ee_mumu(n, seed, first_event, spec.sqrt_s)
    if proc == "gg_tt":
        return gg_tt(n, seed, first_event)
    if proc == "ee_5a":
        return rambo_massive(n, seed, spec.sqrt_s, spec.masses, spec.pt_min, spec.dr_min,
                             first_event=first_event, n_massive_leading=0, eta_max=spec.eta_max)
    return rambo_massive(n, seed, spec.sqrt_s, spec.masses, spec.pt_min, spec.dr_min,
                         first_event=first_event)


def uneven_batches(proc, n=None, lo=65536, hi=262144, seed=None):
    """Seeded batch sizes B_k ~ U{lo..hi} covering `n` events (the workload's
    full sample by default); the last batch is the remainder and may be
    smaller than `lo`."""
    spec = PROCESSES[proc]
    n = spec.n_events if n is None else n
    seed = spec.seed if seed is None else seed
    sizes, b = [], 0
    while sum(sizes) < n:
        s = int(lo + uniform(seed, STREAM_BATCH, b, 0) * (hi - lo + 1))
        sizes.append(min(s, n - sum(sizes)))
        b += 1
    return sizes


def alpha_points(n_points=16, seed=6000, alpha0=1 / 132.5, lo=0.5, hi=1.5):
    """`n_points` iid draws of the electromagnetic coupling, uniform in
    [lo, hi] * alpha0 (a random non-zero value per reweight iteration)."""
    u = uniform(seed, STREAM_KAPPA, np.arange(n_points, dtype=np.uint64), 0)
    return alpha0 * (lo + (hi - lo) * u)


def kappa_points(n_points=16, seed=1000, lo=0.8, hi=1.2):
    """`n_points` iid draws of the top-gluon coupling scale, sorted."""
    u = uniform(seed, STREAM_KAPPA, np.arange(n_points, dtype=np.uint64), 0)
    return np.sort(lo + (hi - lo) * u)
