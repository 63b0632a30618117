"""FP64 CPU oracle for leading-order event reweighting -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never does, and shares no code with it.

It computes, plainly and slowly, what the reweighting method computes:

* ``qcd_me``      |M|^2 of g g -> t tbar + (ng-2) g at several parameter points
                  (Sec. 2.1, eq. (1): the amplitude factor of the weight);
* ``ee_mumu_me``  |M|^2 of e+ e- -> mu+ mu- via photon and Z;
* ``reweight``    W' = W |M'|^2 / |M|^2, NaN where |M|^2 = 0 (Sec. 2.2, eq. (3)).

The C core (``oracle.c``) is built with gcc; ``quad=True`` selects the
__float128 build used to referee FP64 outliers.
"""
import ctypes
import os

import numpy as np

from .colour import colour_matrix, colour_matrix_float, orderings  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {}


class EwPoint(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("sw2", ctypes.c_double),
                ("mz", ctypes.c_double), ("wz", ctypes.c_double)]


class QcdPoint(ctypes.Structure):
    _fields_ = [("alphas", ctypes.c_double), ("mt", ctypes.c_double),
                ("kappa", ctypes.c_double)]


def lib_path(quad=False):
    return os.path.join(_HERE, "liboracle_q.so" if quad else "liboracle.so")


# Optimised for any x86-64 host with AVX2 and FMA (the build host and the
# GPU hosts differ), with floating-point contraction off so that the results
# are those of the plain IEEE operations as written.
CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-Wall"]


def build(verbose=False):
    """Compile the oracle (FP64 and __float128 builds) in place with gcc."""
    import subprocess
    src = os.path.join(_HERE, "oracle.c")
    cmds = [
        ["gcc", *CFLAGS, "-o", lib_path(False), src, "-lm"],
        ["gcc", *CFLAGS, "-DORC_QUAD", "-o", lib_path(True), src, "-lquadmath", "-lm"],
    ]
    for c in cmds:
        if verbose:
            print(" ".join(c))
        subprocess.run(c, check=True)


def _lib(quad=False):
    if quad in _LIBS:
        return _LIBS[quad]
    path = lib_path(quad)
    if not os.path.exists(path):
        raise RuntimeError(f"oracle library {path} is not built; run oracle.build()")
    lib = ctypes.CDLL(path)
    p = "orcq_" if quad else "orc_"
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    getattr(lib, p + "qcd_me").argtypes = [ctypes.c_int, dp, ctypes.c_int64, ctypes.POINTER(QcdPoint),
                                           ctypes.c_int, dp, dp]
    getattr(lib, p + "qcd_flows").argtypes = [ctypes.c_int, dp, ip, ctypes.POINTER(QcdPoint),
                                              ctypes.c_int, dp]
    getattr(lib, p + "ee_mumu_me").argtypes = [dp, ctypes.c_int64, ctypes.POINTER(EwPoint),
                                               ctypes.c_int, dp]
    getattr(lib, p + "ee_mumu_amp").argtypes = [dp, ip, ctypes.POINTER(EwPoint), dp]
    getattr(lib, p + "ee_photons_me").argtypes = [ctypes.c_int, dp, ctypes.c_int64, dp, ctypes.c_int, dp]
    getattr(lib, p + "ee_photons_amp").argtypes = [ctypes.c_int, dp, ip, ctypes.c_double, ctypes.c_int, dp]
    getattr(lib, p + "reweight").argtypes = [dp, ctypes.c_int, ctypes.c_int64, dp, dp]
    getattr(lib, p + "wavefunction").argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, dp]
    _LIBS[quad] = (lib, p)
    return _LIBS[quad]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _call(quad, name, *args):
    lib, p = _lib(quad)
    rc = getattr(lib, p + name)(*args)
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with {rc}")


_CF_CACHE = {}


def cf_matrix(ng):
    if ng not in _CF_CACHE:
        _CF_CACHE[ng] = np.ascontiguousarray(colour_matrix_float(ng))
    return _CF_CACHE[ng]


def qcd_points(points):
    """points: iterable of (alphas, mt, kappa)."""
    pts = list(points)
    arr = (QcdPoint * len(pts))()
    for i, (a, m, k) in enumerate(pts):
        arr[i] = QcdPoint(a, m, k)
    return arr


def ew_points(points):
    pts = list(points)
    arr = (EwPoint * len(pts))()
    for i, (a, s, mz, wz) in enumerate(pts):
        arr[i] = EwPoint(a, s, mz, wz)
    return arr


def set_threads(n):
    """Number of OpenMP threads the oracle's event loops use (timing only)."""
    _lib(False)[0].orc_set_threads(int(n))


def max_threads():
    """Threads the oracle's event loops use now."""
    return int(_lib(False)[0].orc_max_threads())


def qcd_me(ng, mom, points, quad=False):
    """|M|^2 [npts, n] for SoA momenta `mom` (ng+2, 4, n)."""
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    assert mom.shape[0] == ng + 2 and mom.shape[1] == 4
    n = mom.shape[2]
    pts = qcd_points(points)
    out = np.zeros((len(pts), n))
    cf = cf_matrix(ng)
    _call(quad, "qcd_me", ng, _dp(mom), n, pts, len(pts), _dp(cf), _dp(out))
    return out


def qcd_flows(ng, mom_event, hel, point, gauge_leg=-1, quad=False):
    """Colour-ordered amplitudes J_w (complex, ng! of them) of one event.

    mom_event: (ng+2, 4); hel: ng+2 values +-1 in particle order."""
    m = np.ascontiguousarray(mom_event, dtype=np.float64).reshape(-1)
    h = np.ascontiguousarray(hel, dtype=np.int32)
    out = np.zeros(2 * len(orderings(ng)))
    pts = qcd_points([point])
    _call(quad, "qcd_flows", ng, _dp(m), h.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), pts,
          gauge_leg, _dp(out))
    return out[0::2] + 1j * out[1::2]


def ee_mumu_me(mom, points, quad=False):
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    n = mom.shape[2]
    pts = ew_points(points)
    out = np.zeros((len(pts), n))
    _call(quad, "ee_mumu_me", _dp(mom), n, pts, len(pts), _dp(out))
    return out


def ee_mumu_amp(mom_event, hel, point, quad=False):
    m = np.ascontiguousarray(mom_event, dtype=np.float64).reshape(-1)
    h = np.ascontiguousarray(hel, dtype=np.int32)
    out = np.zeros(2)
    _call(quad, "ee_mumu_amp", _dp(m), h.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
          ew_points([point]), _dp(out))
    return complex(out[0], out[1])


def ee_photons_me(mom, alphas, quad=False):
    """|M|^2 of e+ e- -> n photons, n = mom.shape[0] - 2, for each alpha: [len(alphas), n_events]."""
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    n = mom.shape[2]
    a = np.ascontiguousarray(alphas, dtype=np.float64)
    out = np.zeros((len(a), n))
    _call(quad, "ee_photons_me", mom.shape[0] - 2, _dp(mom), n, _dp(a), len(a), _dp(out))
    return out


def ee_photons_amp(mom_event, hel, alpha, gauge_leg=-1, quad=False):
    """One helicity amplitude of e+ e- -> n photons; mom_event [n+2, 4]."""
    m = np.ascontiguousarray(mom_event, dtype=np.float64).reshape(-1)
    h = np.ascontiguousarray(hel, dtype=np.int32)
    out = np.zeros(2)
    _call(quad, "ee_photons_amp", len(h) - 2, _dp(m), h.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
          float(alpha), int(gauge_leg), _dp(out))
    return complex(out[0], out[1])


def reweight(me, w_in=None):
    """me: [npts, n] with the base point first; returns W' [npts-1, n]."""
    me = np.ascontiguousarray(me, dtype=np.float64)
    npts, n = me.shape
    out = np.zeros((npts - 1, n))
    w = None if w_in is None else np.ascontiguousarray(w_in, dtype=np.float64)
    lib, p = _lib(False)
    rc = getattr(lib, p + "reweight")(_dp(me), npts, n, None if w is None else _dp(w), _dp(out))
    if rc != 0:
        raise RuntimeError("oracle reweight failed")
    return out


def wavefunction(kind, p, m, lam, quad=False):
    """kind: 'u', 'v', 'ubar', 'vbar', 'eps', 'epsstar' -> complex[4]."""
    k = {"u": 0, "v": 1, "ubar": 2, "vbar": 3, "eps": 4, "epsstar": 5}[kind]
    pp = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(8)
    _call(quad, "wavefunction", k, _dp(pp), float(m), int(lam), _dp(out))
    return out[0::2] + 1j * out[1::2]
