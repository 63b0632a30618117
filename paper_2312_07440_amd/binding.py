"""Python binding of libmgrw (include/mgrw.h): argument marshalling only.

Every step of the computation runs in the HIP kernels of libmgrw.so; PyTorch
provides device memory and streams.  There is no CPU fallback: if the
library or a GPU is missing, the calls raise.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgrw.so")

OK, ERR_ARG, ERR_UNSUPPORTED, ERR_DEVICE, ERR_ALLOC, ERR_STATE = 0, -1, -2, -3, -4, -5
EE_MUMU, GG_TT, GG_TTG, GG_TTGG, GG_TTGGG, EE_5A = 1, 2, 3, 4, 5, 6
FP64, MIXED = 0, 1
MAX_POINTS = 64

PROCESS_IDS = {"ee_mumu": EE_MUMU, "gg_tt": GG_TT, "gg_ttg": GG_TTG, "gg_ttgg": GG_TTGG,
               "gg_ttggg": GG_TTGGG, "ee_5a": EE_5A}
PRECISIONS = {"fp64": FP64, "mixed": MIXED}


class Params(ctypes.Structure):
    """mgrw_params: one model-parameter point."""
    _fields_ = [("alpha", ctypes.c_double), ("sw2", ctypes.c_double), ("mz", ctypes.c_double),
                ("wz", ctypes.c_double), ("alphas", ctypes.c_double), ("mt", ctypes.c_double),
                ("wt", ctypes.c_double), ("kappa_ttg", ctypes.c_double)]


DEFAULT_PARAMS = dict(alpha=1 / 132.5, sw2=0.2312, mz=91.1876, wz=2.4952, alphas=0.118, mt=173.0,
                      wt=0.0, kappa_ttg=1.0)


def make_params(**kw):
    d = dict(DEFAULT_PARAMS)
    for k in kw:
        if k not in d:
            raise KeyError(f"unknown parameter {k}")
    d.update(kw)
    return Params(**d)


class TrainConfig(ctypes.Structure):
    """mgrw_train_config."""
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("lr_decay", ctypes.c_double), ("seed", ctypes.c_uint64)]


SURROGATE_N_PARAMS = 214273
SURROGATE_N_FEATURES = 53


class MgrwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mgrw status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded libmgrw.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                           "(hipcc, gfx950); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i64, i32 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.mgrw_create_process.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(Params), ctypes.POINTER(vp)]
    L.mgrw_create_process.restype = ctypes.c_int
    L.mgrw_set_params.argtypes = [vp, ctypes.POINTER(Params), i32]
    L.mgrw_set_params.restype = ctypes.c_int
    L.mgrw_eval_me.argtypes = [vp, dp, i64, i32, dp, vp]
    L.mgrw_eval_me.restype = ctypes.c_int
    L.mgrw_reweight.argtypes = [vp, dp, dp, i64, dp, dp, vp]
    L.mgrw_reweight.restype = ctypes.c_int
    ip = ctypes.POINTER(ctypes.c_int)
    L.mgrw_process_info.argtypes = [vp, ip, ip, ip, ip]
    L.mgrw_process_info.restype = ctypes.c_int
    L.mgrw_destroy_process.argtypes = [vp]
    L.mgrw_destroy_process.restype = None
    L.mgrw_last_error.argtypes = []
    L.mgrw_last_error.restype = ctypes.c_char_p
    L.mgrw_surrogate_train.argtypes = [vp, dp, i64, ctypes.POINTER(TrainConfig), ctypes.POINTER(ctypes.c_double), vp]
    L.mgrw_surrogate_train.restype = ctypes.c_int
    L.mgrw_reweight_host.argtypes = [vp, vp, vp, i64, vp, vp, i64]
    L.mgrw_reweight_host.restype = ctypes.c_int
    L.mgrw_surrogate_train_samples.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(TrainConfig),
                                               ctypes.POINTER(ctypes.c_double), vp]
    L.mgrw_surrogate_train_samples.restype = ctypes.c_int
    L.mgrw_reweight_surrogate.argtypes = [vp, dp, dp, i64, ctypes.c_double, ctypes.c_uint64, ctypes.c_double, dp,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), vp]
    L.mgrw_reweight_surrogate.restype = ctypes.c_int
    fp = ctypes.POINTER(ctypes.c_float)
    L.mgrw_surrogate_get.argtypes = [vp, fp]
    L.mgrw_surrogate_get.restype = ctypes.c_int
    L.mgrw_surrogate_set.argtypes = [vp, fp]
    L.mgrw_surrogate_set.restype = ctypes.c_int
    for name in ("mgrw_surrogate_save", "mgrw_surrogate_load"):
        getattr(L, name).argtypes = [vp, ctypes.c_char_p]
        getattr(L, name).restype = ctypes.c_int
    L.mgrw_surrogate_fwd_bwd.argtypes = [vp, vp, vp, vp, i64, vp, fp, ctypes.POINTER(ctypes.c_double), vp]
    L.mgrw_surrogate_fwd_bwd.restype = ctypes.c_int
    L.mgrw_reweight_kpoly.argtypes = [vp, dp, dp, i64, dp, dp, vp]
    L.mgrw_reweight_kpoly.restype = ctypes.c_int
    L.mgrw_multi_reweight.argtypes = [ctypes.POINTER(vp), ctypes.c_int, dp, ctypes.c_int, vp, dp, i64, dp, dp, vp]
    L.mgrw_multi_reweight.restype = ctypes.c_int
    L.mgrw_lhe_open.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
    L.mgrw_lhe_open.restype = ctypes.c_int
    L.mgrw_lhe_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.mgrw_lhe_info.restype = ctypes.c_int
    L.mgrw_lhe_events.argtypes = [vp, ctypes.c_int, dp, dp]
    L.mgrw_lhe_events.restype = ctypes.c_int
    L.mgrw_lhe_write.argtypes = [vp, ctypes.c_char_p, dp, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p)]
    L.mgrw_lhe_write.restype = ctypes.c_int
    L.mgrw_lhe_close.argtypes = [vp]
    L.mgrw_lhe_close.restype = None
    L.mgrw_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_int64]
    L.mgrw_kernel_time_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.mgrw_kernel_time_ms.restype = ctypes.c_int
    L.mgrw_set_option.restype = ctypes.c_int
    L.mgrw_get_option.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
    L.mgrw_get_option.restype = ctypes.c_int
    L.mgrw_reweight_noalloc.argtypes = [vp, dp, dp, i64, dp, dp, vp]
    L.mgrw_reweight_noalloc.restype = ctypes.c_int
    _lib = L
    return L


def check(status):
    if status != OK:
        raise MgrwError(status, lib().mgrw_last_error().decode())
    return status


def _ptr(t, name, n=None, dtype=None, allow_none=False):
    import torch
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def _fptr(t, name, n=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Process:
    """A process handle (mgrw_create_process ... mgrw_destroy_process)."""

    def __init__(self, proc, prec="mixed", base=None):
        self.proc = PROCESS_IDS[proc] if isinstance(proc, str) else int(proc)
        self.prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        base = base if isinstance(base, Params) else make_params(**(base or {}))
        h = ctypes.c_void_p()
        check(lib().mgrw_create_process(self.proc, self.prec, ctypes.byref(base), ctypes.byref(h)))
        self._h = h
        self.n_points = 0
        a, b, c, d = (ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int())
        check(lib().mgrw_process_info(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        self.n_ext, self.n_flows, self.n_hel, self.n_diagrams = a.value, b.value, c.value, d.value

    def close(self):
        if getattr(self, "_h", None):
            lib().mgrw_destroy_process(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, points):
        """points: list of Params or dicts of overrides of the defaults."""
        pts = [p if isinstance(p, Params) else make_params(**p) for p in points]
        arr = (Params * max(1, len(pts)))(*pts)
        check(lib().mgrw_set_params(self._h, arr, len(pts)))
        self.n_points = len(pts)

    def set_lane_mapping(self, mapping):
        """'auto', 'event_per_lane' or 'event_per_wave'."""
        v = {"auto": 0, "event_per_lane": 1, "event_per_wave": 2}[mapping]
        check(lib().mgrw_set_option(self._h, 1, v))

    def set_colour_mfma(self, on=True):
        """g g -> t tbar g g g: colour sum on the matrix cores (default off)."""
        check(lib().mgrw_set_option(self._h, 4, 1 if on else 0))

    def set_kernel_timing(self, on=True):
        """Record HIP events around the amplitude kernel(s) of every launch."""
        check(lib().mgrw_set_option(self._h, 3, 1 if on else 0))

    def kernel_time_ms(self):
        """Device time of the amplitude kernel(s) of the most recent launch."""
        v = ctypes.c_double()
        check(lib().mgrw_kernel_time_ms(self._h, ctypes.byref(v)))
        return v.value

    def set_rescue_threshold(self, tau):
        """FP64 re-evaluation of events with a gluon invariant |2 p_i.p_j|/s < tau
        (mixed precision; 0 switches it off).  Stored in units of 1e-6."""
        check(lib().mgrw_set_option(self._h, 2, int(round(tau * 1e6))))

    def set_surrogate_inputs(self, n):
        """Surrogate input features for training on events and inference:
        53 (momenta, kappa, pair invariants) or 25 (momenta and kappa)."""
        check(lib().mgrw_set_option(self._h, 5, int(n)))

    @property
    def rescue_threshold(self):
        """The FP64 re-evaluation threshold tau in force (0: off)."""
        v = ctypes.c_int64()
        check(lib().mgrw_get_option(self._h, 2, ctypes.byref(v)))
        return v.value * 1e-6

    def _n(self, mom):
        if mom.dim() != 3 or mom.shape[0] != self.n_ext or mom.shape[1] != 4:
            raise ValueError(f"mom must have shape ({self.n_ext}, 4, n)")
        return mom.shape[2]

    def eval_me(self, mom, point=-1, out=None, stream=None):
        import torch
        n = self._n(mom)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=mom.device)
        check(lib().mgrw_eval_me(self._h, _ptr(mom, "mom"), n, point, _ptr(out, "out", n), _stream(stream)))
        return out

    def reweight(self, mom, w_in=None, out=None, me_base_out=None, stream=None):
        import torch
        n = self._n(mom)
        if out is None:
            out = torch.empty((self.n_points, n), dtype=torch.float64, device=mom.device)
        check(lib().mgrw_reweight(self._h, _ptr(mom, "mom"), _ptr(w_in, "w_in", n, allow_none=True), n,
                                  _ptr(out, "out", self.n_points * n),
                                  _ptr(me_base_out, "me_base_out", n, allow_none=True), _stream(stream)))
        return out

    def reweight_noalloc(self, mom, w_in=None, out=None, me_base_out=None, stream=None):
        """mgrw_reweight_noalloc: mgrw_reweight without any device allocation
        inside the library (`out` is allocated here when not given)."""
        import torch
        n = self._n(mom)
        if out is None:
            out = torch.empty((self.n_points, n), dtype=torch.float64, device=mom.device)
        check(lib().mgrw_reweight_noalloc(self._h, _ptr(mom, "mom"), _ptr(w_in, "w_in", n, allow_none=True), n,
                                          _ptr(out, "out", self.n_points * n),
                                          _ptr(me_base_out, "me_base_out", n, allow_none=True), _stream(stream)))
        return out

    def reweight_host(self, mom, w_in=None, chunk=0, me_base=False, out=None):
        """mgrw_reweight_host: events in host memory (numpy array or CPU
        tensor, pinned for overlap), weights returned in a host array
        [n_points, n] (`out`, else a new numpy array; and |M_base|^2 [n] if
        me_base)."""
        import numpy as np

        def host_ptr(a, name, count):
            if a is None:
                return None
            if hasattr(a, "data_ptr"):
                if a.is_cuda or not a.is_contiguous() or a.dtype != __import__("torch").float64:
                    raise ValueError(f"{name}: contiguous float64 CPU tensor expected")
                if a.numel() < count:
                    raise ValueError(f"{name}: {a.numel()} values, {count} needed")
                return ctypes.c_void_p(a.data_ptr())
            if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
                raise ValueError(f"{name}: contiguous float64 array expected")
            if a.size < count:
                raise ValueError(f"{name}: {a.size} values, {count} needed")
            return ctypes.c_void_p(a.ctypes.data)

        n = int(mom.shape[-1])
        if out is None:
            out = np.empty((self.n_points, n))
        me0 = np.empty(n) if me_base else None
        check(lib().mgrw_reweight_host(self._h, host_ptr(mom, "mom", self.n_ext * 4 * n),
                                       host_ptr(w_in, "w_in", n), n, host_ptr(out, "out", self.n_points * n),
                                       host_ptr(me0, "me_base", n), int(chunk)))
        return (out, me0) if me_base else out

    def reweight_kpoly(self, mom, w_in=None, out=None, me_base_out=None, stream=None):
        """Exact reweighting through the kappa polynomial (mgrw_reweight_kpoly)."""
        import torch
        n = self._n(mom)
        if out is None:
            out = torch.empty((self.n_points, n), dtype=torch.float64, device=mom.device)
        check(lib().mgrw_reweight_kpoly(self._h, _ptr(mom, "mom"), _ptr(w_in, "w_in", n, allow_none=True), n,
                                        _ptr(out, "out", self.n_points * n),
                                        _ptr(me_base_out, "me_base_out", n, allow_none=True), _stream(stream)))
        return out

    # ---------------------------------------------------------- surrogate

    def train_surrogate(self, mom, epochs=10, batch=16384, lr=1e-3, lr_decay=0.8, seed=3003):
        """Label with the exact kernels and fit the MLP; returns per-epoch losses."""
        import numpy as np
        n = self._n(mom)
        cfg = TrainConfig(int(epochs), int(batch), float(lr), float(lr_decay), int(seed))
        losses = np.zeros(int(epochs))
        check(lib().mgrw_surrogate_train(self._h, _ptr(mom, "mom"), n, ctypes.byref(cfg),
                                         losses.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(None)))
        return losses

    def train_surrogate_samples(self, x, kd, y, epochs=10, batch=16384, lr=1e-3, lr_decay=0.8, seed=3003):
        """Fit the MLP to given device float32 samples x [m, 53], kd [m], y [m];
        returns per-epoch losses."""
        import numpy as np
        m = x.shape[0]
        cfg = TrainConfig(int(epochs), int(batch), float(lr), float(lr_decay), int(seed))
        losses = np.zeros(int(epochs))
        check(lib().mgrw_surrogate_train_samples(self._h, _fptr(x, "x", m * SURROGATE_N_FEATURES), _fptr(kd, "kd", m),
                                                 _fptr(y, "y", m), m, ctypes.byref(cfg),
                                                 losses.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 _stream(None)))
        return losses

    def reweight_surrogate(self, mom, w_in=None, audit_fraction=0.01, seed=2002, max_audit_error=0.01,
                           out=None, stream=None):
        """Returns (w_out [n_points, n], stats [n_points, 5], fell_back)."""
        import numpy as np
        import torch
        n = self._n(mom)
        if out is None:
            out = torch.empty((self.n_points, n), dtype=torch.float64, device=mom.device)
        stats = np.zeros((self.n_points, 5))
        fb = ctypes.c_int(0)
        check(lib().mgrw_reweight_surrogate(self._h, _ptr(mom, "mom"), _ptr(w_in, "w_in", n, allow_none=True), n,
                                            float(audit_fraction), int(seed), float(max_audit_error),
                                            _ptr(out, "out", self.n_points * n),
                                            stats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            ctypes.byref(fb), _stream(stream)))
        return out, stats, bool(fb.value)

    def surrogate_params(self):
        import numpy as np
        out = np.zeros(SURROGATE_N_PARAMS, dtype=np.float32)
        check(lib().mgrw_surrogate_get(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def set_surrogate_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != SURROGATE_N_PARAMS:
            raise ValueError("wrong number of parameters")
        check(lib().mgrw_surrogate_set(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def save_surrogate(self, path):
        """Write the network to a checkpoint file (mgrw_surrogate_save)."""
        check(lib().mgrw_surrogate_save(self._h, os.fsencode(path)))

    def load_surrogate(self, path):
        """Replace the network by a checkpoint file's (mgrw_surrogate_load)."""
        check(lib().mgrw_surrogate_load(self._h, os.fsencode(path)))

    def surrogate_fwd_bwd(self, x, kd, y, stream=None):
        """One forward/backward pass on device float32 x [m, 53], kd [m], y [m]."""
        import numpy as np
        import torch
        m = x.shape[0]
        pred = torch.empty(m, dtype=torch.float32, device=x.device)
        grad = np.zeros(SURROGATE_N_PARAMS, dtype=np.float32)
        loss = ctypes.c_double(0.0)
        check(lib().mgrw_surrogate_fwd_bwd(self._h, _fptr(x, "x", m * SURROGATE_N_FEATURES), _fptr(kd, "kd", m), _fptr(y, "y", m), m,
                                           _fptr(pred, "pred", m),
                                           grad.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                           ctypes.byref(loss), _stream(stream)))
        return pred, grad, loss.value


def multi_reweight(processes, mom, proc_index, w_in=None, out=None, me_base_out=None, stream=None):
    """mgrw_multi_reweight: one call over events of several processes.
    mom [n_ext_max, 4, N] float64, proc_index [N] int32 (device tensors)."""
    import torch
    if mom.dim() != 3 or mom.shape[1] != 4:
        raise ValueError("mom must have shape (n_ext_max, 4, n)")
    n = mom.shape[2]
    if not isinstance(proc_index, torch.Tensor) or not proc_index.is_cuda or proc_index.dtype != torch.int32 \
            or not proc_index.is_contiguous() or proc_index.numel() != n:
        raise ValueError("proc_index must be a contiguous int32 device tensor of n elements")
    npts = processes[0].n_points
    if out is None:
        out = torch.empty((npts, n), dtype=torch.float64, device=mom.device)
    arr = (ctypes.c_void_p * len(processes))(*[p._h.value for p in processes])
    check(lib().mgrw_multi_reweight(arr, len(processes), _ptr(mom, "mom"), mom.shape[0],
                                    ctypes.c_void_p(proc_index.data_ptr()), _ptr(w_in, "w_in", n, allow_none=True), n,
                                    _ptr(out, "out", npts * n), _ptr(me_base_out, "me_base_out", n, allow_none=True),
                                    _stream(stream)))
    return out


class LHEFile:
    """A Les Houches event file read by libmgrw (mgrw_lhe_*): events in, new
    weights out.  Host arrays (numpy)."""

    def __init__(self, path):
        h = ctypes.c_void_p()
        check(lib().mgrw_lhe_open(os.fsencode(path), ctypes.byref(h)))
        self._h = h

    def __len__(self):
        n = ctypes.c_int64()
        check(lib().mgrw_lhe_info(self._h, ctypes.byref(n)))
        return n.value

    def events(self, proc):
        """(mom [n_ext, 4, N] in the process's particle order and partonic
        centre-of-mass frame, XWGTUP [N]) as float64 numpy arrays."""
        import numpy as np
        pid = PROCESS_IDS[proc] if isinstance(proc, str) else int(proc)
        n_ext = {EE_MUMU: 4, GG_TT: 4, GG_TTG: 5, GG_TTGG: 6, GG_TTGGG: 7, EE_5A: 7}[pid]
        n = len(self)
        mom = np.empty((n_ext, 4, n))
        w = np.empty(n)
        check(lib().mgrw_lhe_events(self._h, pid, ctypes.c_void_p(mom.ctypes.data), ctypes.c_void_p(w.ctypes.data)))
        return mom, w

    def write(self, path, w_new, ids):
        """Write the file with the weights w_new [P, N] added as <wgt id=ids[k]>."""
        import numpy as np
        w = np.ascontiguousarray(w_new, dtype=np.float64)
        if w.ndim != 2 or w.shape[1] != len(self) or w.shape[0] != len(ids):
            raise ValueError("w_new must have shape (len(ids), n_events)")
        arr = (ctypes.c_char_p * len(ids))(*[str(i).encode() for i in ids])
        check(lib().mgrw_lhe_write(self._h, os.fsencode(path), ctypes.c_void_p(w.ctypes.data), len(ids), arr))

    def close(self):
        if getattr(self, "_h", None):
            lib().mgrw_lhe_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
