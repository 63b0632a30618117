"""mgrw_reweight_noalloc through the C ABI: the allocation-free variant of
mgrw_reweight (buffers from the library's per-GPU scratch array, events in
chunks) gives the same weights and base |M|^2, bit for bit, as mgrw_reweight
on the same inputs, for two calls in a row (the second smaller, so the array
still holds the first call's data)."""
import ctypes
import sys

import numpy as np
import pytest

from synth import alpha_points, generate_events, kappa_points

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def both_calls(torch, p, mom_np, w_np):
    """(weights, base |M|^2) of mgrw_reweight and of mgrw_reweight_noalloc."""
    from paper_2312_07440_amd import binding as bd
    L = bd.lib()
    n = mom_np.shape[2]
    mom = torch.from_numpy(np.ascontiguousarray(mom_np)).to("cuda:0")
    w = None if w_np is None else torch.from_numpy(w_np).to("cuda:0")
    res = []
    for fn in (L.mgrw_reweight, L.mgrw_reweight_noalloc):
        out = torch.full((p.n_points, n), -7.0, dtype=torch.float64, device="cuda:0")
        me0 = torch.full((n,), -7.0, dtype=torch.float64, device="cuda:0")
        st = fn(p._h, vp(mom), vp(w), n, vp(out), vp(me0), None)
        assert st == bd.OK, L.mgrw_last_error()
        torch.cuda.synchronize()
        res.append((out.cpu().numpy(), me0.cpu().numpy()))
    return res


CASES = [
    # process, precision, first call's events (several scratch chunks where the
    # records are large), second call's events
    ("gg_ttgg", "mixed", 600_000, 1000),
    ("gg_ttgg", "fp64", 5000, 100),
    ("gg_ttg", "mixed", 100_000, 777),
    ("gg_tt", "mixed", 70_000, 65),
    ("ee_5a", "mixed", 400_000, 333),
    ("ee_mumu", "fp64", 65_536, 100),
]


@pytest.mark.parametrize("name,prec,n1,n2", CASES)
def test_noalloc_equals_reweight(torch_dev, name, prec, n1, n2):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    say(f"case noalloc {name} {prec} n={n1} then n={n2}")
    if name == "ee_5a":
        p = mg.Process(name, prec, {"alpha": 1 / 132.5})
        p.set_params([{"alpha": float(a)} for a in alpha_points(16)])
    elif name == "ee_mumu":
        p = mg.Process(name, prec)
        p.set_params([{"mz": 95.0}])
    else:
        p = mg.Process(name, prec)
        p.set_params([{"kappa_ttg": float(k)} for k in kappa_points(16)])
    rng = np.random.default_rng(11)
    for call, (n, first) in enumerate(((n1, 0), (n2, 5_000_000))):
        mom = generate_events(name, n, first_event=first)
        w = rng.normal(size=n) if call == 0 else None
        if w is not None:
            w[::9] = 0.0
        (a, a0), (b, b0) = both_calls(torch, p, mom, w)
        say(f"  call {call + 1}: {n} events, identical weights {np.array_equal(a, b)}, "
            f"identical |M|^2 {np.array_equal(a0, b0)}")
        assert np.isfinite(a).all() and np.isfinite(a0).all()
        assert np.array_equal(a, b)
        assert np.array_equal(a0, b0)


def test_noalloc_refuses_split_program(torch_dev):
    import paper_2312_07440_amd as mg
    from paper_2312_07440_amd import binding as bd
    torch = torch_dev
    say("case noalloc gg_ttggg refused")
    p = mg.Process("gg_ttggg", "mixed")
    p.set_params([{"kappa_ttg": 1.1}])
    mom = torch.from_numpy(generate_events("gg_ttggg", 8)).to("cuda:0")
    out = torch.empty((1, 8), dtype=torch.float64, device="cuda:0")
    L = bd.lib()
    assert L.mgrw_reweight_noalloc(p._h, vp(mom), None, 8, vp(out), None, None) == bd.ERR_UNSUPPORTED
    assert b"scratch" in L.mgrw_last_error()
