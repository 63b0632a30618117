"""GPU parity of the kappa-polynomial exact reweighting (mgrw_reweight_kpoly)
against the FP64 oracle and against the point-by-point entry point.

Bars as for the other exact paths: FP64 <= 1e-12 and mixed <= 1e-5 relative
per event.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import generate_events, kappa_points

pytestmark = pytest.mark.gpu

MT = 173.0
NG = {"gg_tt": 2, "gg_ttg": 3, "gg_ttgg": 4}
TOL = {"fp64": 1e-12, "mixed": 1e-5}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def points(npts, vary_alphas):
    kap = kappa_points(npts)
    als = np.linspace(0.1, 0.13, npts) if vary_alphas else np.full(npts, 0.118)
    return [(float(a), MT, float(k)) for a, k in zip(als, kap)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name,n", [("gg_tt", 1031), ("gg_ttg", 517), ("gg_ttgg", 261)])
def test_kpoly_parity(torch_dev, name, n, prec):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    mom = generate_events(name, n)
    w = np.random.default_rng(6).normal(size=n)
    pts = points(16, vary_alphas=True)
    say(f"case kpoly {name} n={n} prec={prec}")
    p = mg.Process(name, prec, {"alphas": 0.118, "mt": MT})
    p.set_params([{"alphas": a, "mt": m, "kappa_ttg": k} for a, m, k in pts])
    me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    out = p.reweight_kpoly(to_dev(torch, mom), w_in=to_dev(torch, w), me_base_out=me0)
    torch.cuda.synchronize()
    me_ref = oracle.qcd_me(NG[name], mom, [(0.118, MT, 1.0)] + pts)
    w_ref = oracle.reweight(me_ref, w)
    e_me = np.abs(me0.cpu().numpy() / me_ref[0] - 1)
    e_w = np.abs(out.cpu().numpy() / w_ref - 1)
    say(f"  |M|^2 max {e_me.max():.3e}; W' max {e_w.max():.3e} median {np.median(e_w):.3e}")
    assert e_me.max() <= TOL[prec]
    assert e_w.max() <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_kpoly_agrees_with_point_by_point(torch_dev, prec):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 300
    mom = to_dev(torch, generate_events("gg_ttgg", n, first_event=777))
    say(f"case kpoly vs reweight gg_ttgg n={n} prec={prec}")
    p = mg.Process("gg_ttgg", prec)
    p.set_params([{"kappa_ttg": float(k)} for k in kappa_points(64)])
    a = p.reweight(mom)
    b = p.reweight_kpoly(mom)
    torch.cuda.synchronize()
    e = (b / a - 1).abs().max().item()
    say(f"  max rel diff {e:.3e}")
    assert e <= 2 * TOL[prec]


@pytest.mark.parametrize("n", [0, 1, 63, 65])
def test_kpoly_ragged_and_empty(torch_dev, n):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    say(f"case kpoly ragged gg_ttg n={n}")
    p = mg.Process("gg_ttg", "fp64")
    kap = kappa_points(3)
    p.set_params([{"kappa_ttg": float(k)} for k in kap])
    mom = generate_events("gg_ttg", max(n, 1))[:, :, :n]
    out = torch.full((3, n), -7.0, dtype=torch.float64, device="cuda:0")
    p.reweight_kpoly(to_dev(torch, mom), out=out)
    torch.cuda.synchronize()
    if n == 0:
        return
    ref = oracle.reweight(oracle.qcd_me(3, np.ascontiguousarray(mom), [(0.118, MT, 1.0)] +
                                        [(0.118, MT, float(k)) for k in kap]), np.ones(n))
    assert np.abs(out.cpu().numpy() / ref - 1).max() <= 1e-12


def test_kpoly_nan_at_vanishing_base(torch_dev):
    """Base point at kappa = 0: |M|^2 vanishes exactly, so every weight is NaN."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    say("case kpoly base kappa=0")
    p = mg.Process("gg_tt", "fp64", {"kappa_ttg": 0.0})
    p.set_params([{"kappa_ttg": 1.0}])
    me0 = torch.empty(64, dtype=torch.float64, device="cuda:0")
    out = p.reweight_kpoly(to_dev(torch, generate_events("gg_tt", 64)), me_base_out=me0)
    torch.cuda.synchronize()
    assert torch.all(me0 == 0).item()
    assert torch.all(torch.isnan(out)).item()


def test_kpoly_unsupported_processes(torch_dev):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    say("case kpoly unsupported")
    for name in ("gg_ttggg", "ee_mumu"):
        p = mg.Process(name, "mixed" if name == "gg_ttggg" else "fp64")
        p.set_params([{"kappa_ttg": 1.1}] if name == "gg_ttggg" else [{"sw2": 0.23}])
        n_ext = 7 if name == "gg_ttggg" else 4
        with pytest.raises(RuntimeError, match="kappa-polynomial"):
            p.reweight_kpoly(torch.zeros((n_ext, 4, 4), dtype=torch.float64, device="cuda:0"))


def test_kpoly_full_size_sampled(torch_dev):
    """2^23 g g -> t tbar g g events, 16 points, mixed precision."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 1 << 23
    say("case kpoly full-size gg_ttgg n=2^23 mixed")
    mom = generate_events("gg_ttgg", n)
    kap = kappa_points(16)
    p = mg.Process("gg_ttgg", "mixed")
    p.set_params([{"kappa_ttg": float(k)} for k in kap])
    out = p.reweight_kpoly(to_dev(torch, mom))
    torch.cuda.synchronize()
    idx = np.concatenate([[0, n - 1], np.sort(np.random.default_rng(10).choice(n, 48, replace=False))])
    sub = np.ascontiguousarray(mom[:, :, idx])
    ref = oracle.reweight(oracle.qcd_me(4, sub, [(0.118, MT, 1.0)] + [(0.118, MT, float(k)) for k in kap]),
                          np.ones(len(idx)))
    got = out[:, torch.from_numpy(idx).to("cuda:0")].cpu().numpy()
    e = np.abs(got / ref - 1)
    say(f"  sampled W' max {e.max():.3e}")
    assert e.max() <= 1e-5
