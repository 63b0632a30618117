"""GPU parity of e+ e- -> 5 photons (the process of the paper's timing study,
Sec. 3.3 and Table 1) against the FP64 oracle, which sums the 120 diagrams
explicitly; and the closed-form reweight factor (alpha'/alpha)^5 over the
whole benchmark-size sample.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import alpha_points, generate_events

pytestmark = pytest.mark.gpu

ALPHA0 = 1 / 132.5
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


def make(prec, alphas):
    import paper_2312_07440_amd as mg
    p = mg.Process("ee_5a", prec, {"alpha": ALPHA0})
    p.set_params([{"alpha": float(a)} for a in alphas])
    return p


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_photons_parity(torch_dev, prec):
    torch = torch_dev
    n = 97
    mom = generate_events("ee_5a", n)
    al = alpha_points(4)
    w = np.random.default_rng(11).normal(size=n)
    say(f"case ee_5a parity n={n} prec={prec}")
    p = make(prec, al)
    me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    out = p.reweight(to_dev(torch, mom), w_in=to_dev(torch, w), me_base_out=me0)
    torch.cuda.synchronize()
    me_ref = oracle.ee_photons_me(mom, [ALPHA0] + list(al))
    w_ref = oracle.reweight(me_ref, w)
    e_me = np.abs(me0.cpu().numpy() / me_ref[0] - 1)
    e_w = np.abs(out.cpu().numpy() / w_ref - 1)
    say(f"  |M|^2 max {e_me.max():.3e}; W' max {e_w.max():.3e}")
    assert e_me.max() <= TOL[prec]
    assert e_w.max() <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_photons_eval_me_each_point(torch_dev, prec):
    torch = torch_dev
    n = 65
    mom = generate_events("ee_5a", n, first_event=5000)
    al = alpha_points(3)
    say(f"case ee_5a eval_me n={n} prec={prec}")
    p = make(prec, al)
    d = to_dev(torch, mom)
    ref = oracle.ee_photons_me(mom, [ALPHA0] + list(al))
    for k in range(-1, 3):
        got = p.eval_me(d, point=k).cpu().numpy()
        assert np.abs(got / ref[k + 1] - 1).max() <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_photons_closed_form_ratio_full_sample(torch_dev, prec):
    """|M|^2 is proportional to alpha^5, so every weight is W (alpha_k/alpha_0)^5:
    checked for all 2^22 events x 16 points."""
    torch = torch_dev
    n = 1 << 22
    say(f"case ee_5a closed-form ratio n=2^22 prec={prec}")
    mom = to_dev(torch, generate_events("ee_5a", n))
    al = alpha_points(16)
    p = make(prec, al)
    out = p.reweight(mom)
    torch.cuda.synchronize()
    r = torch.from_numpy((al / ALPHA0) ** 5).to("cuda:0")[:, None]
    e = (out / r - 1).abs()
    say(f"  max rel err {e.max().item():.3e}")
    assert e.max().item() <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_photons_coupling_polynomial(torch_dev, prec):
    """mgrw_reweight_kpoly on this process: one evaluation at e = 1, every
    point as e^10 times it."""
    torch = torch_dev
    n = 97
    mom = generate_events("ee_5a", n, first_event=777)
    al = alpha_points(4)
    say(f"case ee_5a coupling polynomial n={n} prec={prec}")
    p = make(prec, al)
    me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    out = p.reweight_kpoly(to_dev(torch, mom), me_base_out=me0).cpu().numpy()
    me_ref = oracle.ee_photons_me(mom, [ALPHA0])[0]
    assert np.abs(me0.cpu().numpy() / me_ref - 1).max() <= TOL[prec]
    assert np.abs(out / ((al / ALPHA0) ** 5)[:, None] - 1).max() <= 1e-13


@pytest.mark.parametrize("n", [0, 1, 63, 257])
def test_photons_ragged(torch_dev, n):
    torch = torch_dev
    say(f"case ee_5a ragged n={n}")
    mom = generate_events("ee_5a", max(n, 1), first_event=31)[:, :, :n]
    al = alpha_points(2)
    p = make("fp64", al)
    out = torch.full((2, n), -5.0, dtype=torch.float64, device="cuda:0")
    p.reweight(to_dev(torch, mom), out=out)
    torch.cuda.synchronize()
    if n:
        assert np.abs(out.cpu().numpy() / ((al / ALPHA0) ** 5)[:, None] - 1).max() <= 1e-12


def test_photons_options_rejected(torch_dev):
    say("case ee_5a option errors")
    p = make("mixed", alpha_points(1))
    with pytest.raises(RuntimeError):
        p.set_lane_mapping("event_per_lane")
    with pytest.raises(RuntimeError, match="rescue"):
        p.set_rescue_threshold(1e-3)
    p.set_lane_mapping("event_per_wave")
