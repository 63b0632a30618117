"""Mixed precision over whole samples, and the FP64 re-evaluation of
ill-conditioned events.

Single-precision amplitudes lose digits where a final-state gluon is nearly
collinear to a beam or to another gluon; the library re-evaluates such events
in FP64.  These tests compare every weight of the benchmark-size samples with
the FP64 kernels (themselves held to 1e-12 against the oracle by the parity
tests): the mixed-precision bar of 1e-5 must hold for every event, not only
for sampled ones.
"""
import sys

import numpy as np
import pytest

from synth import generate_events, kappa_points

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-5
TAU = 3e-3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def flagged(mom, tau):
    """Events with a gluon pair other than the beams below tau (|2 p.p|/s)."""
    n_ext = mom.shape[0]
    s = (mom[0, 0] + mom[1, 0]) ** 2 - ((mom[0, 1:] + mom[1, 1:]) ** 2).sum(axis=0)
    glu = [0, 1] + list(range(4, n_ext))
    ymin = np.full(mom.shape[2], np.inf)
    for a in range(len(glu)):
        for b in range(a + 1, len(glu)):
            i, j = glu[a], glu[b]
            if (i, j) == (0, 1):
                continue
            d = mom[i, 0] * mom[j, 0] - (mom[i, 1:] * mom[j, 1:]).sum(axis=0)
            ymin = np.minimum(ymin, np.abs(2 * d) / s)
    return ymin < tau


@pytest.mark.parametrize("name,n", [("gg_ttgg", 1 << 23), ("gg_ttg", 1 << 22)])
def test_every_mixed_weight_within_bar(torch_dev, name, n):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    say(f"case full population {name} n={n}: generating")
    mom = torch.from_numpy(generate_events(name, n)).to("cuda:0")
    kap = kappa_points(16)
    res = {}
    for prec in ("fp64", "mixed"):
        p = mg.Process(name, prec)
        p.set_params([{"kappa_ttg": float(k)} for k in kap])
        me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
        say(f"  {prec} reweight")
        out = p.reweight(mom, me_base_out=me0)
        torch.cuda.synchronize()
        res[prec] = (out, me0)
        if prec == "mixed":
            say("  mixed kappa polynomial")
            res["kpoly"] = (p.reweight_kpoly(mom), None)
            torch.cuda.synchronize()
    ref, me_ref = res["fp64"]
    e0 = (res["mixed"][1] / me_ref - 1).abs().max().item()
    say(f"  |M|^2 base: max rel err {e0:.3e}")
    assert e0 <= TOL_MIXED
    for key in ("mixed", "kpoly"):
        e = (res[key][0] / ref - 1).abs()
        emax = e.max().item()
        say(f"  {key} W': max rel err {emax:.3e}, weights above 1e-6: {(e > 1e-6).sum().item()} "
            f"of {e.numel()}")
        assert emax <= TOL_MIXED


@pytest.mark.timeout(900)
def test_gg_ttggg_every_mixed_weight_within_bar(torch_dev):
    """The full g g -> t tbar g g g workload (2^20 events in the seeded uneven
    batches, 16 points): every mixed-precision weight and base |M|^2, with the
    library's default re-evaluation threshold, against the FP64 pipeline.
    Without the re-evaluation 4 events of this sample exceed 1e-5 (max
    2.0e-5), all with a gluon invariant below 5.7e-4."""
    import paper_2312_07440_amd as mg
    from synth import uneven_batches
    torch = torch_dev
    n = 1 << 20
    say(f"case full population gg_ttggg n={n}: generating")
    mom_np = generate_events("gg_ttggg", n)
    kap = kappa_points(16)
    procs = {}
    for prec in ("fp64", "mixed"):
        procs[prec] = mg.Process("gg_ttggg", prec)
        procs[prec].set_params([{"kappa_ttg": float(k)} for k in kap])
    assert procs["mixed"].rescue_threshold == pytest.approx(1e-3)
    emax, e0 = 0.0, 0
    for s in uneven_batches("gg_ttggg", n):
        mom = torch.from_numpy(np.ascontiguousarray(mom_np[:, :, e0:e0 + s])).to("cuda:0")
        res = {}
        for prec, p in procs.items():
            me = torch.empty(s, dtype=torch.float64, device="cuda:0")
            res[prec] = (p.reweight(mom, me_base_out=me), me)
            torch.cuda.synchronize()
        e = max((res["mixed"][0] / res["fp64"][0] - 1).abs().max().item(),
                (res["mixed"][1] / res["fp64"][1] - 1).abs().max().item())
        say(f"  batch [{e0}, {e0 + s}): max rel err {e:.3e}")
        emax = max(emax, e)
        e0 += s
        del mom, res
    say(f"  every weight: max rel err {emax:.3e}")
    assert emax <= TOL_MIXED


def test_rescue_replaces_only_flagged_events(torch_dev):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 40000
    mom_np = generate_events("gg_ttgg", n, first_event=123456)
    fl = flagged(mom_np, TAU)
    say(f"case rescue selection gg_ttgg n={n}: {fl.sum()} flagged")
    assert 0 < fl.sum() < n
    mom = torch.from_numpy(mom_np).to("cuda:0")
    kap = kappa_points(4)
    outs = {}
    for label, prec, tau in (("off", "mixed", 0.0), ("on", "mixed", TAU), ("fp64", "fp64", None)):
        p = mg.Process("gg_ttgg", prec)
        p.set_params([{"kappa_ttg": float(k)} for k in kap])
        if tau is not None:
            p.set_rescue_threshold(tau)
        outs[label] = p.reweight(mom).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(outs["on"][:, ~fl], outs["off"][:, ~fl])
    assert np.abs(outs["on"][:, fl] / outs["fp64"][:, fl] - 1).max() <= 1e-12


def test_gg_ttggg_rescue_replaces_only_flagged_events(torch_dev):
    """g g -> t tbar g g g, mixed precision: the listed events go through the
    double-precision (chunk, flow range) pipeline, which takes list positions
    as slots; they then equal the FP64 call to 1e-12 and every other event is
    bit-identical to the call with the re-evaluation off."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 3000
    mom_np = generate_events("gg_ttggg", n, first_event=4242)
    fl = flagged(mom_np, TAU)
    say(f"case rescue selection gg_ttggg n={n}: {fl.sum()} flagged")
    assert 0 < fl.sum() < n
    mom = torch.from_numpy(mom_np).to("cuda:0")
    kap = kappa_points(4)
    outs = {}
    for label, prec, tau in (("off", "mixed", 0.0), ("on", "mixed", TAU), ("fp64", "fp64", None)):
        say(f"  {label}")
        p = mg.Process("gg_ttggg", prec)
        p.set_params([{"kappa_ttg": float(k)} for k in kap])
        if tau is not None:
            p.set_rescue_threshold(tau)
        me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
        outs[label] = (p.reweight(mom, me_base_out=me0).cpu().numpy(), me0.cpu().numpy())
    torch.cuda.synchronize()
    assert np.array_equal(outs["on"][0][:, ~fl], outs["off"][0][:, ~fl])
    assert np.array_equal(outs["on"][1][~fl], outs["off"][1][~fl])
    assert np.abs(outs["on"][0][:, fl] / outs["fp64"][0][:, fl] - 1).max() <= 1e-12
    assert np.abs(outs["on"][1][fl] / outs["fp64"][1][fl] - 1).max() <= 1e-12


def test_gg_ttggg_split_pipeline_repeatable_on_a_side_stream(torch_dev):
    """The double-precision pipeline of g g -> t tbar g g g runs the flow
    ranges of each chunk on the caller's stream and on library streams,
    joined per chunk: repeated calls on a stream of the caller's own, mixed
    precision (its listed events go through the pipeline) and FP64, give
    bit-identical weights, also with other work queued on the stream."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 2500
    mom_np = generate_events("gg_ttggg", n, first_event=777)
    fl = flagged(mom_np, TAU)
    say(f"case split pipeline repeatable gg_ttggg n={n}: {fl.sum()} flagged")
    assert fl.sum() > 0
    mom = torch.from_numpy(mom_np).to("cuda:0")
    kap = kappa_points(4)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for prec in ("mixed", "fp64"):
        say(f"  {prec}")
        p = mg.Process("gg_ttggg", prec)
        p.set_params([{"kappa_ttg": float(k)} for k in kap])
        if prec == "mixed":
            p.set_rescue_threshold(TAU)
        with torch.cuda.stream(side):
            a = p.reweight(mom, stream=side)
            filler = torch.ones(1 << 20, device="cuda:0").cumsum(0)   # other work on the stream
            b = p.reweight(mom, stream=side)
        side.synchronize()
        assert torch.isfinite(a).all()
        assert torch.equal(a, b)
        assert float(filler[-1]) == float(1 << 20)


def test_rescue_applies_to_eval_me(torch_dev):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 5000
    mom_np = generate_events("gg_ttg", n, first_event=99)
    fl = flagged(mom_np, TAU)
    say(f"case rescue eval_me gg_ttg n={n}: {fl.sum()} flagged")
    mom = torch.from_numpy(mom_np).to("cuda:0")
    a = mg.Process("gg_ttg", "mixed").eval_me(mom).cpu().numpy()
    b = mg.Process("gg_ttg", "fp64").eval_me(mom).cpu().numpy()
    assert fl.sum() > 0
    assert np.abs(a[fl] / b[fl] - 1).max() <= 1e-12
    assert np.abs(a / b - 1).max() <= TOL_MIXED


def test_rescue_option_errors(torch_dev):
    import paper_2312_07440_amd as mg
    say("case rescue option errors")
    with pytest.raises(RuntimeError, match="rescue"):
        mg.Process("gg_ttgg", "fp64").set_rescue_threshold(1e-3)
    with pytest.raises(RuntimeError, match="rescue"):
        mg.Process("gg_ttggg", "fp64").set_rescue_threshold(1e-3)
    mg.Process("gg_ttggg", "mixed").set_rescue_threshold(1e-3)
    with pytest.raises(RuntimeError, match="ppm"):
        mg.Process("gg_ttgg", "mixed").set_rescue_threshold(2.0)
    mg.Process("gg_ttgg", "fp64").set_rescue_threshold(0.0)
