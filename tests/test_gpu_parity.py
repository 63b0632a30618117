"""GPU parity: libmgrw (through its C ABI) against the FP64 oracle.

Bars: FP64 arithmetic <= 1e-12 relative per event; mixed precision <= 1e-5
relative per event (|M|^2 and reweighted weights).  Sizes span several
256-lane blocks with a ragged tail; the full-size case uses the benchmark's
launch configuration and compares sampled events.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import generate_events, kappa_points

pytestmark = pytest.mark.gpu

ALS, MT = 0.118, 173.0
EW = dict(alpha=1 / 132.5, sw2=0.2312, mz=91.1876, wz=2.4952)
NG = {"gg_tt": 2, "gg_ttg": 3, "gg_ttgg": 4, "gg_ttggg": 5}
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


def qcd_case(name, n, seed_shift=0):
    mom = generate_events(name, n, first_event=seed_shift)
    kap = kappa_points(16)
    w = np.random.default_rng(5).normal(size=n)
    return mom, kap, w


def oracle_qcd(name, mom, kap, w, base_kappa=1.0):
    me = oracle.qcd_me(NG[name], mom, [(ALS, MT, base_kappa)] + [(ALS, MT, k) for k in kap])
    return me, oracle.reweight(me, w)


def relerr(a, b):
    return np.abs(a / b - 1)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name,n", [("gg_tt", 1031), ("gg_ttg", 517), ("gg_ttgg", 261)])
def test_qcd_reweight_parity(torch_dev, name, n, prec):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    mom, kap, w = qcd_case(name, n)
    say(f"case reweight {name} n={n} prec={prec}")
    p = mg.Process(name, prec, {"alphas": ALS, "mt": MT})
    p.set_params([{"alphas": ALS, "mt": MT, "kappa_ttg": float(k)} for k in kap])
    me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    out = p.reweight(to_dev(torch, mom), w_in=to_dev(torch, w), me_base_out=me0)
    torch.cuda.synchronize()
    me_ref, w_ref = oracle_qcd(name, mom, kap, w)
    e_me = relerr(me0.cpu().numpy(), me_ref[0])
    e_w = relerr(out.cpu().numpy(), w_ref)
    say(f"  |M|^2 rel err max {e_me.max():.3e} median {np.median(e_me):.3e}; "
        f"W' rel err max {e_w.max():.3e} p99 {np.quantile(e_w, 0.99):.3e} median {np.median(e_w):.3e}")
    assert e_me.max() <= TOL[prec]
    assert e_w.max() <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [1, 97, 261])
def test_event_per_wave_mapping_parity(torch_dev, prec, n):
    """The one-event-per-wave kernels (helicities on the lanes) against the
    oracle, including a single event and a ragged count."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    mom, kap, w = qcd_case("gg_ttgg", n, seed_shift=500)
    say(f"case event-per-wave gg_ttgg n={n} prec={prec}")
    p = mg.Process("gg_ttgg", prec)
    p.set_lane_mapping("event_per_wave")
    p.set_params([{"kappa_ttg": float(k)} for k in kap])
    me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    out = p.reweight(to_dev(torch, mom), w_in=to_dev(torch, w), me_base_out=me0)
    me_b = p.eval_me(to_dev(torch, mom), 3)
    torch.cuda.synchronize()
    me_ref, w_ref = oracle_qcd("gg_ttgg", mom, kap, w)
    assert relerr(me0.cpu().numpy(), me_ref[0]).max() <= TOL[prec]
    assert relerr(out.cpu().numpy(), w_ref).max() <= TOL[prec]
    assert relerr(me_b.cpu().numpy(), me_ref[4]).max() <= TOL[prec]


def test_lane_mapping_option_errors(torch_dev):
    import paper_2312_07440_amd as mg
    from paper_2312_07440_amd import binding as bd
    with pytest.raises(bd.MgrwError) as e:
        mg.Process("gg_ttg", "mixed").set_lane_mapping("event_per_wave")   # 32 helicities
    assert e.value.status == bd.ERR_UNSUPPORTED


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_qcd_eval_me_points(torch_dev, prec):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    name, n = "gg_ttg", 300
    mom, kap, _ = qcd_case(name, n)
    say(f"case eval_me {name} n={n} prec={prec}")
    p = mg.Process(name, prec)
    p.set_params([{"kappa_ttg": float(k)} for k in kap])
    d = to_dev(torch, mom)
    me_b = p.eval_me(d, -1)
    me_5 = p.eval_me(d, 5)
    torch.cuda.synchronize()
    ref = oracle.qcd_me(3, mom, [(ALS, MT, 1.0), (ALS, MT, float(kap[5]))])
    assert relerr(me_b.cpu().numpy(), ref[0]).max() <= TOL[prec]
    assert relerr(me_5.cpu().numpy(), ref[1]).max() <= TOL[prec]


def test_ee_mumu_parity(torch_dev):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 1031
    mom = generate_events("ee_mumu", n)
    say(f"case ee_mumu n={n}")
    p = mg.Process("ee_mumu", "fp64", EW)
    p.set_params([dict(EW, mz=95.0)])
    me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    out = p.reweight(to_dev(torch, mom), me_base_out=me0)
    torch.cuda.synchronize()
    pts = [tuple(EW.values()), (EW["alpha"], EW["sw2"], 95.0, EW["wz"])]
    ref = oracle.ee_mumu_me(mom, pts)
    assert relerr(me0.cpu().numpy(), ref[0]).max() <= 1e-12
    assert relerr(out.cpu().numpy()[0], oracle.reweight(ref)[0]).max() <= 1e-12


@pytest.mark.parametrize("n", [1, 63, 64, 65, 257])
def test_ragged_sizes(torch_dev, n):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    mom, kap, w = qcd_case("gg_ttg", n, seed_shift=1000)
    say(f"case ragged gg_ttg n={n}")
    p = mg.Process("gg_ttg", "fp64")
    p.set_params([{"kappa_ttg": float(k)} for k in kap[:3]])
    out = p.reweight(to_dev(torch, mom), w_in=to_dev(torch, w))
    torch.cuda.synchronize()
    me = oracle.qcd_me(3, mom, [(ALS, MT, 1.0)] + [(ALS, MT, float(k)) for k in kap[:3]])
    assert relerr(out.cpu().numpy(), oracle.reweight(me, w)).max() <= 1e-12


def test_zero_events_launches_nothing(torch_dev):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    p = mg.Process("gg_tt", "mixed")
    p.set_params([{"kappa_ttg": 1.1}])
    mom = torch.zeros((4, 4, 0), dtype=torch.float64, device="cuda:0")
    out = p.reweight(mom)
    torch.cuda.synchronize()
    assert out.shape == (1, 0)


def test_nan_where_base_me_vanishes(torch_dev):
    """kappa = 0 at the base point makes every diagram vanish: |M|^2 = 0 and
    eq. (3) is undefined -> NaN."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 100
    mom, _, w = qcd_case("gg_ttg", n)
    say("case nan base kappa=0")
    p = mg.Process("gg_ttg", "mixed", {"kappa_ttg": 0.0})
    p.set_params([{"kappa_ttg": 1.0}, {"kappa_ttg": 0.0}])
    me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    out = p.reweight(to_dev(torch, mom), w_in=to_dev(torch, w), me_base_out=me0)
    torch.cuda.synchronize()
    assert np.all(me0.cpu().numpy() == 0.0)
    assert np.all(np.isnan(out.cpu().numpy()))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_same_point_gives_input_weight(torch_dev, prec):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 200
    mom, _, w = qcd_case("gg_ttgg", n)
    p = mg.Process("gg_ttgg", prec)
    p.set_params([{"kappa_ttg": 1.0}])
    out = p.reweight(to_dev(torch, mom), w_in=to_dev(torch, w))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy()[0], w)


def test_stream_ordering_and_determinism(torch_dev):
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 4097
    mom, kap, w = qcd_case("gg_ttg", n)
    p = mg.Process("gg_ttg", "mixed")
    p.set_params([{"kappa_ttg": float(k)} for k in kap])
    d = to_dev(torch, mom)
    a = p.reweight(d)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = p.reweight(d, stream=s)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_host_pointer_rejected(torch_dev):
    import paper_2312_07440_amd as mg
    from paper_2312_07440_amd import binding as bd
    import ctypes
    p = mg.Process("gg_tt", "mixed")
    p.set_params([{"kappa_ttg": 1.1}])
    host = np.zeros((4, 4, 8))
    out = np.zeros(8)
    st = bd.lib().mgrw_reweight(p._h, ctypes.c_void_p(host.ctypes.data), None, 8,
                                ctypes.c_void_p(out.ctypes.data), None, None)
    assert st == bd.ERR_ARG


def test_full_size_sampled_parity(torch_dev):
    """g g -> t tbar g g at the benchmark's size (2^23 events, 16 points,
    mixed precision), sampled events against the oracle."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 1 << 23
    say("case full-size gg_ttgg n=2^23 mixed: generating events")
    mom = generate_events("gg_ttgg", n)
    kap = kappa_points(16)
    p = mg.Process("gg_ttgg", "mixed")
    p.set_params([{"kappa_ttg": float(k)} for k in kap])
    d = to_dev(torch, mom)
    me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    say("  launching")
    out = p.reweight(d, me_base_out=me0)
    torch.cuda.synchronize()
    say("  done; oracle on samples")
    idx = np.sort(np.random.default_rng(9).choice(n, 48, replace=False))
    idx = np.concatenate([[0, n - 1], idx])
    sub = np.ascontiguousarray(mom[:, :, idx])
    me_ref, w_ref = oracle_qcd("gg_ttgg", sub, kap, np.ones(len(idx)))
    got = out[:, torch.from_numpy(idx).to("cuda:0")].cpu().numpy()
    e = relerr(got, w_ref)
    say(f"  sampled W' rel err max {e.max():.3e} median {np.median(e):.3e}")
    assert relerr(me0[torch.from_numpy(idx).to("cuda:0")].cpu().numpy(), me_ref[0]).max() <= 1e-5
    assert e.max() <= 1e-5


@pytest.mark.parametrize("n", [1, 70])
def test_gg_ttggg_parity(torch_dev, n):
    """g g -> t tbar g g g (1240 diagrams, 120 flows, program split over
    kernels), mixed precision, against the oracle."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    mom, kap, w = qcd_case("gg_ttggg", n, seed_shift=300)
    kap = kap[::4]
    say(f"case gg_ttggg n={n}")
    p = mg.Process("gg_ttggg", "mixed")
    p.set_params([{"kappa_ttg": float(k)} for k in kap])
    me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    out = p.reweight(to_dev(torch, mom), w_in=to_dev(torch, w), me_base_out=me0)
    torch.cuda.synchronize()
    me_ref, w_ref = oracle_qcd("gg_ttggg", mom, kap, w)
    e_me, e_w = relerr(me0.cpu().numpy(), me_ref[0]), relerr(out.cpu().numpy(), w_ref)
    say(f"  |M|^2 rel err max {e_me.max():.3e}; W' rel err max {e_w.max():.3e} median {np.median(e_w):.3e}")
    assert e_me.max() <= TOL["mixed"]
    assert e_w.max() <= TOL["mixed"]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_gg_ttggg_varied_alphas(torch_dev, prec):
    """g g -> t tbar g g g with alpha_s and kappa varied per point: its
    programs run at unit strong coupling and restore g_s^10 on |M|^2 per
    point, in both the single-precision parts and the FP64 pipeline."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 6
    mom = generate_events("gg_ttggg", n, first_event=555)
    kap = kappa_points(4)
    als = [0.100, 0.112, 0.125, 0.135]
    w = np.random.default_rng(12).normal(size=n)
    say(f"case gg_ttggg varied alpha_s prec={prec} n={n}")
    p = mg.Process("gg_ttggg", prec, {"alphas": ALS, "mt": MT})
    p.set_params([{"alphas": a, "mt": MT, "kappa_ttg": float(k)} for a, k in zip(als, kap)])
    me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    out = p.reweight(to_dev(torch, mom), w_in=to_dev(torch, w), me_base_out=me0)
    torch.cuda.synchronize()
    me = oracle.qcd_me(5, mom, [(ALS, MT, 1.0)] + [(a, MT, float(k)) for a, k in zip(als, kap)])
    ref = oracle.reweight(me, w)
    e_me, e_w = relerr(me0.cpu().numpy(), me[0]), relerr(out.cpu().numpy(), ref)
    say(f"  |M|^2 rel err max {e_me.max():.3e}; W' rel err max {e_w.max():.3e}")
    assert e_me.max() <= TOL[prec]
    assert e_w.max() <= TOL[prec]


@pytest.mark.parametrize("n", [1, 70])
def test_gg_ttggg_fp64_parity(torch_dev, n):
    """g g -> t tbar g g g in FP64 (the program cut by closing-group chunk and
    colour-flow range, J through device memory, double colour sum) against
    the oracle at the FP64 bar, with input weights of both signs."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    mom, kap, w = qcd_case("gg_ttggg", n, seed_shift=900)
    kap = kap[::4]
    say(f"case gg_ttggg fp64 n={n}")
    p = mg.Process("gg_ttggg", "fp64")
    p.set_params([{"kappa_ttg": float(k)} for k in kap])
    me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    out = p.reweight(to_dev(torch, mom), w_in=to_dev(torch, w), me_base_out=me0)
    me3 = p.eval_me(to_dev(torch, mom), 2)
    torch.cuda.synchronize()
    me_ref, w_ref = oracle_qcd("gg_ttggg", mom, kap, w)
    e_me, e_w = relerr(me0.cpu().numpy(), me_ref[0]), relerr(out.cpu().numpy(), w_ref)
    e3 = relerr(me3.cpu().numpy(), me_ref[3])
    say(f"  |M|^2 rel err max {e_me.max():.3e}; point 2 {e3.max():.3e}; W' rel err max {e_w.max():.3e}")
    assert e_me.max() <= TOL["fp64"]
    assert e3.max() <= TOL["fp64"]
    assert e_w.max() <= TOL["fp64"]


def test_gg_ttggg_fp64_batch_boundary(torch_dev):
    """FP64 g g -> t tbar g g g over more events than one internal batch
    (8192 at three points): events on both sides of the boundary and at the
    ends against the oracle at the FP64 bar."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 8192 + 37
    mom, kap, _ = qcd_case("gg_ttggg", n, seed_shift=7000)
    kap = kap[::8]
    say(f"case gg_ttggg fp64 batch boundary n={n}")
    p = mg.Process("gg_ttggg", "fp64")
    p.set_params([{"kappa_ttg": float(k)} for k in kap])
    out = p.reweight(to_dev(torch, mom)).cpu().numpy()
    torch.cuda.synchronize()
    assert np.isfinite(out).all()
    idx = np.array([0, 1, 4000, 8190, 8191, 8192, 8193, n - 2, n - 1])
    sub = np.ascontiguousarray(mom[:, :, idx])
    _, w_ref = oracle_qcd("gg_ttggg", sub, kap, np.ones(len(idx)))
    e = relerr(out[:, idx], w_ref)
    say(f"  sampled W' rel err max {e.max():.3e}")
    assert e.max() <= TOL["fp64"]


def test_gg_ttggg_batch_boundary(torch_dev):
    """More events than one internal batch (8192): events on both sides of
    the boundary and at the ends, against the oracle."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 8192 + 37
    mom, kap, _ = qcd_case("gg_ttggg", n, seed_shift=7000)
    kap = kap[::8]
    say(f"case gg_ttggg batch boundary n={n}")
    p = mg.Process("gg_ttggg", "mixed")
    p.set_params([{"kappa_ttg": float(k)} for k in kap])
    out = p.reweight(to_dev(torch, mom))
    torch.cuda.synchronize()
    idx = np.array([0, 1, 4000, 8190, 8191, 8192, 8193, n - 2, n - 1])
    sub = np.ascontiguousarray(mom[:, :, idx])
    _, w_ref = oracle_qcd("gg_ttggg", sub, kap, np.ones(len(idx)))
    assert relerr(out.cpu().numpy()[:, idx], w_ref).max() <= TOL["mixed"]


def test_gg_ttggg_full_configuration_uneven_batches(torch_dev):
    """The full g g -> t tbar g g g workload: 2^20 events handed over in
    seeded uneven batches of 65 536..262 144 events (the last one the
    remainder), 16 points; sampled events against the oracle."""
    import paper_2312_07440_amd as mg
    from synth import uneven_batches
    from synth.phase_space import PROCESSES
    torch = torch_dev
    spec = PROCESSES["gg_ttggg"]
    n = spec.n_events
    say(f"case gg_ttggg full configuration n={n}: generating events")
    mom = generate_events("gg_ttggg", n)
    kap = kappa_points(16)
    p = mg.Process("gg_ttggg", "mixed")
    p.set_params([{"kappa_ttg": float(k)} for k in kap])
    sizes = uneven_batches("gg_ttggg", n)
    out = np.empty((16, n))
    e0 = 0
    for s in sizes:
        say(f"  batch [{e0}, {e0 + s})")
        o = p.reweight(to_dev(torch, mom[:, :, e0:e0 + s]))
        torch.cuda.synchronize()
        out[:, e0:e0 + s] = o.cpu().numpy()
        e0 += s
    idx = np.sort(np.random.default_rng(4).choice(n, 24, replace=False))
    idx = np.unique(np.concatenate([idx, [0, n - 1], np.cumsum(sizes)[:-1], np.cumsum(sizes)[:-1] - 1]))
    sub = np.ascontiguousarray(mom[:, :, idx])
    say(f"  oracle on {len(idx)} sampled events")
    _, w_ref = oracle_qcd("gg_ttggg", sub, kap, np.ones(len(idx)))
    e = relerr(out[:, idx], w_ref)
    say(f"  batches {sizes}; sampled W' rel err max {e.max():.3e} median {np.median(e):.3e}")
    assert e.max() <= TOL["mixed"]


def test_kernel_timing(torch_dev):
    """HIP events recorded by the library around its amplitude kernel lie
    inside the caller's events around the whole call."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    say("case kernel timing gg_ttgg n=4096")
    p = mg.Process("gg_ttgg", "mixed")
    p.set_params([{"kappa_ttg": float(k)} for k in kappa_points(4)])
    mom = to_dev(torch, generate_events("gg_ttgg", 4096))
    with pytest.raises(RuntimeError):
        p.kernel_time_ms()
    p.set_kernel_timing(True)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    p.reweight(mom)
    e.record()
    t = p.kernel_time_ms()
    torch.cuda.synchronize()
    step = s.elapsed_time(e)
    say(f"  kernel {t:.3f} ms, call {step:.3f} ms")
    assert 0 < t <= step
    p.set_kernel_timing(False)
    with pytest.raises(RuntimeError):
        p.kernel_time_ms()


@pytest.mark.parametrize("n", [70, 8229])
def test_gg_ttggg_matrix_core_colour_sum(torch_dev, n):
    """The colour sum of g g -> t tbar g g g on the matrix cores (bfloat16-split
    operands, float32 accumulation) against the VALU colour sum and, for the
    small case, the oracle."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    say(f"case gg_ttggg matrix-core colour sum n={n}")
    mom = generate_events("gg_ttggg", n, first_event=555)
    kap = kappa_points(4)
    outs = []
    for mf in (True, False):
        p = mg.Process("gg_ttggg", "mixed")
        p.set_params([{"kappa_ttg": float(k)} for k in kap])
        if mf:
            p.set_colour_mfma(True)
        me0 = torch.empty(n, dtype=torch.float64, device="cuda:0")
        out = p.reweight(to_dev(torch, mom), me_base_out=me0)
        torch.cuda.synchronize()
        outs.append((out.cpu().numpy(), me0.cpu().numpy()))
    e = relerr(outs[0][0], outs[1][0]).max()
    e0 = relerr(outs[0][1], outs[1][1]).max()
    say(f"  matrix cores vs VALU: |M|^2 {e0:.3e}, W' {e:.3e}")
    assert e <= 1e-5 and e0 <= 1e-5
    if n <= 100:
        me_ref, w_ref = oracle_qcd("gg_ttggg", mom, kap, np.ones(n))
        assert relerr(outs[0][1], me_ref[0]).max() <= TOL["mixed"]
        assert relerr(outs[0][0], w_ref).max() <= TOL["mixed"]


def test_maximum_points_and_varied_couplings(torch_dev):
    """64 new points (the maximum) that vary alpha_s as well as kappa, with input
    weights of both signs and zeros, g g -> t tbar g g (mixed, event per wave)."""
    import paper_2312_07440_amd as mg
    torch = torch_dev
    n = 65
    say(f"case 64 points, varied alpha_s, gg_ttgg n={n}")
    mom = generate_events("gg_ttgg", n, first_event=31337)
    w = np.random.default_rng(8).normal(size=n)
    w[::7] = 0.0
    kap = kappa_points(64)
    als = np.linspace(0.09, 0.14, 64)
    p = mg.Process("gg_ttgg", "mixed")
    p.set_params([{"alphas": float(a), "kappa_ttg": float(k)} for a, k in zip(als, kap)])
    out = p.reweight(to_dev(torch, mom), w_in=to_dev(torch, w)).cpu().numpy()
    me = oracle.qcd_me(4, mom, [(ALS, MT, 1.0)] + [(float(a), MT, float(k)) for a, k in zip(als, kap)])
    ref = oracle.reweight(me, w)
    nz = w != 0
    assert np.all(out[:, ~nz] == 0)
    assert relerr(out[:, nz], ref[:, nz]).max() <= TOL["mixed"]
