#!/usr/bin/env python3
"""Benchmark: reweighted events/s x 16 parameter points, g g -> t tbar g g.

One step = one call of mgrw_reweight over the whole batch: the base |M|^2 and
the 16 new points are evaluated in full for every event (Sec. 3.2, steps 3-8)
and the 16 reweighted weights written (eq. (3)).  Inputs (seeded synthetic
events, 2^23 by default) are resident in device memory before the timed
region.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (the packed rate)
PEAK_FP64_TFLOPS = 78.6
HBM_TBS = 8.0
ALPHA0 = 1 / 132.5


# HBM traffic of the exact amplitude kernel measured with rocprofv3 FETCH_SIZE /
# WRITE_SIZE (copy-calibrated; see profiles/), valid only for the sources that
# kernel is built from: keyed by a fingerprint of those sources.
MEASURED_TRAFFIC = {("gg_ttgg", "mixed", "0ed74d1fbbe9ee7b"): 2398.2}   # bytes per event per launch
WAVE_SECTION = ("// ------------------------------------------------ one event per wave",
                "// ------------------------------------------------ kappa-polynomial kernels")


def kernel_fingerprint(proc="gg_ttgg"):
    """sha256 prefix of the one-event-per-wave kernel section of mgrw_kernels.h,
    the Lorentz and event headers and the generated program of the process."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "paper_2312_07440_amd", "csrc")
    if not os.path.exists(os.path.join(csrc, "gen", f"{proc}.inc")):
        return None
    k = open(os.path.join(csrc, "mgrw_kernels.h")).read()
    h.update(k[k.index(WAVE_SECTION[0]):k.index(WAVE_SECTION[1])].encode())
    for f in ("mgrw_lorentz.h", "mgrw_event.h", os.path.join("gen", f"{proc}.inc")):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


# Executed FP32 flops of the amplitude kernel over the counted (algorithmic)
# flops of the events it evaluates, from SQ_INSTS_VALU_{FMA,MUL,ADD}_F32
# (profiles/), for the same kernel sources as MEASURED_TRAFFIC.
MEASURED_EXEC_RATIO = {("gg_ttgg", "mixed", "0ed74d1fbbe9ee7b"): 0.861}
def rescued_events(mom_np, tau):
    """Events the mixed-precision call leaves to its FP64 re-evaluation: a
    gluon pair other than the two beams with |2 p_i.p_j| / s below tau (the
    library's criterion, evaluated here in float64)."""
    n_ext = mom_np.shape[0]
    p = mom_np
    s = (p[0, 0] + p[1, 0]) ** 2 - ((p[0, 1:] + p[1, 1:]) ** 2).sum(axis=0)
    glu = [0, 1] + list(range(4, n_ext))
    bad = np.zeros(p.shape[2], dtype=bool)
    for a in range(len(glu)):
        for b in range(a + 1, len(glu)):
            i, j = glu[a], glu[b]
            if (i, j) == (0, 1):
                continue
            d = p[i, 0] * p[j, 0] - p[i, 1] * p[j, 1] - p[i, 2] * p[j, 2] - p[i, 3] * p[j, 3]
            bad |= np.abs(2.0 * d) < tau * s
    return int(bad.sum())


def host_info():
    """CPU model and logical CPUs of the host, and the CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc_online": os.cpu_count(), "cpus_usable": len(os.sched_getaffinity(0))}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_per_event(proc, n_points_total, n_hel):
    path = os.path.join(HERE, "paper_2312_07440_amd", "csrc", "gen", "flops.json")
    f = json.load(open(path))[proc]
    n_hel = f.get("evaluated_helicities", n_hel)
    per = f["per_helicity_flops"]
    if n_hel == 64 and "external_flops" in f:
        # one block of 64 configurations per wave: the external wavefunctions
        # are assembled once per event, not once per point
        ext = f["external_flops"]
        return n_hel * (n_points_total * (per - ext) + ext), f
    return n_points_total * n_hel * per, f


def cpu_baseline(proc, ng, mom_np, kap, gpu_out, sample, points_per_event):
    """The oracle (FP64, OpenMP) on a bounded sample of the same workload."""
    import oracle

    def run(m):
        sub = np.ascontiguousarray(mom_np[:, :, :m])
        t0 = time.perf_counter()
        if proc == "ee_5a":
            me = oracle.ee_photons_me(sub, [ALPHA0] + [float(a) for a in kap])
        else:
            me = oracle.qcd_me(ng, sub, [(0.118, 173.0, 1.0)] + [(0.118, 173.0, float(k)) for k in kap])
        w = oracle.reweight(me)
        return w, time.perf_counter() - t0

    cores = oracle.max_threads()
    info = host_info()
    w, dt = run(sample)
    err = np.abs(gpu_out[:, :sample] / w - 1)
    # one thread on a sixteenth of the sample
    oracle.set_threads(1)
    s1 = max(1, sample // 16)
    _, dt1 = run(s1)
    oracle.set_threads(cores)
    return {"value": sample * points_per_event / dt, "unit": "events*points/s", "cores": cores,
            "kind": "oracle",
            "sample": f"first {sample} events of the same sample, base + {len(kap)} points, FP64 oracle "
                      f"({dt:.1f} s wall)",
            "host": info, "build": " ".join(["gcc"] + oracle.CFLAGS),
            "single_thread": {"value": s1 * points_per_event / dt1, "events": s1, "seconds": dt1}}, \
        float(err.max()), float(np.median(err))


def surrogate_leg(args, proc, mom, exact_out, kap, torch, generate_events, exact_ms, kpoly_ms):
    """Train the MLP on disjoint events (labels from the exact kernels), then
    time the audited surrogate reweight of the same batch; error measured
    against the exact weights.  Also: the time per batch with the training
    included, the number of batches after which the training has paid for
    itself against each exact path, and the same network fitted to the 25
    inputs of the workload's definition (momenta and kappa only)."""
    log(f"surrogate: generating {args.train_events} training events")
    train = torch.from_numpy(generate_events(args.proc, args.train_events, first_event=1 << 26)).to(mom.device)

    def fit():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = proc.train_surrogate(train, epochs=args.epochs, batch=16384, lr=2e-3, lr_decay=0.7, seed=3003)
        torch.cuda.synchronize()
        return losses, time.perf_counter() - t0

    def calls(sout, n_calls, bound=0.01):
        proc.reweight_surrogate(mom, out=sout, audit_fraction=args.audit, seed=7, max_audit_error=1.0)
        torch.cuda.synchronize()
        times, stats, fb = [], None, False
        for i in range(n_calls):
            t0 = time.perf_counter()
            _, stats, fb = proc.reweight_surrogate(mom, out=sout, audit_fraction=args.audit, seed=7 + i,
                                                   max_audit_error=bound)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        err = torch.abs(sout / exact_out - 1.0)
        return 1e3 * float(np.mean(times)), err, stats, fb

    losses, t_train = fit()
    log(f"surrogate: trained in {t_train:.2f}s, losses {losses}")
    sout = torch.empty_like(exact_out)
    ms, err, stats, fb = calls(sout, args.steps)
    e_mean = float(err.mean())
    e_p99 = float(torch.quantile(err.flatten()[:: max(1, err.numel() // 4000000)].float(), 0.99))
    work = args.n * args.points
    res = {"value": work / (ms * 1e-3), "unit": "events*points/s", "ms_per_step": ms,
           "mean_abs_weight_err": e_mean, "p99_abs_weight_err": e_p99, "audit_fraction": args.audit,
           "audit_mean_err_estimate": float(np.mean(stats[:, 2])), "fell_back": bool(fb),
           "train_events": args.train_events, "epochs": args.epochs, "train_seconds": t_train,
           "final_loss": float(losses[-1]), "inputs": 53,
           "timing": "host wall clock per call (the call synchronises once for the audit statistics)",
           "amortised": {
               "value_one_batch_with_training": work / (t_train + ms * 1e-3),
               "break_even_batches_vs_exact": t_train / ((exact_ms - ms) * 1e-3),
               "break_even_batches_vs_kpoly": (t_train / ((kpoly_ms - ms) * 1e-3)) if kpoly_ms else None,
               "note": "training (exact labels included) + one audited call per batch of the same size; "
                       "break-even = batches after which training plus calls cost less than the exact path"}}
    # the workload's 25 inputs (momentum components and kappa), same training
    proc.set_surrogate_inputs(25)
    losses25, t25 = fit()
    # no fallback: the network's own error (an audit bound of 1 % would fall
    # back to the exact path where it exceeds that)
    ms25, err25, st25, _ = calls(sout, 1, bound=1.0)
    proc.set_surrogate_inputs(53)
    log(f"surrogate (25 inputs): trained in {t25:.2f}s, mean err {float(err25.mean()):.4f}")
    res["inputs_25"] = {"mean_abs_weight_err": float(err25.mean()), "final_loss": float(losses25[-1]),
                        "audit_mean_err_estimate": float(np.mean(st25[:, 2])), "train_seconds": t25,
                        "falls_back_at_1pct": bool((st25[:, 2] > 0.01).any())}
    del train
    return res


def kpoly_leg(args, proc, mom, exact_out, stream, torch, n_eval):
    """The kappa-polynomial exact variant on the same batch and points: timed
    with device events like the main leg, checked against its weights."""
    kout = torch.empty_like(exact_out)
    for _ in range(args.warmup):
        proc.reweight_kpoly(mom, out=kout)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    kms = []
    for i in range(args.steps):
        starts[i].record(stream)
        proc.reweight_kpoly(mom, out=kout)
        ends[i].record(stream)
        kms.append(proc.kernel_time_ms())
    torch.cuda.synchronize()
    ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    kms = float(np.mean(kms))
    f = json.load(open(os.path.join(HERE, "paper_2312_07440_amd", "csrc", "gen", "flops.json")))[args.proc]
    fpe = (f["evaluated_helicities"] * f["per_helicity_flops"] if args.proc == "ee_5a"
           else proc.n_hel * f["kpoly_per_helicity_flops"])
    achieved = fpe * n_eval / (kms * 1e-3) / 1e12   # the events its kernel evaluates
    peak = PEAK_FP32_TFLOPS if args.prec == "mixed" else PEAK_FP64_TFLOPS
    diff = float(torch.abs(kout / exact_out - 1.0).max())
    return {"value": args.n * args.points / (ms * 1e-3), "unit": "events*points/s", "ms_per_step": ms,
            "path": "exact, kappa polynomial (one unit-coupling program per helicity for all points)",
            "max_rel_diff_vs_exact": diff,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                         "frac": achieved / peak, "kernel_ms": kms, "flops_per_event": fpe}}


def time_calls(fn, reps, stream, torch):
    """Mean, min and max device time (ms) of `reps` calls of fn after one warm-up."""
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for s, e in ev:
        s.record(stream)
        fn()
        e.record(stream)
    torch.cuda.synchronize()
    t = [s.elapsed_time(e) for s, e in ev]
    return float(np.mean(t)), float(np.min(t)), float(np.max(t))


def end_to_end_leg(args, proc, mom_np, mom, out, stream, torch):
    """The same call with the events in (pinned) host memory and the weights
    copied back: host-to-device copy of the momenta, the reweight, the
    device-to-host copy of the weights, each timed with device events."""
    h_mom = torch.empty(mom_np.shape, dtype=torch.float64, pin_memory=True)
    h_mom.numpy()[...] = mom_np
    h_out = torch.empty(tuple(out.shape), dtype=torch.float64, pin_memory=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    best = None
    for _ in range(2):   # the first pass warms the copy engines
        ev[0].record(stream)
        mom.copy_(h_mom, non_blocking=True)
        ev[1].record(stream)
        proc.reweight(mom, out=out)
        ev[2].record(stream)
        h_out.copy_(out, non_blocking=True)
        ev[3].record(stream)
        torch.cuda.synchronize()
        best = [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
    total = float(sum(best))
    # the library's chunked host-memory call: copies of one chunk overlap the
    # kernels of the other (two streams)
    proc.reweight_host(h_mom, out=h_out)
    t0 = time.perf_counter()
    proc.reweight_host(h_mom, out=h_out)
    piped = 1e3 * (time.perf_counter() - t0)
    return {"value": args.n * args.points / (total * 1e-3), "unit": "events*points/s", "ms_per_step": total,
            "h2d_ms": best[0], "reweight_ms": best[1], "d2h_ms": best[2],
            "pipelined_value": args.n * args.points / (piped * 1e-3), "pipelined_ms": piped,
            "h2d_bytes": int(mom_np.nbytes), "d2h_bytes": int(out.numel() * 8),
            "path": "events in pinned host memory: copy in, exact reweight, weights copied out"}


def sweep(args, mom_np, kappa_points, mg, torch):
    """Run time against the number of events (16 points) and against the
    number of points (2^21 events): the paper's two scaling studies (Sec. 3.3)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    n_sweep, p_sweep = [], []
    proc = mg.Process(args.proc, args.prec)
    proc.set_params([{"kappa_ttg": float(k)} for k in kappa_points(16)])
    for e in list(range(10, 23, 2)) + [23]:
        n = min(1 << e, mom_np.shape[2])
        mom = torch.from_numpy(np.ascontiguousarray(mom_np[:, :, :n])).to(dev)
        out = torch.empty((16, n), dtype=torch.float64, device=dev)
        ms, lo, hi = time_calls(lambda: proc.reweight(mom, out=out), 3, stream, torch)
        log(f"sweep N={n}: {ms:.2f} ms")
        n_sweep.append({"events": n, "ms": ms, "min_ms": lo, "max_ms": hi,
                        "events_points_per_s": n * 16 / (ms * 1e-3)})
        del mom, out
    n = min(1 << 21, mom_np.shape[2])
    mom = torch.from_numpy(np.ascontiguousarray(mom_np[:, :, :n])).to(dev)
    for P in (1, 2, 4, 8, 16, 32, 64):
        pr = mg.Process(args.proc, args.prec)
        pr.set_params([{"kappa_ttg": float(k)} for k in kappa_points(P)])
        out = torch.empty((P, n), dtype=torch.float64, device=dev)
        ms, lo, hi = time_calls(lambda: pr.reweight(mom, out=out), 3, stream, torch)
        log(f"sweep P={P}: {ms:.2f} ms")
        p_sweep.append({"points": P, "ms": ms, "min_ms": lo, "max_ms": hi,
                        "events_points_per_s": n * P / (ms * 1e-3)})
        del out, pr
    return {"metric": f"reweight call time vs events and vs points, {args.proc}, {args.prec} precision",
            "unit": "ms", "n_gpus": 1, "data": "synthetic", "events_sweep_points": 16,
            "points_sweep_events": n, "events_sweep": n_sweep, "points_sweep": p_sweep}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--proc", default="gg_ttgg")
    ap.add_argument("--n", type=int, default=1 << 23)
    ap.add_argument("--prec", default="mixed")
    ap.add_argument("--points", type=int, default=16)
    ap.add_argument("--cpu-sample", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-kpoly", action="store_true")
    ap.add_argument("--train-events", type=int, default=1 << 21)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--audit", type=float, default=0.01)
    ap.add_argument("--no-end-to-end", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark line: call time against events and against points")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device-to-device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the reweighting is embarrassingly parallel over events, so "
              "several GPUs take separate event batches, one process each; it measures one GPU's share.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2312_07440_amd as mg
    from synth import alpha_points, generate_events, kappa_points

    ng = {"gg_tt": 2, "gg_ttg": 3, "gg_ttgg": 4, "gg_ttggg": 5, "ee_5a": 0}[args.proc]
    log(f"generating {args.n} {args.proc} events")
    mom_np = generate_events(args.proc, args.n)
    dev = torch.device("cuda:0")
    if args.sweep:
        if args.proc == "ee_5a":
            sys.exit("--sweep covers the QCD processes")
        print(json.dumps(sweep(args, mom_np, kappa_points, mg, torch)), flush=True)
        return
    mom = torch.from_numpy(mom_np).to(dev)
    if args.proc == "ee_5a":
        kap = alpha_points(args.points)
        proc = mg.Process(args.proc, args.prec, {"alpha": ALPHA0})
        proc.set_params([{"alpha": float(a)} for a in kap])
    else:
        kap = kappa_points(args.points)
        proc = mg.Process(args.proc, args.prec)
        proc.set_params([{"kappa_ttg": float(k)} for k in kap])
    out = torch.empty((args.points, args.n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    proc.set_kernel_timing(True)
    for i in range(args.warmup):
        log(f"warmup {i}")
        proc.reweight(mom, out=out)
        torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    amp_ms = []
    for i in range(args.steps):
        starts[i].record(stream)
        proc.reweight(mom, out=out)
        ends[i].record(stream)
        # HIP events the library records on the same stream around its
        # amplitude kernel (read after the step's own events are queued)
        amp_ms.append(proc.kernel_time_ms())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms = float(np.mean(step_ms))
    kms = float(np.mean(amp_ms))
    log(f"step times (ms): {['%.1f' % x for x in step_ms]}, amplitude kernel (ms): "
        f"{['%.1f' % x for x in amp_ms]}, wall {wall:.2f}s")

    n_total_points = args.points + 1
    fpe, fcounts = flops_per_event(args.proc, n_total_points, proc.n_hel)
    # the amplitude kernel skips the events left to the FP64 re-evaluation
    # (outside the timed interval): count only the events it evaluates
    tau = proc.rescue_threshold if args.proc != "ee_5a" else 0.0
    n_rescued = rescued_events(mom_np, tau) if tau > 0 and ng >= 3 else 0
    n_eval = args.n - n_rescued
    achieved = fpe * n_eval / (kms * 1e-3) / 1e12
    peak = PEAK_FP32_TFLOPS if args.prec == "mixed" else PEAK_FP64_TFLOPS
    exec_ratio = MEASURED_EXEC_RATIO.get((args.proc, args.prec, kernel_fingerprint(args.proc)))
    value = args.n * args.points / (ms * 1e-3)
    tb = MEASURED_TRAFFIC.get((args.proc, args.prec, kernel_fingerprint(args.proc)))
    traffic = None if tb is None else tb * args.n

    res = {
        "metric": "reweighted events/s x16 param pts, gg->ttbar gg: exact vs surrogate at <=1% weight err",
        "value": value,
        "unit": "events*points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_min": float(np.min(step_ms)), "ms_max": float(np.max(step_ms)), "ms_median": float(np.median(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.proc} exact reweight, {args.n} events, {args.points} "
                               f"{'alpha' if args.proc == 'ee_5a' else 'kappa'} points + base, {args.prec} precision",
                   "events": args.n, "points": args.points, "process": args.proc,
                   "precision": args.prec, "path": "exact"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": ("amplitude kernels (split program parts)" if args.proc == "gg_ttggg"
                                else "amplitude kernel (one event per wave)"),
                     "kernel_ms": kms,
                     "flops_per_event": fpe, "per_helicity_flops": fcounts["per_helicity_flops"],
                     "events_evaluated": n_eval, "events_rescued_fp64": n_rescued, "rescue_tau": tau,
                     "counts": "algorithmic flops of the generated program (currents rebuilt per closing "
                               "group included) x the events the timed kernel evaluates",
                     "frac_executed": None if exec_ratio is None else exec_ratio * achieved / peak},
    }
    if not args.no_end_to_end:
        log("end-to-end (host buffers)")
        res["end_to_end"] = end_to_end_leg(args, proc, mom_np, mom, out, stream, torch)
    if not args.no_kpoly and args.proc in ("gg_tt", "gg_ttg", "gg_ttgg", "ee_5a"):
        log("kappa-polynomial variant")
        res["kpoly"] = kpoly_leg(args, proc, mom, out, stream, torch, n_eval)
    if not args.no_surrogate and args.proc != "ee_5a":
        res["surrogate"] = surrogate_leg(args, proc, mom, out, kap, torch, generate_events, ms,
                                         res.get("kpoly", {}).get("ms_per_step"))
    if not args.no_cpu_baseline:
        sample = min(args.cpu_sample, args.n)
        log(f"cpu baseline: oracle on {sample} events")
        cb, emax, emed = cpu_baseline(args.proc, ng, mom_np, kap, out[:, :sample].cpu().numpy(), sample,
                                      args.points)
        res["cpu_baseline"] = cb
        res["parity_sample"] = {"events": sample, "max_rel_err": emax, "median_rel_err": emed}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
