"""The reweighting procedure end to end (Sec. 3.2 steps 1-8): events parsed
from a Les Houches file, reweighted on the GPU, new weights written back;
the written weights are compared with the FP64 oracle on the events'
centre-of-mass momenta."""
import re
import sys

import numpy as np
import pytest

import oracle
from lhe_fixture import write_lhe
from synth import generate_events, kappa_points

pytestmark = pytest.mark.gpu


def test_lhe_to_lhe_reweighting(tmp_path):
    import torch
    import paper_2312_07440_amd as mg
    assert torch.cuda.is_available()
    n = 300
    mom_cm = generate_events("gg_ttg", n, first_event=4242)
    w = np.random.default_rng(4).uniform(0.5, 2.0, n)
    src, dst = tmp_path / "in.lhe", tmp_path / "out.lhe"
    write_lhe(src, "gg_ttg", mom_cm, w)
    print("case LHE -> GPU reweight -> LHE, gg_ttg n=300", flush=True)
    sys.stdout.flush()
    f = mg.LHEFile(src)                                   # step 2
    mom, w_in = f.events("gg_ttg")
    kap = kappa_points(4)
    p = mg.Process("gg_ttg", "mixed")                     # step 1
    p.set_params([{"kappa_ttg": float(k)} for k in kap])  # steps 4-7 run on the device
    out = p.reweight(torch.from_numpy(mom).cuda(), w_in=torch.from_numpy(w_in).cuda())
    torch.cuda.synchronize()
    ids = [f"kappa_{k:.4f}" for k in kap]
    f.write(dst, out.cpu().numpy(), ids)                  # step 8
    text = dst.read_text()
    got = np.array([float(v) for v in re.findall(r"<wgt id='kappa_[0-9.]+'> (\S+) </wgt>", text)])
    got = got.reshape(n, len(kap)).T
    me = oracle.qcd_me(3, np.ascontiguousarray(mom), [(0.118, 173.0, 1.0)] + [(0.118, 173.0, float(k)) for k in kap])
    ref = oracle.reweight(me, w)
    err = np.abs(got / ref - 1).max()
    print(f"  max rel err of the written weights {err:.3e}", flush=True)
    assert err <= 1e-5
