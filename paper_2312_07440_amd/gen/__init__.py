"""Build-time process generator: emits the per-process amplitude programs
(``csrc/gen/*.inc``) that the HIP kernels and the host validation build include."""
import os

from .process import emit_process, n_diagrams, flows, colour_matrix_loops  # noqa: F401

QCD_PROCESSES = {"gg_tt": 2, "gg_ttg": 3, "gg_ttgg": 4}


def generate(outdir=None, procs=None, force=False):
    """Write csrc/gen/<proc>.inc for each process; returns {proc: emitter}."""
    here = os.path.dirname(os.path.abspath(__file__))
    outdir = outdir or os.path.join(os.path.dirname(here), "csrc", "gen")
    os.makedirs(outdir, exist_ok=True)
    res = {}
    for name, ng in (procs or QCD_PROCESSES).items():
        path = os.path.join(outdir, f"{name}.inc")
        src, em = emit_process(name, ng)
        old = open(path).read() if os.path.exists(path) else None
        if force or old != src:
            with open(path, "w") as f:
                f.write(src)
        tu = os.path.join(outdir, f"qcd_{name}.hip")
        tu_src = (f"// Generated: kernel instantiations for {name}.\n"
                  f'#include "../mgrw_kernels.h"\n#include "{name}.inc"\n'
                  "namespace mgrw {\n"
                  f"hipError_t launch_{name}(int fp64, const double* mom, const double* w_in, int64_t n,\n"
                  "                         const qcd_launch& a, double* out, double* me0, hipStream_t s) {\n"
                  f"    return launch_qcd<{name}>(fp64, mom, w_in, n, a, out, me0, s);\n"
                  "}\n}  // namespace mgrw\n")
        old = open(tu).read() if os.path.exists(tu) else None
        if force or old != tu_src:
            with open(tu, "w") as f:
                f.write(tu_src)
        res[name] = em
    return res
