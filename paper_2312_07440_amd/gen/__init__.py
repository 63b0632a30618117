"""Build-time process generator: emits the per-process amplitude programs
(``csrc/gen/*.inc``) that the HIP kernels and the host validation build include."""
import os

from .process import emit_process, n_diagrams, flows, colour_matrix_loops  # noqa: F401

QCD_PROCESSES = {"gg_tt": 2, "gg_ttg": 3, "gg_ttgg": 4, "gg_ttggg": 5}
# processes whose per-helicity program is split into kernels
CHUNKS = {"gg_ttggg": 4}
# their double-precision instance: (chunks of closing groups, ranges of colour flows)
FP64_SPLIT = {"gg_ttggg": (4, 4)}
# processes evaluated one event per wave, whose programs read the momentum
# combinations of their vertices from the event record (the one-event-per-lane
# kernel keeps the record in per-lane LDS, where a larger record costs occupancy)
VERTEX_KIN = {"gg_ttgg", "gg_ttggg"}


def translation_units(names=None):
    """Generated HIP translation units of the processes (paths relative to gen/)."""
    out = []
    for name in (names or QCD_PROCESSES):
        out.append(f"qcd_{name}.hip")
        out += [f"qcd_{name}_part{c}.hip" for c in range(CHUNKS.get(name, 0))]
        if name in FP64_SPLIT:
            nch, nfr = FP64_SPLIT[name]
            out += [f"qcd_{name}_fr{c}_{r}.hip" for c in range(nch) for r in range(nfr)]
    return out


def generate(outdir=None, procs=None, force=False):
    """Write csrc/gen/<proc>.inc for each process; returns {proc: emitter}."""
    here = os.path.dirname(os.path.abspath(__file__))
    outdir = outdir or os.path.join(os.path.dirname(here), "csrc", "gen")
    os.makedirs(outdir, exist_ok=True)
    res = {}
    def put(path, src):
        old = open(path).read() if os.path.exists(path) else None
        if force or old != src:
            with open(path, "w") as f:
                f.write(src)

    sig = ("(int fp64, const double* mom, const double* w_in, int64_t n,\n"
           "    const qcd_launch& a, double* out, double* me0, hipStream_t s)")
    for name, ng in (procs or QCD_PROCESSES).items():
        nch = CHUNKS.get(name, 1)
        src, em = emit_process(name, ng, chunks=nch, fp64_split=FP64_SPLIT.get(name),
                               vertex_kin=name in VERTEX_KIN)
        put(os.path.join(outdir, f"{name}.inc"), src)
        head = f"// Generated: kernel instantiations for {name}.\n" \
               f'#include "../mgrw_kernels.h"\n#include "{name}.inc"\nnamespace mgrw {{\n'
        if nch == 1:
            body = (f"hipError_t launch_{name}{sig} {{\n"
                    f"    return launch_qcd<{name}>(fp64, mom, w_in, n, a, out, me0, s);\n}}\n")
        else:
            psig = (f"(const event_data<{name}, float>* ev, int64_t e0, int64_t nb, float* jbuf,\n"
                    "    const double* w_in, int64_t n, const qcd_launch& a, double* out, double* me0, hipStream_t s)")
            fsig = (f"(const event_data<{name}, double>* ev, const unsigned long long* count, int64_t e0,\n"
                    "    int64_t nb, double* jbuf, const qcd_launch& a, hipStream_t s)")
            for c in range(nch):
                put(os.path.join(outdir, f"qcd_{name}_part{c}.hip"),
                    head + f"hipError_t launch_{name}_part{c}{psig} {{\n"
                    f"    return launch_part<{name}, float, {c}>(ev, e0, nb, jbuf, w_in, n, a, out, me0, s);\n}}\n"
                    "}  // namespace mgrw\n")
            nch64, nfr = FP64_SPLIT[name]
            frs = [(c, r) for c in range(nch64) for r in range(nfr)]
            for c, r in frs:
                put(os.path.join(outdir, f"qcd_{name}_fr{c}_{r}.hip"),
                    head + f"hipError_t launch_{name}_fr{c}_{r}{fsig} {{\n"
                    f"    return launch_fr<{name}, {c}, {r}>(ev, count, e0, nb, jbuf, a, s);\n}}\n"
                    "}  // namespace mgrw\n")
            decls = "".join(f"hipError_t launch_{name}_part{c}{psig};\n" for c in range(nch))
            decls += "".join(f"hipError_t launch_{name}_fr{c}_{r}{fsig};\n" for c, r in frs)
            parts = ", ".join(f"launch_{name}_part{c}" for c in range(nch))
            fr = ", ".join(f"launch_{name}_fr{c}_{r}" for c, r in frs)
            body = (decls +
                    f"// Single-precision parts, double-precision (chunk, flow range) parts.\n"
                    f"static const split_launchers<{name}> kLaunch{name} = {{{{{parts}}}, {{{fr}}}}};\n"
                    f"hipError_t launch_{name}{sig} {{\n"
                    f"    return launch_split<{name}>(kLaunch{name}, fp64, mom, w_in, n, a, out, me0, s);\n}}\n")
        put(os.path.join(outdir, f"qcd_{name}.hip"), head + body + "}  // namespace mgrw\n")
        res[name] = em
    return res
