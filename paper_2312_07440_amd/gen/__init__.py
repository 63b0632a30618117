"""Build-time process generator: emits the per-process amplitude programs
(``csrc/gen/*.inc``) that the HIP kernels and the host validation build include."""
import os

from .process import emit_process, n_diagrams, flows, colour_matrix_loops  # noqa: F401

QCD_PROCESSES = {"gg_tt": 2, "gg_ttg": 3, "gg_ttgg": 4, "gg_ttggg": 5}
# processes whose per-helicity program is split into kernels (float only)
CHUNKS = {"gg_ttggg": 4}


def translation_units(names=None):
    """Generated HIP translation units of the processes (paths relative to gen/)."""
    out = []
    for name in (names or QCD_PROCESSES):
        out.append(f"qcd_{name}.hip")
        out += [f"qcd_{name}_part{c}.hip" for c in range(CHUNKS.get(name, 0))]
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
        src, em = emit_process(name, ng, chunks=nch)
        put(os.path.join(outdir, f"{name}.inc"), src)
        head = f"// Generated: kernel instantiations for {name}.\n" \
               f'#include "../mgrw_kernels.h"\n#include "{name}.inc"\nnamespace mgrw {{\n'
        if nch == 1:
            body = (f"hipError_t launch_{name}{sig} {{\n"
                    f"    return launch_qcd<{name}>(fp64, mom, w_in, n, a, out, me0, s);\n}}\n")
        else:
            psig = (f"(const event_data<{name}, float>* ev, int64_t e0, int64_t nb, float* jbuf,\n"
                    "    const double* w_in, int64_t n, const qcd_launch& a, double* out, double* me0, hipStream_t s)")
            for c in range(nch):
                put(os.path.join(outdir, f"qcd_{name}_part{c}.hip"),
                    head + f"hipError_t launch_{name}_part{c}{psig} {{\n"
                    f"    return launch_part<{name}, float, {c}>(ev, e0, nb, jbuf, w_in, n, a, out, me0, s);\n}}\n"
                    "}  // namespace mgrw\n")
            decls = "".join(f"hipError_t launch_{name}_part{c}{psig};\n" for c in range(nch))
            calls = "\n".join(
                f"        if (err == hipSuccess) err = launch_{name}_part{c}(ev, e0, nb, jbuf, w_in, n, a, out, me0, s);"
                for c in range(nch))
            calls += (f"\n        if (err == hipSuccess) err = launch_colour_mfma<{name}>(jbuf, e0, nb, w_in, n, a, out, "
                      "me0, s);")
            body = (decls +
                    f"// Single precision only: kinematics for all events, then batches of\n"
                    f"// kPartBatch events through the {nch} program parts and the colour sum.\n"
                    f"hipError_t launch_{name}{sig} {{\n"
                    "    if (fp64) return hipErrorInvalidValue;\n"
                    f"    using ED = event_data<{name}, float>;\n"
                    "    const int64_t B = n < kPartBatch ? n : kPartBatch;\n"
                    "    ED* ev = nullptr;\n"
                    "    float* jbuf = nullptr;\n"
                    "    hipError_t err = hipMallocAsync(reinterpret_cast<void**>(&ev), sizeof(ED) * size_t(n), s);\n"
                    "    if (err != hipSuccess) return err;\n"
                    f"    err = hipMallocAsync(reinterpret_cast<void**>(&jbuf), sizeof(float) * size_t(B) * a.npts * 2 * {name}::K * {name}::NHEL, s);\n"
                    "    if (err != hipSuccess) { (void)hipFreeAsync(ev, s); return err; }\n"
                    f"    hipLaunchKernelGGL((qcd_setup_kernel<{name}, float>), dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, mom, n, a.mt, ev, 0.0, nullptr, nullptr);\n"
                    "    err = hipGetLastError();\n"
                    "    mark(a.t0, s);\n"
                    "    for (int64_t e0 = 0; e0 < n && err == hipSuccess; e0 += B) {\n"
                    "        const int64_t nb = n - e0 < B ? n - e0 : B;\n"
                    f"{calls}\n"
                    "    }\n"
                    "    mark(a.t1, s);\n"
                    "    hipError_t f1 = hipFreeAsync(jbuf, s), f2 = hipFreeAsync(ev, s);\n"
                    "    return err != hipSuccess ? err : (f1 != hipSuccess ? f1 : f2);\n}\n")
        put(os.path.join(outdir, f"qcd_{name}.hip"), head + body + "}  // namespace mgrw\n")
        res[name] = em
    return res
