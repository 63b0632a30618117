"""Build libmgrw.so (HIP, gfx950) and the host validation library.

Steps: run the process generator (csrc/gen/), compile every HIP translation
unit in parallel with hipcc for gfx950, link libmgrw.so into the package
directory, build libmgrw_hostcheck.so with g++ (tests only), and record the
exact per-helicity operation counts of each generated program in
csrc/gen/flops.json.
"""
import ctypes
import json
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "gen")
ROOT = os.path.dirname(HERE)
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmgrw.so")
HOSTLIB = os.path.join(HERE, "libmgrw_hostcheck.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are disabled on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(verbose=False, jobs=None):
    from .gen import generate, translation_units
    generate()
    os.makedirs(OBJ, exist_ok=True)
    units = [os.path.join(CSRC, "mgrw_abi.hip"), os.path.join(CSRC, "mgrw_mlp.hip"),
             os.path.join(CSRC, "mgrw_qed.hip"), os.path.join(CSRC, "mgrw_multi.hip"),
             os.path.join(CSRC, "mgrw_stream.hip")] + \
        [os.path.join(GEN, u) for u in translation_units()]
    # the split program parts take longest: start them first
    units.sort(key=lambda u: ("_part" not in u, u))
    objs = [os.path.join(OBJ, os.path.basename(u).replace(".hip", ".o")) for u in units]
    jobs = jobs or min(len(units) + 1, os.cpu_count() or 4)
    host_tmp = HOSTLIB + ".tmp"
    with ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_run, [HIPCC, *HIP_FLAGS, "-c", u, "-o", o], verbose) for u, o in zip(units, objs)]
        # host-only parts of the library (LHE files)
        lhe_obj = os.path.join(OBJ, "mgrw_lhe.o")
        futs.append(ex.submit(_run, ["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"),
                                     "-c", os.path.join(CSRC, "mgrw_lhe.cpp"), "-o", lhe_obj], verbose))
        objs = objs + [lhe_obj]
        # host validation build (tests only), compiled alongside
        futs.append(ex.submit(_run, ["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, "-o", host_tmp,
                                     os.path.join(CSRC, "host_check.cpp")], verbose))
        for f in futs:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    os.replace(host_tmp, HOSTLIB)
    write_flops()


def write_flops():
    lib = ctypes.CDLL(HOSTLIB)
    from .gen import QCD_PROCESSES
    out = {}
    for name, ng in QCD_PROCESSES.items():
        c = (ctypes.c_longlong * 6)()
        if lib.mgrw_host_qcd_flops(ng, c) != 0:
            raise RuntimeError("flop count failed")
        out[name] = {"per_helicity_add": c[0], "per_helicity_mul": c[1],
                     "per_helicity_flops": c[0] + c[1],
                     "colour_sum_flops": c[2] + c[3], "external_flops": c[4] + c[5]}
        lib.mgrw_host_kpoly_flops.restype = ctypes.c_longlong
        kf = lib.mgrw_host_kpoly_flops(ng)
        if kf > 0:
            out[name]["kpoly_per_helicity_flops"] = kf
    lib.mgrw_host_ee5a_flops.restype = ctypes.c_longlong
    out["ee_5a"] = {"per_helicity_flops": lib.mgrw_host_ee5a_flops(), "evaluated_helicities": 64}
    with open(os.path.join(GEN, "flops.json"), "w") as f:
        json.dump(out, f, indent=1)
    return out


if __name__ == "__main__":
    build(verbose=True)
