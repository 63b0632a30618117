// libmgrw: the C ABI declared in include/mgrw.h (argument checks, parameter
// points, dispatch to the per-process launchers) and the e+ e- -> mu+ mu-
// kernel.
//
// Every launch reads each event's momenta once (structure of arrays: lanes
// read consecutive doubles of each component), builds the helicity-
// independent kinematics in double, then evaluates the amplitude program at
// the base point and at every new parameter point and writes the reweighted
// weights (Sec. 3.2, steps 3-8; eq. (3)).  QCD processes whose number of
// helicity configurations is a multiple of 64 run one event per 64-lane wave
// with the configurations on the lanes (mgrw_kernels.h); the others one event
// per lane with a wave-uniform helicity loop, so lanes never diverge inside
// the diagram chains.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/mgrw.h"
#include "mgrw_internal.h"
#include "mgrw_kernels.h"
#include "gen/gg_tt.inc"
#include "gen/gg_ttg.inc"
#include "gen/gg_ttgg.inc"
#include "gen/gg_ttggg.inc"

using namespace mgrw;

// Per-process launchers, one translation unit each (mgrw_qcd_<proc>.hip).
#define MGRW_DECLARE_LAUNCHER(name)                                                                     \
    namespace mgrw {                                                                                    \
    hipError_t launch_##name(int fp64, const double* mom, const double* w_in, int64_t n, const qcd_launch& a, \
                             double* out, double* me0, hipStream_t s);                                  \
    }
MGRW_DECLARE_LAUNCHER(gg_tt)
MGRW_DECLARE_LAUNCHER(gg_ttg)
MGRW_DECLARE_LAUNCHER(gg_ttgg)
MGRW_DECLARE_LAUNCHER(gg_ttggg)
namespace mgrw {
hipError_t launch_ee5a(int fp64, const double* mom, const double* w_in, int64_t n, const qed_launch& a, double* out,
                       double* me0, hipStream_t s);
}

namespace {

__global__ void __launch_bounds__(kBlock)
ee_mumu_kernel(const double* __restrict__ mom, const double* __restrict__ w_in, int64_t n, ew_launch a,
               double* __restrict__ out, double* __restrict__ me0_out) {
    const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (e >= n) return;
    double p[4][4];
    load_event<4>(mom, n, e, p);
    ee_mumu_event ev;
    ev.setup(p);
    const double me0 = ev.me(a.pts[0]);
    if (a.mode == 1) {
        out[e] = me0;
        return;
    }
    if (me0_out) me0_out[e] = me0;
    const double w = w_in ? w_in[e] : 1.0;
    for (int k = 1; k < a.npts; ++k) out[int64_t(k - 1) * n + e] = reweighted(w, ev.me(a.pts[k]), me0);
}


// ------------------------------------------------------------------ host side

thread_local std::string g_last_error;

mgrw_status fail(mgrw_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

bool finite(double x) { return std::isfinite(x); }

}  // namespace


namespace {

struct proc_info {
    int n_ext, n_flows, n_hel, n_diagrams;
};

proc_info info_of(int proc) {
    switch (proc) {
        case MGRW_EE_MUMU: return {4, 1, 4, 2};
        case MGRW_EE_5A: return {7, 1, 128, 120};
        case MGRW_GG_TT: return {mgrw::gg_tt::NEXT, mgrw::gg_tt::K, mgrw::gg_tt::NHEL, mgrw::gg_tt::NDIAG};
        case MGRW_GG_TTG: return {mgrw::gg_ttg::NEXT, mgrw::gg_ttg::K, mgrw::gg_ttg::NHEL, mgrw::gg_ttg::NDIAG};
        case MGRW_GG_TTGG:
            return {mgrw::gg_ttgg::NEXT, mgrw::gg_ttgg::K, mgrw::gg_ttgg::NHEL, mgrw::gg_ttgg::NDIAG};
        case MGRW_GG_TTGGG:
            return {mgrw::gg_ttggg::NEXT, mgrw::gg_ttggg::K, mgrw::gg_ttggg::NHEL, mgrw::gg_ttggg::NDIAG};
        default: return {0, 0, 0, 0};
    }
}

mgrw_status check_params(int proc, const mgrw_params& q, const char* what) {
    const double v[8] = {q.alpha, q.sw2, q.mz, q.wz, q.alphas, q.mt, q.wt, q.kappa_ttg};
    for (double x : v)
        if (!finite(x)) return fail(MGRW_ERR_ARG, std::string(what) + ": non-finite parameter");
    if (proc == MGRW_EE_5A) {
        if (!(q.alpha > 0)) return fail(MGRW_ERR_ARG, std::string(what) + ": need alpha > 0");
    } else if (proc == MGRW_EE_MUMU) {
        if (!(q.alpha > 0) || !(q.sw2 > 0 && q.sw2 < 1) || !(q.mz > 0) || !(q.wz >= 0))
            return fail(MGRW_ERR_ARG, std::string(what) + ": need alpha > 0, 0 < sw2 < 1, mz > 0, wz >= 0");
    } else {
        if (!(q.alphas > 0) || !(q.mt > 0))
            return fail(MGRW_ERR_ARG, std::string(what) + ": need alphas > 0 and mt > 0");
        if (q.wt != 0.0) return fail(MGRW_ERR_ARG, std::string(what) + ": top width must be 0");
    }
    return MGRW_OK;
}

mgrw::qcd_point qcd_point_of(const mgrw_params& q) {
    const double gs = std::sqrt(4.0 * M_PI * q.alphas);
    return {gs, gs * gs, gs * q.kappa_ttg};
}

mgrw::ew_point ew_point_of(const mgrw_params& q) {
    const double e2 = 4.0 * M_PI * q.alpha;
    return {e2, e2 / (q.sw2 * (1.0 - q.sw2)), -0.5 + q.sw2, q.sw2, q.mz * q.mz, q.mz * q.wz};
}

mgrw_status launched(hipError_t err) {
    if (err != hipSuccess) return fail(MGRW_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(err));
    return MGRW_OK;
}

// Shared body of eval_me (mode 1, one point) and reweight (mode 0).  With a
// scratch span the launch allocates nothing (its buffers come from the span)
// and records no kernel timing.
mgrw_status run(mgrw_process* p, const double* mom, const double* w_in, int64_t n, const mgrw_params* pts,
                int npts, int mode, double* out, double* me0, void* stream, int kpoly = 0,
                scratch_span sc = {nullptr, 0}) {
    if (n < 0) return fail(MGRW_ERR_ARG, "n_events < 0");
    if (n == 0) return MGRW_OK;
    const hipEvent_t t0 = sc.ptr ? nullptr : p->t0, t1 = sc.ptr ? nullptr : p->t1;
    mgrw_status st;
    if ((st = check_device_ptr(mom, "mom", false)) != MGRW_OK) return st;
    if ((st = check_device_ptr(out, mode == 1 ? "me_out" : "w_out", false)) != MGRW_OK) return st;
    if ((st = check_device_ptr(w_in, "w_in", true)) != MGRW_OK) return st;
    if ((st = check_device_ptr(me0, "me_base_out", true)) != MGRW_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->proc == MGRW_EE_5A) {
        qed_launch a;
        std::memset(&a, 0, sizeof a);
        for (int k = 0; k < npts; ++k) a.e[k] = std::sqrt(4.0 * M_PI * pts[k].alpha);
        a.npts = npts;
        a.mode = mode;
        a.kpoly = kpoly;
        a.t0 = t0;
        a.t1 = t1;
        a.scratch = sc;
        p->timed = t0 != nullptr;
        if ((n + 3) / 4 > 0x7fffffffLL) return fail(MGRW_ERR_ARG, "n_events too large for one launch");
        return launched(launch_ee5a(p->prec == MGRW_FP64, mom, w_in, n, a, out, me0, s));
    }
    if (p->proc == MGRW_EE_MUMU) {
        ew_launch a;
        std::memset(&a, 0, sizeof a);
        for (int k = 0; k < npts; ++k) a.pts[k] = ew_point_of(pts[k]);
        a.npts = npts;
        a.mode = mode;
        const int64_t blocks = (n + kBlock - 1) / kBlock;
        if (blocks > 0x7fffffffLL) return fail(MGRW_ERR_ARG, "n_events too large for one launch");
        hipLaunchKernelGGL(ee_mumu_kernel, dim3(unsigned(blocks)), dim3(kBlock), 0, s, mom, w_in, n, a, out, me0);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess)
            return fail(MGRW_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(err));
        return MGRW_OK;
    }
    // the widest grid: one event per wave, four waves per workgroup
    if ((n + 3) / 4 > 0x7fffffffLL) return fail(MGRW_ERR_ARG, "n_events too large for one launch");
    qcd_launch a;
    std::memset(&a, 0, sizeof a);
    for (int k = 0; k < npts; ++k) a.pts[k] = qcd_point_of(pts[k]);
    a.npts = npts;
    a.mode = mode;
    a.mt = p->base.mt;
    // automatic choice: one event per wave when the helicity configurations fill
    // whole waves (kinematics then live in the scalar cache, not in VGPRs/LDS)
    a.mapping = p->mapping != MGRW_MAP_AUTO ? p->mapping
                : (info_of(p->proc).n_hel % 64 == 0 ? MGRW_MAP_EVENT_PER_WAVE : MGRW_MAP_EVENT_PER_LANE);
    a.kpoly = kpoly;
    a.rescue_tau = p->rescue_tau;
    a.colour_mfma = p->colour_mfma;
    a.t0 = t0;
    a.t1 = t1;
    a.scratch = sc;
    p->timed = t0 != nullptr;
    const int fp64 = p->prec == MGRW_FP64;
    switch (p->proc) {
        case MGRW_GG_TT: return launched(launch_gg_tt(fp64, mom, w_in, n, a, out, me0, s));
        case MGRW_GG_TTG: return launched(launch_gg_ttg(fp64, mom, w_in, n, a, out, me0, s));
        case MGRW_GG_TTGG: return launched(launch_gg_ttgg(fp64, mom, w_in, n, a, out, me0, s));
        case MGRW_GG_TTGGG: return launched(launch_gg_ttggg(fp64, mom, w_in, n, a, out, me0, s));
        default: return fail(MGRW_ERR_UNSUPPORTED, "process not built");
    }
}

// ------------------------------------------- allocation-free reweighting
//
// mgrw_reweight_noalloc takes every intermediate buffer of a launch (per-event
// kinematics records, the list of events for the FP64 re-evaluation) from
// this file-scope device array instead of allocating; the events run in
// chunks whose buffers fit.  Each GPU holds its own copy at its own address,
// looked up once per device with that device current.  In host code the
// array's name is only a handle for that lookup, never a device address.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch span of the device the stream belongs to (the current device
// for the null stream), which must be the current device.
mgrw_status device_scratch(hipStream_t s, scratch_span* out) {
    int dev = -1;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return fail(MGRW_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(err));
    if (s) {
        hipDevice_t sd = -1;
        err = hipStreamGetDevice(s, &sd);
        if (err != hipSuccess) return fail(MGRW_ERR_ARG, std::string("stream: ") + hipGetErrorString(err));
        if (sd != dev) return fail(MGRW_ERR_ARG, "stream belongs to another device than the current one");
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(MGRW_ERR_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !ptr)
            return fail(MGRW_ERR_DEVICE, std::string("scratch address: ") + hipGetErrorString(err));
        g_scratch_ptr[dev] = ptr;
    }
    *out = {g_scratch_ptr[dev], kScratchBytes};
    return MGRW_OK;
}

}  // namespace

extern "C" {

mgrw_status mgrw_reweight_noalloc(mgrw_process* p, const double* mom, const double* w_in, int64_t n_events,
                                  double* w_out, double* me_base_out, void* stream) {
    if (!p) return fail(MGRW_ERR_ARG, "process is NULL");
    if (p->n_points == 0) return fail(MGRW_ERR_STATE, "no parameter points set");
    if (p->proc == MGRW_GG_TTGGG)
        return fail(MGRW_ERR_UNSUPPORTED,
                    "allocation-free reweight: g g -> t tbar g g g needs colour-flow buffers of about 2 MB per "
                    "event, beyond the 256 MiB scratch; use mgrw_reweight");
    if (n_events <= 0) return run(p, mom, w_in, n_events, nullptr, 0, 0, w_out, me_base_out, stream);
    scratch_span sc;
    mgrw_status st = device_scratch(static_cast<hipStream_t>(stream), &sc);
    if (st != MGRW_OK) return st;
    mgrw_params all[kMaxLaunchPoints];
    all[0] = p->base;
    for (int k = 0; k < p->n_points; ++k) all[k + 1] = p->points[k];
    return run(p, mom, w_in, n_events, all, p->n_points + 1, 0, w_out, me_base_out, stream, 0, sc);
}

mgrw_status mgrw_create_process(int proc, int prec, const mgrw_params* base, mgrw_process** out) {
    if (!out) return fail(MGRW_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!base) return fail(MGRW_ERR_ARG, "base is NULL");
    if (proc < MGRW_EE_MUMU || proc > MGRW_EE_5A) return fail(MGRW_ERR_ARG, "unknown process");
    if (prec != MGRW_FP64 && prec != MGRW_MIXED) return fail(MGRW_ERR_ARG, "unknown precision");
    if (info_of(proc).n_ext == 0) return fail(MGRW_ERR_UNSUPPORTED, "process not built into this library");
    if (proc == MGRW_EE_MUMU && prec != MGRW_FP64)
        return fail(MGRW_ERR_UNSUPPORTED, "e+e- -> mu+mu- is built in FP64 only");
    mgrw_status st = check_params(proc, *base, "base");
    if (st != MGRW_OK) return st;
    mgrw_process* p = new (std::nothrow) mgrw_process;
    if (!p) return fail(MGRW_ERR_ALLOC, "out of host memory");
    p->proc = proc;
    p->prec = prec;
    p->base = *base;
    p->n_points = 0;
    p->mapping = MGRW_MAP_AUTO;
    // FP64 re-evaluation thresholds, from full-sample comparisons of mixed
    // precision with the FP64 kernels (every weight within 1e-5)
    p->rescue_tau = (prec == MGRW_MIXED && proc >= MGRW_GG_TT && proc <= MGRW_GG_TTGGG)
                        ? (proc == MGRW_GG_TTGGG ? 1e-3 : 3e-3) : 0.0;
    p->sur = nullptr;
    p->t0 = p->t1 = nullptr;
    p->timed = 0;
    p->colour_mfma = 0;
    p->hp = nullptr;
    p->sur_inputs = MGRW_SURROGATE_N_FEATURES;
    *out = p;
    return MGRW_OK;
}

mgrw_status mgrw_set_params(mgrw_process* p, const mgrw_params* points, int32_t n_points) {
    if (!p) return fail(MGRW_ERR_ARG, "process is NULL");
    if (!points) return fail(MGRW_ERR_ARG, "points is NULL");
    if (n_points < 1 || n_points > MGRW_MAX_POINTS) return fail(MGRW_ERR_ARG, "n_points out of [1, 64]");
    for (int k = 0; k < n_points; ++k) {
        mgrw_status st = check_params(p->proc, points[k], "point");
        if (st != MGRW_OK) return st;
        if (p->proc != MGRW_EE_MUMU && p->proc != MGRW_EE_5A && points[k].mt != p->base.mt)
            return fail(MGRW_ERR_ARG, "external masses must equal the base point's");
    }
    std::memcpy(p->points, points, sizeof(mgrw_params) * size_t(n_points));
    p->n_points = n_points;
    return MGRW_OK;
}

mgrw_status mgrw_eval_me(mgrw_process* p, const double* mom, int64_t n_events, int32_t point, double* me_out,
                         void* stream) {
    if (!p) return fail(MGRW_ERR_ARG, "process is NULL");
    if (point < -1) return fail(MGRW_ERR_ARG, "point < -1");
    if (point >= 0 && p->n_points == 0) return fail(MGRW_ERR_STATE, "no parameter points set");
    if (point >= p->n_points) return fail(MGRW_ERR_ARG, "point out of range");
    const mgrw_params& q = point < 0 ? p->base : p->points[point];
    return run(p, mom, nullptr, n_events, &q, 1, 1, me_out, nullptr, stream);
}

mgrw_status mgrw_reweight(mgrw_process* p, const double* mom, const double* w_in, int64_t n_events,
                          double* w_out, double* me_base_out, void* stream) {
    if (!p) return fail(MGRW_ERR_ARG, "process is NULL");
    if (p->n_points == 0) return fail(MGRW_ERR_STATE, "no parameter points set");
    mgrw_params all[kMaxLaunchPoints];
    all[0] = p->base;
    for (int k = 0; k < p->n_points; ++k) all[k + 1] = p->points[k];
    return run(p, mom, w_in, n_events, all, p->n_points + 1, 0, w_out, me_base_out, stream);
}

mgrw_status mgrw_reweight_kpoly(mgrw_process* p, const double* mom, const double* w_in, int64_t n_events,
                                double* w_out, double* me_base_out, void* stream) {
    if (!p) return fail(MGRW_ERR_ARG, "process is NULL");
    if (p->proc == MGRW_EE_MUMU || p->proc == MGRW_GG_TTGGG)
        return fail(MGRW_ERR_UNSUPPORTED,
                    "kappa-polynomial reweighting: g g -> t tbar + 0..2 g and e+ e- -> 5 photons only");
    if (p->n_points == 0) return fail(MGRW_ERR_STATE, "no parameter points set");
    mgrw_params all[kMaxLaunchPoints];
    all[0] = p->base;
    for (int k = 0; k < p->n_points; ++k) all[k + 1] = p->points[k];
    return run(p, mom, w_in, n_events, all, p->n_points + 1, 0, w_out, me_base_out, stream, 1);
}

mgrw_status mgrw_process_info(const mgrw_process* p, int* n_ext, int* n_flows, int* n_hel, int* n_diagrams) {
    if (!p) return fail(MGRW_ERR_ARG, "process is NULL");
    proc_info i = info_of(p->proc);
    if (n_ext) *n_ext = i.n_ext;
    if (n_flows) *n_flows = i.n_flows;
    if (n_hel) *n_hel = i.n_hel;
    if (n_diagrams) *n_diagrams = i.n_diagrams;
    return MGRW_OK;
}

mgrw_status mgrw_set_option(mgrw_process* p, int option, int64_t value) {
    if (!p) return fail(MGRW_ERR_ARG, "process is NULL");
    if (option == MGRW_OPT_RESCUE_PPM) {
        if (value < 0 || value > 1000000) return fail(MGRW_ERR_ARG, "rescue threshold must be 0..1000000 ppm");
        if (value != 0 && (p->prec != MGRW_MIXED || p->proc < MGRW_GG_TT || p->proc > MGRW_GG_TTGGG))
            return fail(MGRW_ERR_UNSUPPORTED, "FP64 rescue: mixed precision g g -> t tbar + 0..3 g only");
        p->rescue_tau = double(value) * 1e-6;
        return MGRW_OK;
    }
    if (option == MGRW_OPT_COLOUR_MFMA) {
        if (value != 0 && value != 1) return fail(MGRW_ERR_ARG, "matrix-core colour sum: 0 or 1");
        if (value == 1 && p->proc != MGRW_GG_TTGGG)
            return fail(MGRW_ERR_UNSUPPORTED, "matrix-core colour sum: g g -> t tbar g g g only");
        p->colour_mfma = int(value);
        return MGRW_OK;
    }
    if (option == MGRW_OPT_SURROGATE_INPUTS) {
        if (value != MGRW_SURROGATE_N_FEATURES && value != 25)
            return fail(MGRW_ERR_ARG, "surrogate inputs: 53 (with the pair invariants) or 25");
        p->sur_inputs = int(value);
        return MGRW_OK;
    }
    if (option == MGRW_OPT_KERNEL_TIMING) {
        if (value != 0 && value != 1) return fail(MGRW_ERR_ARG, "kernel timing: 0 or 1");
        if (value == 1 && !p->t0) {
            if (hipEventCreate(&p->t0) != hipSuccess || hipEventCreate(&p->t1) != hipSuccess) {
                if (p->t0) (void)hipEventDestroy(p->t0);
                p->t0 = p->t1 = nullptr;
                return fail(MGRW_ERR_DEVICE, "hipEventCreate failed");
            }
        } else if (value == 0 && p->t0) {
            (void)hipEventDestroy(p->t0);
            (void)hipEventDestroy(p->t1);
            p->t0 = p->t1 = nullptr;
        }
        p->timed = 0;
        return MGRW_OK;
    }
    if (option != MGRW_OPT_LANE_MAPPING) return fail(MGRW_ERR_ARG, "unknown option");
    if (value != MGRW_MAP_AUTO && value != MGRW_MAP_EVENT_PER_LANE && value != MGRW_MAP_EVENT_PER_WAVE)
        return fail(MGRW_ERR_ARG, "unknown lane mapping");
    if (value == MGRW_MAP_EVENT_PER_WAVE && (p->proc == MGRW_EE_MUMU || info_of(p->proc).n_hel % 64 != 0))
        return fail(MGRW_ERR_UNSUPPORTED, "one event per wave needs a multiple of 64 helicity configurations");
    if (value == MGRW_MAP_EVENT_PER_LANE && (p->proc == MGRW_GG_TTGGG || p->proc == MGRW_EE_5A))
        return fail(MGRW_ERR_UNSUPPORTED, "g g -> t tbar g g g runs one event per wave only");
    p->mapping = int(value);
    return MGRW_OK;
}

mgrw_status mgrw_get_option(const mgrw_process* p, int option, int64_t* value) {
    if (!p || !value) return fail(MGRW_ERR_ARG, "process or value is NULL");
    switch (option) {
        case MGRW_OPT_LANE_MAPPING: *value = p->mapping; return MGRW_OK;
        case MGRW_OPT_RESCUE_PPM: *value = int64_t(p->rescue_tau * 1e6 + 0.5); return MGRW_OK;
        case MGRW_OPT_KERNEL_TIMING: *value = p->t0 != nullptr; return MGRW_OK;
        case MGRW_OPT_COLOUR_MFMA: *value = p->colour_mfma; return MGRW_OK;
        case MGRW_OPT_SURROGATE_INPUTS: *value = p->sur_inputs; return MGRW_OK;
        default: return fail(MGRW_ERR_ARG, "unknown option");
    }
}

mgrw_status mgrw_kernel_time_ms(mgrw_process* p, double* ms) {
    if (!p || !ms) return fail(MGRW_ERR_ARG, "process or ms is NULL");
    if (!p->t0 || !p->timed) return fail(MGRW_ERR_STATE, "kernel timing is off or nothing was launched");
    float f = 0.0f;
    hipError_t err = hipEventSynchronize(p->t1);
    if (err == hipSuccess) err = hipEventElapsedTime(&f, p->t0, p->t1);
    if (err != hipSuccess) return fail(MGRW_ERR_DEVICE, std::string("event timing: ") + hipGetErrorString(err));
    *ms = double(f);
    return MGRW_OK;
}

void mgrw_destroy_process(mgrw_process* p) {
    if (!p) return;
    if (p->t0) {
        (void)hipEventDestroy(p->t0);
        (void)hipEventDestroy(p->t1);
    }
    mgrw::surrogate_destroy(p->sur);
    mgrw::host_pipeline_destroy(p->hp);
    delete p;
}

const char* mgrw_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

mgrw_status mgrw::set_error(mgrw_status code, const std::string& msg) { return fail(code, msg); }

mgrw_status mgrw::check_device_ptr(const void* ptr, const char* what, bool allow_null) {
    if (!ptr) {
        if (allow_null) return MGRW_OK;
        return fail(MGRW_ERR_ARG, std::string(what) + " is NULL");
    }
    hipPointerAttribute_t attr;
    hipError_t err = hipPointerGetAttributes(&attr, ptr);
    if (err != hipSuccess) {
        (void)hipGetLastError();
        return fail(MGRW_ERR_ARG, std::string(what) + " is not a HIP allocation");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(MGRW_ERR_ARG, std::string(what) + " is not device memory");
    return MGRW_OK;
}
