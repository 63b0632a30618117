// Kernels of e+ e- -> 5 photons: one event per 64-lane wave, the 64
// non-vanishing helicity configurations on the lanes.  The event's
// helicity-independent data (propagator vectors q_S / q_S^2 of the 30 proper
// photon subsets, polarisation bases, e+ e- spinors) are built once per event
// in double precision by a setup kernel and read by the waves through the
// scalar cache.
#include <hip/hip_runtime.h>

#include "mgrw_kernels.h"
#include "mgrw_qed.h"

namespace mgrw {

namespace {

// Events e0 .. e0 + nb - 1 of the n in mom; record el holds event e0 + el.
template <typename T>
__global__ void __launch_bounds__(kBlock)
ee5a_setup_kernel(const double* __restrict__ mom, int64_t n, int64_t e0, int64_t nb,
                  ee_5a::event<T>* __restrict__ ev) {
    const int64_t el = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (el >= nb) return;
    double p[ee_5a::NEXT][4];
    load_event<ee_5a::NEXT>(mom, n, e0 + el, p);
    ee_5a::setup(p, ev[el]);
}

// Events 0 .. nb - 1 of a chunk: records ev, and w_in, out, me0_out, passed
// from the chunk's first event on (out and me0_out keep the stride n).
template <typename T>
__global__ void __launch_bounds__(kBlock)
ee5a_wave_kernel(const ee_5a::event<T>* __restrict__ ev, const double* __restrict__ w_in, int64_t nb, int64_t n,
                 qed_launch a, double* __restrict__ out, double* __restrict__ me0_out) {
    static_assert(ee_5a::NLIVE == 64, "one live helicity configuration per lane");
    const int64_t e = int64_t(blockIdx.x) * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (e >= nb) return;   // whole wave; no barriers below
    const int lane = threadIdx.x & 63;
    const ee_5a::event<T>& d = ev[e];
    const double w = (a.mode == 0 && w_in) ? w_in[e] : 1.0;
    const double scale = d.flux * ee_5a::NORM;
    double me0 = 0.0;
    double me1 = 0.0;   // |M|^2 at e = 1 (coupling-polynomial mode)
    if (a.kpoly) {
        const cx<T> amp = ee_5a::amplitude<T>(d, lane, T(1));
        me1 = wave_sum(double(amp.re) * double(amp.re) + double(amp.im) * double(amp.im)) * scale;
    }
#pragma unroll 1
    for (int kp = 0; kp < a.npts; ++kp) {
        double me;
        if (a.kpoly) {
            const double e2 = a.e[kp] * a.e[kp];
            me = me1 * (e2 * e2 * e2 * e2 * e2);
        } else {
            __asm__ volatile("" ::: "memory");
            const cx<T> amp = ee_5a::amplitude<T>(d, lane, T(a.e[kp]));
            me = wave_sum(double(amp.re) * double(amp.re) + double(amp.im) * double(amp.im)) * scale;
        }
        if (kp == 0) {
            me0 = me;
            if (lane == 0) {
                if (a.mode == 1)
                    out[e] = me;
                else if (me0_out)
                    me0_out[e] = me;
            }
        } else if (lane == 0) {
            out[int64_t(kp - 1) * n + e] = reweighted(w, me, me0);
        }
    }
}

// Per-event records: a stream-ordered allocation for all n events, or (with
// a scratch span) carved from it, the events then run in chunks that fit.
template <typename T>
hipError_t launch(const double* mom, const double* w_in, int64_t n, const qed_launch& a, double* out, double* me0,
                  hipStream_t s) {
    ee_5a::event<T>* ev = nullptr;
    int64_t chunk = n;
    if (a.scratch.ptr) {
        chunk = scratch_chunk(a.scratch, sizeof(ee_5a::event<T>), 0);
        if (chunk < 1) return hipErrorInvalidValue;
        ev = static_cast<ee_5a::event<T>*>(a.scratch.ptr);
    } else {
        hipError_t err = hipMallocAsync(reinterpret_cast<void**>(&ev), sizeof(ee_5a::event<T>) * size_t(n), s);
        if (err != hipSuccess) return err;
    }
    hipError_t err = hipSuccess;
    for (int64_t e0 = 0; e0 < n && err == hipSuccess; e0 += chunk) {
        const int64_t nb = n - e0 < chunk ? n - e0 : chunk;
        hipLaunchKernelGGL((ee5a_setup_kernel<T>), dim3(unsigned((nb + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           mom, n, e0, nb, ev);
        mark(a.t0, s);
        // the chunk's inputs and outputs are passed from its first event on
        hipLaunchKernelGGL((ee5a_wave_kernel<T>), dim3(unsigned((nb + kBlock / 64 - 1) / (kBlock / 64))),
                           dim3(kBlock), 0, s, ev, w_in ? w_in + e0 : w_in, nb, n, a, out + e0,
                           me0 ? me0 + e0 : me0);
        mark(a.t1, s);
        err = hipGetLastError();
    }
    if (a.scratch.ptr) return err;
    hipError_t ferr = hipFreeAsync(ev, s);
    return err != hipSuccess ? err : ferr;
}

}  // namespace

hipError_t launch_ee5a(int fp64, const double* mom, const double* w_in, int64_t n, const qed_launch& a,
                       double* out, double* me0, hipStream_t s) {
    return fp64 ? launch<double>(mom, w_in, n, a, out, me0, s) : launch<float>(mom, w_in, n, a, out, me0, s);
}

}  // namespace mgrw
