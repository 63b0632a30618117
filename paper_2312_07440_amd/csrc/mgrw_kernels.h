// Kernel templates of libmgrw (one event per lane) and the per-process
// launcher, shared by the per-process translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <type_traits>

#include "../../include/mgrw.h"
#include "mgrw_event.h"

namespace mgrw {

constexpr int kBlock = 256;
constexpr int kMaxLaunchPoints = MGRW_MAX_POINTS + 1;   // base + new points

// Device memory a launch may use for its intermediate buffers instead of
// allocating them.  ptr == nullptr: the launch allocates (stream-ordered).
// Otherwise the buffers are carved from [ptr, ptr + bytes) (ptr 256-byte
// aligned) and the events are processed in chunks whose buffers fit.
struct scratch_span {
    void* ptr;
    size_t bytes;
};

// Events per chunk when each event needs per_event bytes of scratch and the
// chunk a fixed head of head bytes (0 if not even one event fits).
inline int64_t scratch_chunk(const scratch_span& sc, size_t per_event, size_t head) {
    if (sc.bytes <= head || per_event == 0) return 0;
    return int64_t((sc.bytes - head) / per_event);
}

// Round up to the 256-byte alignment of every carved buffer.
constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Parameters travel by value with each launch (kernel-argument segment), so a
// later mgrw_set_params never races with work already queued.
struct qcd_launch {
    mgrw::qcd_point pts[kMaxLaunchPoints];
    int npts;        // points in pts (base first)
    int mode;        // 0: reweight, 1: |M|^2 of pts[0] only
    double mt;
    int mapping;     // MGRW_MAP_EVENT_PER_LANE or MGRW_MAP_EVENT_PER_WAVE
    int kpoly;       // 1: kappa-polynomial evaluation (one program per helicity for all points)
    double rescue_tau;   // > 0: events with a gluon invariant |2 p_i.p_j|/s below it are redone in FP64
    hipEvent_t t0, t1;   // non-null: recorded around the amplitude kernel(s) of the launch
    int colour_mfma;     // split programs: colour sum on the matrix cores (after the last part)
    scratch_span scratch;   // non-null: caller-provided device scratch (no allocation; events in chunks)
};

struct ew_launch {
    mgrw::ew_point pts[kMaxLaunchPoints];
    int npts;
    int mode;
};

// e+ e- -> n photons: the coupling e = sqrt(4 pi alpha) of every point.
struct qed_launch {
    double e[kMaxLaunchPoints];
    int npts;
    int mode;
    int kpoly;       // 1: one evaluation at e = 1, |M|^2 = e^(2n) |M_1|^2 for every point
    hipEvent_t t0, t1;
    scratch_span scratch;
};

// Device-side timestamps around the amplitude kernel(s) of a launch.
inline void mark(hipEvent_t ev, hipStream_t s) {
    if (ev) (void)hipEventRecord(ev, s);
}

// Library-owned streams of the current device (default priority, created on
// first use, kept until the process ends), on which independent kernels of
// one call run beside the caller's stream.
constexpr int kAuxStreams = 3;
constexpr int kMaxDevices = 64;
inline hipError_t aux_streams(hipStream_t* out) {
    static std::mutex mu;
    static hipStream_t pool[kMaxDevices][kAuxStreams] = {};
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < kAuxStreams; ++i) {
        if (!pool[dev][i]) {
            err = hipStreamCreateWithFlags(&pool[dev][i], hipStreamNonBlocking);
            if (err != hipSuccess) {
                pool[dev][i] = nullptr;
                return err;
            }
        }
        out[i] = pool[dev][i];
    }
    return hipSuccess;
}

template <int NEXT>
__device__ __forceinline__ void load_event(const double* __restrict__ mom, int64_t n, int64_t e,
                                           double (&p)[NEXT][4]) {
#pragma unroll
    for (int i = 0; i < NEXT; ++i)
#pragma unroll
        for (int m = 0; m < 4; ++m) p[i][m] = __builtin_nontemporal_load(mom + (int64_t(i) * 4 + m) * n + e);
}

// w_out[k-1][e] = W * (me_k / me_0), NaN where me_0 = 0 (eq. (3)).
__device__ __forceinline__ double reweighted(double w, double me, double me0) {
    return me0 != 0.0 ? w * (me / me0) : __builtin_nan("");
}

// Per-lane LDS slot with an odd number of 32-bit words, so that lanes reading
// the same member hit distinct banks.
template <typename S>
struct lds_slot {
    S v;
    float pad[(sizeof(S) / 4) % 2 == 0 ? 1 : 2];
};

// The reweight loop of one event over the points (one call site, so the
// amplitude program is inlined once).
template <class Proc, typename T, typename KN, typename BS>
__device__ __forceinline__ void run_points(const KN& k, const BS& b, const qcd_launch& a, int64_t n, int64_t e,
                                           const double* __restrict__ w_in, double* __restrict__ out,
                                           double* __restrict__ me0_out) {
    const double w = (a.mode == 0 && w_in) ? w_in[e] : 1.0;
    double me0 = 0.0;
#pragma unroll 1
    for (int kp = 0; kp < a.npts; ++kp) {
        const double me = point_me<Proc, T>(k, b, a.pts[kp]);
        if (kp == 0) {
            me0 = me;
            if (a.mode == 1)
                out[e] = me;
            else if (me0_out)
                me0_out[e] = me;
        } else {
            out[int64_t(kp - 1) * n + e] = reweighted(w, me, me0);
        }
    }
}

// Lanes per workgroup of the one-event-per-lane kernel: in single precision
// each lane owns an LDS slot for its kinematics and bases, and the workgroup
// size is the one of 256, 128, 64 that keeps the most waves resident per CU
// within its 160 KiB of LDS (larger on ties).
constexpr int lane_waves_per_cu(size_t slot, int nb) {
    return slot * nb <= 160 * 1024 ? int((160 * 1024) / (slot * nb)) * (nb / 64) : 0;
}
template <class Proc, typename T>
constexpr int lane_block() {
    if constexpr (sizeof(T) == 4) {
        constexpr size_t slot = sizeof(lds_slot<typename Proc::template kin<T>>) +
                                sizeof(lds_slot<typename Proc::template basis<T>>);
        constexpr int w256 = lane_waves_per_cu(slot, 256), w128 = lane_waves_per_cu(slot, 128),
                      w64 = lane_waves_per_cu(slot, 64);
        return (w256 >= w128 && w256 >= w64) ? 256 : (w128 >= w64 ? 128 : 64);
    } else {
        return kBlock;
    }
}

// One event per lane.  In single precision the per-lane kinematics and
// wavefunction bases live in LDS (each lane owns a slot; no barriers); in
// double precision they stay in registers.
template <class Proc, typename T>
__global__ void __launch_bounds__((lane_block<Proc, T>()))
qcd_kernel(const double* __restrict__ mom, const double* __restrict__ w_in, int64_t n, qcd_launch a,
           double* __restrict__ out, double* __restrict__ me0_out) {
    constexpr int NB = lane_block<Proc, T>();
    const int64_t e = int64_t(blockIdx.x) * NB + threadIdx.x;
    if (e >= n) return;   // no barriers below: early exit is safe
    double p[Proc::NEXT][4];
    load_event<Proc::NEXT>(mom, n, e, p);
    using KinT = typename Proc::template kin<T>;
    using BasT = typename Proc::template basis<T>;
    if constexpr (sizeof(T) == 4) {
        __shared__ lds_slot<KinT> ks[NB];
        __shared__ lds_slot<BasT> bs[NB];
        KinT& k = ks[threadIdx.x].v;
        BasT& b = bs[threadIdx.x].v;
        Proc::kinematics(p, a.mt, k);
        Proc::external_basis(p, a.mt, b);
        run_points<Proc, T>(k, b, a, n, e, w_in, out, me0_out);
    } else {
        KinT k;
        BasT b;
        Proc::kinematics(p, a.mt, k);
        Proc::external_basis(p, a.mt, b);
        run_points<Proc, T>(k, b, a, n, e, w_in, out, me0_out);
    }
}

// ------------------------------------------------ one event per wave
//
// Lanes carry helicity configurations (h = lane + 64 c); the event's
// kinematics and wavefunction bases are wave-uniform, computed once per event
// by qcd_setup_kernel and read through the scalar cache, so they occupy
// neither vector registers nor LDS.  The helicity sum is a wave reduction.

#ifndef MGRW_WAVE_WPE
#define MGRW_WAVE_WPE 2
#endif

// Single-precision amplitudes lose digits where diagrams cancel strongly
// against each other: a final-state gluon nearly collinear to a beam gluon or
// to another final-state gluon (small |2 p_i.p_j| / s).  Such events are
// evaluated again in FP64 after the single-precision pass.
template <class Proc>
__device__ __forceinline__ bool ill_conditioned(const double (&p)[Proc::NEXT][4], double tau) {
    const double E = p[0][0] + p[1][0], X = p[0][1] + p[1][1], Y = p[0][2] + p[1][2], Z = p[0][3] + p[1][3];
    const double s = E * E - X * X - Y * Y - Z * Z;
    bool ill = false;
    // gluons: the beams (particles 0 and 1) and the final state (4 ...)
#pragma unroll
    for (int i = 0; i < Proc::NEXT; ++i) {
#pragma unroll
        for (int j = i + 1; j < Proc::NEXT; ++j) {
            const bool gi = i < 2 || i >= 4, gj = j < 2 || j >= 4;
            if (!gi || !gj || (i == 0 && j == 1)) continue;
            const double d = p[i][0] * p[j][0] - p[i][1] * p[j][1] - p[i][2] * p[j][2] - p[i][3] * p[j][3];
            ill = ill || (fabs(2.0 * d) < tau * s);
        }
    }
    return ill;
}

template <class Proc, typename T>
struct event_data {
    typename Proc::template kin<T> k;
    typename Proc::template basis<T> b;
    int skip;   // 1: left to the FP64 re-evaluation
};

// Kinematics and wavefunction bases of every event; with tau > 0 also lists
// the ill-conditioned events (count, list) and marks them to be skipped.
// Events e0 .. e0 + nb - 1 of the n in mom; record el holds event e0 + el and
// the list holds event numbers.
template <class Proc, typename T>
__global__ void __launch_bounds__(kBlock)
qcd_setup_kernel(const double* __restrict__ mom, int64_t n, int64_t e0, int64_t nb, double mt,
                 event_data<Proc, T>* __restrict__ ev, double tau, unsigned long long* __restrict__ count,
                 int64_t* __restrict__ list) {
    const int64_t el = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (el >= nb) return;
    const int64_t e = e0 + el;
    double p[Proc::NEXT][4];
    load_event<Proc::NEXT>(mom, n, e, p);
    Proc::kinematics(p, mt, ev[el].k);
    Proc::external_basis(p, mt, ev[el].b);
    int skip = 0;
    if (tau > 0.0 && ill_conditioned<Proc>(p, tau)) {
        skip = 1;
        list[atomicAdd(count, 1ull)] = e;
    }
    ev[el].skip = skip;
}

// An event's kinematics record, staged in LDS, as the generated programs
// should read it: each value loaded where the program uses it.  The record is
// wave-uniform; read through its plain address the compiler loads all of it
// ahead of the program and spills (from global memory: into scalar registers,
// then to vector lanes; from LDS: into vector registers, then to scratch).
// An opaque copy of the address keeps each read next to its use, and the
// assumption keeps the reads LDS reads (ds_read) rather than flat loads.  The
// address must be wave-uniform (it is held in scalar registers).
template <class K>
__device__ __forceinline__ const K& lds_near_use(const K& k) {
    const K* p = &k;
    __asm__ volatile("" : "+s"(p));
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_assume(__builtin_amdgcn_is_shared(reinterpret_cast<const void*>(p)));
#endif
    return *p;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Events e0 .. e0 + nb - 1 (record el = event e0 + el).
template <class Proc, typename T>
__global__ void __launch_bounds__(kBlock, MGRW_WAVE_WPE)
qcd_wave_kernel(const event_data<Proc, T>* __restrict__ ev, int64_t e0, int64_t nb, const double* __restrict__ w_in,
                int64_t n, qcd_launch a, double* __restrict__ out, double* __restrict__ me0_out) {
    static_assert(Proc::NHEL % 64 == 0, "helicity configurations must fill whole waves");
    const int64_t el = int64_t(blockIdx.x) * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (el >= nb || ev[el].skip) return;   // whole wave; no barriers below
    const int64_t e = e0 + el;
    const int lane = threadIdx.x & 63;
    // the event's kinematics record, staged once per event in LDS (one record
    // per wave): the program reads it with broadcast LDS loads
    using KIN = typename Proc::template kin<T>;
    struct alignas(16) kin_slot { KIN v; };
    static_assert(sizeof(KIN) % 4 == 0, "record copied in 32-bit words");
    __shared__ kin_slot kl[kBlock / 64];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&ev[el].k);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&kl[wv].v);
        for (int i = lane; i < int(sizeof(KIN) / 4); i += 64) dst[i] = src[i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    const KIN& k = kl[wv].v;
    const typename Proc::template basis<T>& b = ev[el].b;
    const double w = (a.mode == 0 && w_in) ? w_in[e] : 1.0;
    // the lane's external wavefunctions live in its own LDS slot: they are
    // read throughout the program, and in registers they push the program's
    // working set into scratch.  With one block of 64 configurations they do
    // not depend on the point and are assembled once per event.
    __shared__ lds_slot<typename Proc::template ext<T>> wfs[kBlock];
    typename Proc::template ext<T>& wf = wfs[threadIdx.x].v;
    constexpr bool one_block = Proc::NHEL == 64;
    if constexpr (one_block) Proc::template external<T>(b, lane, wf);
    double me0 = 0.0;
#pragma unroll 1
    for (int kp = 0; kp < a.npts; ++kp) {
        const qcd_point pt = a.pts[kp];
        const auto c = Proc::template couplings<T>(pt.gs, pt.gs2, pt.gk);
        double acc = 0.0;
#pragma unroll 1
        for (int hc = 0; hc < Proc::NHEL; hc += 64) {
            __asm__ volatile("" ::: "memory");
            if constexpr (!one_block) Proc::template external<T>(b, hc + lane, wf);
            cx<T> J[Proc::K];
            Proc::amplitude(wf, lds_near_use(k), c, J);
            acc += double(Proc::colour_sum(J));
        }
        const double me = wave_sum(acc) * Proc::point_norm(pt.gs);
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

// ------------------------------------------------ kappa-polynomial kernels

// Outputs of one event from its helicity-summed B.
template <class Proc>
__device__ __forceinline__ void kpoly_outputs(const double* B, const qcd_launch& a, int64_t n, int64_t e,
                                              double w, double* __restrict__ out, double* __restrict__ me0_out) {
    double me0 = 0.0;
    for (int kp = 0; kp < a.npts; ++kp) {
        const double me = kpoly_me<Proc>(B, a.pts[kp].gs, a.pts[kp].gk / a.pts[kp].gs);
        if (kp == 0) {
            me0 = me;
            if (a.mode == 1)
                out[e] = me;
            else if (me0_out)
                me0_out[e] = me;
        } else {
            out[int64_t(kp - 1) * n + e] = reweighted(w, me, me0);
        }
    }
}

// One event per lane (processes with fewer than 64 helicity configurations).
template <class Proc, typename T>
__global__ void __launch_bounds__(kBlock)
qcd_kpoly_lane_kernel(const double* __restrict__ mom, const double* __restrict__ w_in, int64_t n, qcd_launch a,
                      double* __restrict__ out, double* __restrict__ me0_out) {
    const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (e >= n) return;
    double p[Proc::NEXT][4];
    load_event<Proc::NEXT>(mom, n, e, p);
    typename Proc::template kin<T> k;
    typename Proc::template basis<T> b;
    Proc::kinematics(p, a.mt, k);
    Proc::external_basis(p, a.mt, b);
    double B[kpoly_pairs<Proc>()] = {};
#pragma unroll 1
    for (int h = 0; h < Proc::NHEL; ++h) kpoly_helicity<Proc, T>(k, b, h, B);
    kpoly_outputs<Proc>(B, a, n, e, (a.mode == 0 && w_in) ? w_in[e] : 1.0, out, me0_out);
}

// Accumulators of the kappa-polynomial program with the first NL complex
// entries in the lane's LDS column (entry i at lds[i * S]) and the others in
// registers; the program's indices are constants after inlining, so each
// access resolves to one storage at compile time.
template <typename T, int N, int NL, int S>
struct split_acc {
    cx<T>* lds;
    cx<T> reg[N - NL];
    __device__ __forceinline__ cx<T>& operator[](int i) { return i < NL ? lds[i * S] : reg[i - NL]; }
};

// Large single-precision programs (NG K >= 96 accumulators) keep half of
// their kappa-power accumulators in LDS while the program runs.
template <class Proc, typename T>
constexpr bool kpoly_lds_split() {
    return sizeof(T) == 4 && Proc::NG * Proc::K >= 96;
}

// One event per wave, helicity configurations on the lanes.
template <class Proc, typename T>
__global__ void __launch_bounds__(kBlock)
qcd_kpoly_wave_kernel(const event_data<Proc, T>* __restrict__ ev, int64_t e0, int64_t nb,
                      const double* __restrict__ w_in, int64_t n, qcd_launch a, double* __restrict__ out,
                      double* __restrict__ me0_out) {
    const int64_t el = int64_t(blockIdx.x) * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (el >= nb || ev[el].skip) return;   // whole wave
    const int64_t e = e0 + el;
    const int lane = threadIdx.x & 63;
    double B[kpoly_pairs<Proc>()] = {};
#pragma unroll 1
    for (int hc = 0; hc < Proc::NHEL; hc += 64) {
        __asm__ volatile("" ::: "memory");
        if constexpr (kpoly_lds_split<Proc, T>()) {
            constexpr int N = Proc::NG * Proc::K, NL = N / 2;
            __shared__ cx<T> jl[NL * kBlock];
            split_acc<T, N, NL, kBlock> acc{&jl[threadIdx.x]};
            typename Proc::template ext<T> w;
            typename Proc::template coup<T> c = {T(1), T(1), T(1)};
            Proc::template external<T>(ev[el].b, hc + lane, w);
            Proc::amplitude_kpoly(w, ev[el].k, c, acc);
            cx<T> J[N];
#pragma unroll
            for (int i = 0; i < N; ++i) J[i] = acc[i];
            kpoly_colour<Proc, T>(J, B);
        } else if constexpr (sizeof(T) == 8) {
            // double precision: external wavefunctions in the lane's own LDS
            // slot, as in qcd_wave_kernel (10 % faster for g g -> t tbar g g;
            // in single precision registers are faster)
            __shared__ lds_slot<typename Proc::template ext<T>> wfs[kBlock];
            kpoly_helicity<Proc, T>(ev[el].k, ev[el].b, hc + lane, B, wfs[threadIdx.x].v);
        } else {
            kpoly_helicity<Proc, T>(ev[el].k, ev[el].b, hc + lane, B);
        }
    }
#pragma unroll
    for (int i = 0; i < kpoly_pairs<Proc>(); ++i) B[i] = wave_sum(B[i]);
    if (lane == 0) kpoly_outputs<Proc>(B, a, n, e, (a.mode == 0 && w_in) ? w_in[e] : 1.0, out, me0_out);
}

// ------------------------------------- FP64 rescue of ill-conditioned events
//
// In single precision the helicity amplitudes lose digits where diagrams
// cancel strongly against each other: a final-state gluon nearly collinear to
// a beam gluon or to another final-state gluon (small |2 p_i.p_j| / s).  After
// the single-precision pass, events with such an invariant below a threshold
// are listed and evaluated again in double precision, one event per wave,
// overwriting their results.

template <class Proc>
__global__ void rescue_reset_kernel(unsigned long long* count) {
    if (blockIdx.x == 0 && threadIdx.x == 0) count[0] = 0;
}

// Events e0 .. e0 + nb - 1 of the n in mom.
template <class Proc>
__global__ void __launch_bounds__(kBlock)
rescue_flag_kernel(const double* __restrict__ mom, int64_t n, int64_t e0, int64_t nb, double tau,
                   unsigned long long* __restrict__ count, int64_t* __restrict__ list) {
    const int64_t el = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (el >= nb) return;
    const int64_t e = e0 + el;
    double p[Proc::NEXT][4];
    load_event<Proc::NEXT>(mom, n, e, p);
    if (ill_conditioned<Proc>(p, tau)) list[atomicAdd(count, 1ull)] = e;
}

// Grid-stride over the listed events; each wave takes one event at a time and
// every wave leaves the loop once the list is exhausted.
template <class Proc, bool KP>
__global__ void __launch_bounds__(kBlock, 1)
qcd_rescue_kernel(const double* __restrict__ mom, const int64_t* __restrict__ list,
                  const unsigned long long* __restrict__ count, const double* __restrict__ w_in, int64_t n,
                  qcd_launch a, double* __restrict__ out, double* __restrict__ me0_out) {
    __shared__ event_data<Proc, double> sh[kBlock / 64];
    __shared__ lds_slot<typename Proc::template ext<double>> wfs[kBlock];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t cnt = int64_t(count[0]);
    const int64_t stride = int64_t(gridDim.x) * (kBlock / 64);
    event_data<Proc, double>& d = sh[wv];
#pragma unroll 1
    for (int64_t i = int64_t(blockIdx.x) * (kBlock / 64) + wv; i < cnt; i += stride) {
        const int64_t e = list[i];
        if (lane == 0) {
            double p[Proc::NEXT][4];
            load_event<Proc::NEXT>(mom, n, e, p);
            Proc::kinematics(p, a.mt, d.k);
            Proc::external_basis(p, a.mt, d.b);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double w = (a.mode == 0 && w_in) ? w_in[e] : 1.0;
        if constexpr (KP) {
            double B[kpoly_pairs<Proc>()] = {};
#pragma unroll 1
            for (int hc = 0; hc < Proc::NHEL; hc += 64)
                if (hc + lane < Proc::NHEL) kpoly_helicity<Proc, double>(d.k, d.b, hc + lane, B);
#pragma unroll
            for (int q = 0; q < kpoly_pairs<Proc>(); ++q) B[q] = wave_sum(B[q]);
            if (lane == 0) kpoly_outputs<Proc>(B, a, n, e, w, out, me0_out);
        } else {
            typename Proc::template ext<double>& wf = wfs[threadIdx.x].v;   // own slot
            // one block of 64 configurations: assembled once for all points
            constexpr bool one_block = Proc::NHEL == 64;
            if constexpr (one_block) Proc::template external<double>(d.b, lane, wf);
            double me0 = 0.0;
#pragma unroll 1
            for (int kp = 0; kp < a.npts; ++kp) {
                const qcd_point pt = a.pts[kp];
                const auto c = Proc::template couplings<double>(pt.gs, pt.gs2, pt.gk);
                double acc = 0.0;
#pragma unroll 1
                for (int hc = 0; hc < Proc::NHEL; hc += 64) {
                    if (hc + lane < Proc::NHEL) {
                        if constexpr (!one_block) Proc::template external<double>(d.b, hc + lane, wf);
                        cx<double> J[Proc::K];
                        Proc::amplitude(wf, d.k, c, J);
                        acc += Proc::colour_sum(J);
                    }
                }
                const double me = wave_sum(acc) * Proc::point_norm(pt.gs);
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
        // every lane has read the slot before the next event overwrites it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

constexpr unsigned kRescueBlocks = 1024;

// The FP64 re-evaluation after a one-event-per-lane pass: list the
// ill-conditioned events, then redo them.  With a scratch span the count and
// list live there and the events are flagged and redone chunk by chunk.
template <class Proc>
hipError_t launch_rescue(const double* mom, const double* w_in, int64_t n, const qcd_launch& a, double* out,
                         double* me0, hipStream_t s) {
    if constexpr (Proc::NEXT <= 4) {
        return hipSuccess;   // no final-state gluon
    } else {
        int64_t* buf = nullptr;
        int64_t chunk = n;
        if (a.scratch.ptr) {
            chunk = scratch_chunk(a.scratch, sizeof(int64_t), 256);
            if (chunk < 1) return hipErrorInvalidValue;
            buf = static_cast<int64_t*>(a.scratch.ptr);
        } else {
            hipError_t err = hipMallocAsync(reinterpret_cast<void**>(&buf), sizeof(int64_t) * size_t(n + 1), s);
            if (err != hipSuccess) return err;
        }
        unsigned long long* count = reinterpret_cast<unsigned long long*>(buf);
        int64_t* list = a.scratch.ptr ? buf + 32 : buf + 1;   // after the 256-byte head in a scratch span
        hipError_t err = hipSuccess;
        for (int64_t e0 = 0; e0 < n && err == hipSuccess; e0 += chunk) {
            const int64_t nb = n - e0 < chunk ? n - e0 : chunk;
            hipLaunchKernelGGL((rescue_reset_kernel<Proc>), dim3(1), dim3(64), 0, s, count);
            hipLaunchKernelGGL((rescue_flag_kernel<Proc>), dim3(unsigned((nb + kBlock - 1) / kBlock)), dim3(kBlock),
                               0, s, mom, n, e0, nb, a.rescue_tau, count, list);
            if (a.kpoly)
                hipLaunchKernelGGL((qcd_rescue_kernel<Proc, true>), dim3(kRescueBlocks), dim3(kBlock), 0, s, mom,
                                   list, count, w_in, n, a, out, me0);
            else
                hipLaunchKernelGGL((qcd_rescue_kernel<Proc, false>), dim3(kRescueBlocks), dim3(kBlock), 0, s, mom,
                                   list, count, w_in, n, a, out, me0);
            err = hipGetLastError();
        }
        hipError_t ferr = a.scratch.ptr ? hipSuccess : hipFreeAsync(buf, s);
        return err != hipSuccess ? err : ferr;
    }
}

// One event per wave: per-event data (in single precision with the rescue
// on, also the list of ill-conditioned events, which the amplitude kernel
// skips), the amplitude kernel, then the FP64 re-evaluation of the listed
// events.  KP: kappa-polynomial evaluation.  Without a scratch span the
// buffers are stream-ordered allocations for all n events; with one they are
// carved from it (records, then count and list) and the events run in chunks
// whose buffers fit.
template <class Proc, typename T, bool KP>
hipError_t launch_wave_pipeline(const double* mom, const double* w_in, int64_t n, const qcd_launch& a, double* out,
                                double* me0, hipStream_t s) {
    const bool rescue = sizeof(T) == 4 && a.rescue_tau > 0.0 && Proc::NEXT > 4;
    using ED = event_data<Proc, T>;
    ED* ev = nullptr;
    int64_t* buf = nullptr;
    int64_t chunk = n;
    if (a.scratch.ptr) {
        // per event: one record and (rescue) one list entry; head: the count
        // word and the alignment of the list
        chunk = scratch_chunk(a.scratch, sizeof(ED) + (rescue ? sizeof(int64_t) : 0), 512);
        if (chunk < 1) return hipErrorInvalidValue;
        ev = static_cast<ED*>(a.scratch.ptr);
        if (rescue)
            buf = reinterpret_cast<int64_t*>(static_cast<char*>(a.scratch.ptr) + align256(sizeof(ED) * size_t(chunk)));
    } else {
        hipError_t err = hipMallocAsync(reinterpret_cast<void**>(&ev), sizeof(ED) * size_t(n), s);
        if (err != hipSuccess) return err;
        if (rescue) {
            err = hipMallocAsync(reinterpret_cast<void**>(&buf), sizeof(int64_t) * size_t(n + 1), s);
            if (err != hipSuccess) {
                (void)hipFreeAsync(ev, s);
                return err;
            }
        }
    }
    unsigned long long* count = rescue ? reinterpret_cast<unsigned long long*>(buf) : nullptr;
    int64_t* list = rescue ? buf + 1 : nullptr;
    hipError_t err = hipSuccess;
    for (int64_t e0 = 0; e0 < n && err == hipSuccess; e0 += chunk) {
        const int64_t nb = n - e0 < chunk ? n - e0 : chunk;
        if (rescue) hipLaunchKernelGGL((rescue_reset_kernel<Proc>), dim3(1), dim3(64), 0, s, count);
        hipLaunchKernelGGL((qcd_setup_kernel<Proc, T>), dim3(unsigned((nb + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, mom, n, e0, nb, a.mt, ev, rescue ? a.rescue_tau : 0.0, count, list);
        const dim3 grid(unsigned((nb + kBlock / 64 - 1) / (kBlock / 64)));
        mark(a.t0, s);
        if constexpr (KP)
            hipLaunchKernelGGL((qcd_kpoly_wave_kernel<Proc, T>), grid, dim3(kBlock), 0, s, ev, e0, nb, w_in, n, a,
                               out, me0);
        else
            hipLaunchKernelGGL((qcd_wave_kernel<Proc, T>), grid, dim3(kBlock), 0, s, ev, e0, nb, w_in, n, a, out,
                               me0);
        mark(a.t1, s);
        if (rescue)
            hipLaunchKernelGGL((qcd_rescue_kernel<Proc, KP>), dim3(kRescueBlocks), dim3(kBlock), 0, s, mom, list,
                               count, w_in, n, a, out, me0);
        err = hipGetLastError();
    }
    if (a.scratch.ptr) return err;
    hipError_t f1 = rescue ? hipFreeAsync(buf, s) : hipSuccess;
    hipError_t f2 = hipFreeAsync(ev, s);
    return err != hipSuccess ? err : (f1 != hipSuccess ? f1 : f2);
}

template <class Proc, typename T>
hipError_t launch_kpoly(const double* mom, const double* w_in, int64_t n, const qcd_launch& a, double* out,
                        double* me0, hipStream_t s) {
    if constexpr (Proc::NHEL % 64 == 0) {
        return launch_wave_pipeline<Proc, T, true>(mom, w_in, n, a, out, me0, s);
    } else {
        mark(a.t0, s);
        hipLaunchKernelGGL((qcd_kpoly_lane_kernel<Proc, T>), dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, s, mom, w_in, n, a, out, me0);
        mark(a.t1, s);
        return hipGetLastError();
    }
}

// ------------------------------------------- programs split over kernels
//
// For the largest process the per-helicity program is split into NCHUNK
// functions (consecutive closing groups); kernel C runs part C for every
// point and helicity of a batch of events, one event per wave with the
// helicity configurations on the lanes.  The colour-flow amplitudes J travel
// between the parts through HBM in a [event][point][component][helicity]
// layout (consecutive lanes touch consecutive words).  By default the last
// part forms the colour sum (VALU), the helicity sum (wave reduction) and the
// reweighted weights; with the matrix-core colour sum selected it stores J
// too, and qcd_colour_mfma_kernel contracts J with the colour matrix.

// Processes whose generated struct provides the bfloat16 split of the colour
// matrix (MFMA_COLOUR) take the matrix-core colour sum.
template <class P, class = void>
struct mfma_colour : std::false_type {};
template <class P>
struct mfma_colour<P, std::void_t<decltype(P::MFMA_COLOUR)>> : std::bool_constant<P::MFMA_COLOUR> {};

#ifndef MGRW_PART_WPE
#define MGRW_PART_WPE 1
#endif

template <class Proc, typename T, int C, bool STORE_LAST>
__global__ void __launch_bounds__(kBlock, MGRW_PART_WPE)
qcd_part_kernel(const event_data<Proc, T>* __restrict__ ev, int64_t e0, int64_t nb, T* __restrict__ jbuf,
                const double* __restrict__ w_in, int64_t n, qcd_launch a, double* __restrict__ out,
                double* __restrict__ me0_out) {
    constexpr int NH = Proc::NHEL, K2 = 2 * Proc::K;
    constexpr bool LAST = C + 1 == Proc::NCHUNK && !STORE_LAST;   // finishes the events here
    static_assert(NH % 64 == 0, "helicity configurations must fill whole waves");
    const int64_t el = int64_t(blockIdx.x) * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (el >= nb) return;   // whole wave; no barriers below
    const int64_t e = e0 + el;
    if (ev[e].skip) return;   // left to the FP64 re-evaluation
    const int lane = threadIdx.x & 63;
    const typename Proc::template kin<T>& k = ev[e].k;
    const typename Proc::template basis<T>& b = ev[e].b;
    const double w = (LAST && a.mode == 0 && w_in) ? w_in[e] : 1.0;
    double me0 = 0.0;
#pragma unroll 1
    for (int kp = 0; kp < a.npts; ++kp) {
        const qcd_point pt = a.pts[kp];
        const auto c = Proc::template couplings<T>(pt.gs, pt.gs2, pt.gk);
        double acc = 0.0;
#pragma unroll 1
        for (int hc = 0; hc < NH; hc += 64) {
            __asm__ volatile("" ::: "memory");
            __shared__ lds_slot<typename Proc::template ext<T>> wfs[kBlock];
            typename Proc::template ext<T>& wf = wfs[threadIdx.x].v;   // own slot, as in qcd_wave_kernel
            Proc::template external<T>(b, hc + lane, wf);
            T* jp = jbuf + (el * a.npts + kp) * int64_t(K2) * NH + hc + lane;
            cx<T> J[Proc::K];
            if constexpr (C == 0) {
#pragma unroll
                for (int f = 0; f < Proc::K; ++f) J[f] = {T(0), T(0)};
            } else {
#pragma unroll
                for (int f = 0; f < Proc::K; ++f) J[f] = {jp[(2 * f) * NH], jp[(2 * f + 1) * NH]};
            }
            Proc::template amplitude_part<C>(wf, k, c, J);
            if constexpr (!LAST) {
#pragma unroll
                for (int f = 0; f < Proc::K; ++f) {
                    jp[(2 * f) * NH] = J[f].re;
                    jp[(2 * f + 1) * NH] = J[f].im;
                }
            } else {
                acc += double(Proc::colour_sum(J));
            }
        }
        if constexpr (LAST) {
            const double me = wave_sum(acc) * Proc::point_norm(pt.gs);
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
}

template <class Proc, typename T, int C>
hipError_t launch_part(const event_data<Proc, T>* ev, int64_t e0, int64_t nb, T* jbuf, const double* w_in,
                       int64_t n, const qcd_launch& a, double* out, double* me0, hipStream_t s) {
    const dim3 grid(unsigned((nb + kBlock / 64 - 1) / (kBlock / 64)));
    if constexpr (C + 1 == Proc::NCHUNK && mfma_colour<Proc>::value) {
        if (a.colour_mfma) {
            hipLaunchKernelGGL((qcd_part_kernel<Proc, T, C, true>), grid, dim3(kBlock), 0, s, ev, e0, nb, jbuf, w_in, n,
                               a, out, me0);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((qcd_part_kernel<Proc, T, C, false>), grid, dim3(kBlock), 0, s, ev, e0, nb, jbuf, w_in, n, a,
                       out, me0);
    return hipGetLastError();
}

// ---------------------------------------------- colour sum on the matrix cores
//
// After the last program part, J of every (event, point, helicity) is in HBM
// as X[c][n] (c = 2 flow + re/im, n = helicity).  Per event and point the
// colour sum over all helicities is
//   sum_h J_h^+ CF J_h = sum_{f, n} X_f[n] (CF X)_f[n],
// with X_f the 2 NHEL real columns (real and imaginary parts) of flow f.
// D = CF X runs on v_mfma_f32_32x32x16_bf16: CF's integer numerators are the
// exact sum of two bfloat16 matrices (CF_BF16_HI + CF_BF16_LO, padded to KP),
// X is split into three bfloat16 terms x1 + x2 + x3 (24 significant bits), and
// the five products with weight above 2^-24 are accumulated in float32; the
// final dot product uses X itself (float32) from HBM.  One workgroup (4 waves)
// per event; each wave owns a quarter of D's columns.

typedef __attribute__((ext_vector_type(8))) __bf16 cbf16x8;
typedef __attribute__((ext_vector_type(8))) unsigned short cu16x8;
typedef __attribute__((ext_vector_type(16))) float cf32x16;

__device__ __forceinline__ unsigned short bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short b) { return __uint_as_float(unsigned(b) << 16); }

template <class Proc>
__global__ void __launch_bounds__(kBlock)
qcd_colour_mfma_kernel(const float* __restrict__ jbuf, int64_t e0, int64_t nb, const double* __restrict__ w_in,
                       int64_t n, qcd_launch a, double* __restrict__ out, double* __restrict__ me0_out) {
    constexpr int K = Proc::K, KP = Proc::KP, NH = Proc::NHEL, NCOL = 2 * NH;
    static_assert(KP % 32 == 0 && NCOL % 128 == 0, "tile shapes");
    constexpr int MT = KP / 32, KS = KP / 16, NT_WAVE = NCOL / 32 / (kBlock / 64);
    const int64_t el = blockIdx.x;
    if (el >= nb) return;   // whole block
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 31, lh = lane >> 5;
    __shared__ double part[kBlock / 64];
    const double w = (a.mode == 0 && w_in) ? w_in[e0 + el] : 1.0;
    double me0 = 0.0;
#pragma unroll 1
    for (int kp = 0; kp < a.npts; ++kp) {
        const float* X = jbuf + (el * a.npts + kp) * int64_t(2 * K) * NH;
        float s = 0.0f;
#pragma unroll 1
        for (int t = 0; t < NT_WAVE; ++t) {
            const int ncol = (wv * NT_WAVE + t) * 32 + lr;   // this lane's column of D
            const int re_im = ncol / NH, h = ncol % NH;
            // B = X in three bfloat16 terms, all k-steps of this column tile
            cbf16x8 b1[KS], b2[KS], b3[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                cu16x8 u1, u2, u3;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int f = ks * 16 + lh * 8 + r;
                    const float x = f < K ? X[int64_t(2 * f + re_im) * NH + h] : 0.0f;
                    const unsigned short x1 = bf16_rne(x);
                    const float r1 = x - bf16_float(x1);
                    const unsigned short x2 = bf16_rne(r1);
                    const unsigned short x3 = bf16_rne(r1 - bf16_float(x2));
                    u1[r] = x1;
                    u2[r] = x2;
                    u3[r] = x3;
                }
                b1[ks] = __builtin_bit_cast(cbf16x8, u1);
                b2[ks] = __builtin_bit_cast(cbf16x8, u2);
                b3[ks] = __builtin_bit_cast(cbf16x8, u3);
            }
#pragma unroll 1
            for (int mt = 0; mt < MT; ++mt) {
                cf32x16 acc = {};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    cu16x8 hi, lo;
                    const int row = mt * 32 + lr, k0 = ks * 16 + lh * 8;
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        hi[r] = Proc::CF_BF16_HI[row * KP + k0 + r];
                        lo[r] = Proc::CF_BF16_LO[row * KP + k0 + r];
                    }
                    const cbf16x8 ah = __builtin_bit_cast(cbf16x8, hi), al = __builtin_bit_cast(cbf16x8, lo);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b1[ks], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b2[ks], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b1[ks], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b3[ks], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b2[ks], acc, 0, 0, 0);
                }
                // D[m][ncol] for m = mt*32 + (r/4)*8 + lh*4 + r%4, dotted with X[m][ncol]
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int f = mt * 32 + (r / 4) * 8 + lh * 4 + r % 4;
                    if (f < K) s += X[int64_t(2 * f + re_im) * NH + h] * acc[r];
                }
            }
        }
        double v = wave_sum(double(s));
        if (lane == 0) part[wv] = v;
        __syncthreads();
        double me = 0.0;
        for (int i = 0; i < kBlock / 64; ++i) me += part[i];
        me *= Proc::point_norm(a.pts[kp].gs);
        __syncthreads();   // part[] is rewritten for the next point
        if (threadIdx.x == 0) {
            const int64_t e = e0 + el;
            if (kp == 0) {
                me0 = me;
                if (a.mode == 1)
                    out[e] = me;
                else if (me0_out)
                    me0_out[e] = me;
            } else {
                out[int64_t(kp - 1) * n + e] = reweighted(w, me, me0);
            }
        }
    }
}

template <class Proc>
hipError_t launch_colour_mfma(const float* jbuf, int64_t e0, int64_t nb, const double* w_in, int64_t n,
                              const qcd_launch& a, double* out, double* me0, hipStream_t s) {
    if constexpr (mfma_colour<Proc>::value) {
        if (!a.colour_mfma) return hipSuccess;
        hipLaunchKernelGGL((qcd_colour_mfma_kernel<Proc>), dim3(unsigned(nb)), dim3(kBlock), 0, s, jbuf, e0, nb, w_in,
                           n, a, out, me0);
        return hipGetLastError();
    } else {
        return hipSuccess;
    }
}

// ------------------------------ double-precision instance of the split programs
//
// In double precision the 120 colour-flow amplitudes of g g -> t tbar g g g
// alone would take 480 registers per lane.  The generated program is
// therefore also cut by colour flow: amplitude_fr<C, R> holds the diagrams of
// chunk C of the closing groups that contribute to flow range R (KR flows),
// so only KR amplitudes are live at a time; diagrams with terms in several
// ranges are evaluated once per range.  Kernel (C, R) runs it for a batch of
// events, one event per wave with the helicity configurations on the lanes,
// and passes the range's amplitudes through HBM ([event][point][component]
// [helicity], as the single-precision parts do); qcd_colour64_kernel then
// forms the colour sum from HBM, the helicity sum and the weights.
//
// The same pipeline re-evaluates the ill-conditioned events of the
// single-precision pass: slots are then positions in the list of those
// events (count on the device), and slots beyond the count exit at once.

// Per-event data of one slot: event e itself, or list[slot].
template <class Proc>
__global__ void __launch_bounds__(kBlock)
qcd_setup64_kernel(const double* __restrict__ mom, int64_t n, double mt, const int64_t* __restrict__ list,
                   const unsigned long long* __restrict__ count, int64_t slots,
                   event_data<Proc, double>* __restrict__ ev) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= slots || (count && i >= int64_t(count[0]))) return;
    const int64_t e = list ? list[i] : i;
    double p[Proc::NEXT][4];
    load_event<Proc::NEXT>(mom, n, e, p);
    Proc::kinematics(p, mt, ev[i].k);
    Proc::external_basis(p, mt, ev[i].b);
    ev[i].skip = 0;
}

template <class Proc, int C, int R>
__global__ void __launch_bounds__(kBlock, 1)
qcd_fr_kernel(const event_data<Proc, double>* __restrict__ ev, const unsigned long long* __restrict__ count,
              int64_t e0, int64_t nb, double* __restrict__ jbuf, qcd_launch a) {
    constexpr int NH = Proc::NHEL, K2 = 2 * Proc::K, KR = Proc::KR;
    static_assert(NH % 64 == 0, "helicity configurations must fill whole waves");
    const int64_t el = int64_t(blockIdx.x) * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (el >= nb) return;   // whole wave; no barriers below
    const int64_t i = e0 + el;
    if (count && i >= int64_t(count[0])) return;
    const int lane = threadIdx.x & 63;
    const typename Proc::template kin<double>& k = ev[i].k;
    const typename Proc::template basis<double>& b = ev[i].b;
#pragma unroll 1
    for (int kp = 0; kp < a.npts; ++kp) {
        const qcd_point pt = a.pts[kp];
        const auto c = Proc::template couplings<double>(pt.gs, pt.gs2, pt.gk);
#pragma unroll 1
        for (int hc = 0; hc < NH; hc += 64) {
            __asm__ volatile("" ::: "memory");
            __shared__ lds_slot<typename Proc::template ext<double>> wfs[kBlock];
            typename Proc::template ext<double>& wf = wfs[threadIdx.x].v;   // own slot
            Proc::template external<double>(b, hc + lane, wf);
            double* jp = jbuf + (el * a.npts + kp) * int64_t(K2) * NH + int64_t(2 * R * KR) * NH + hc + lane;
            cx<double> J[KR];
            if constexpr (C == 0) {
#pragma unroll
                for (int f = 0; f < KR; ++f) J[f] = {0.0, 0.0};
            } else {
#pragma unroll
                for (int f = 0; f < KR; ++f) J[f] = {jp[(2 * f) * NH], jp[(2 * f + 1) * NH]};
            }
            Proc::template amplitude_fr<C, R>(wf, k, c, J);
#pragma unroll
            for (int f = 0; f < KR; ++f) {
                jp[(2 * f) * NH] = J[f].re;
                jp[(2 * f + 1) * NH] = J[f].im;
            }
        }
    }
}

// Flows per block of the streamed colour sum (z = CF J for BS rows at a time).
constexpr int kColourBlock = 40;

// sum_h J_h^+ CF J_h from the amplitudes in HBM: per lane (helicity) and block
// of kColourBlock rows, z_i = sum_t CF[t][i] J_t with J_t streamed from memory
// (CF symmetric, row t of the table contiguous in i, read through the scalar
// cache), then the block's Re(J_i^* z_i); helicity sum by wave reduction.
template <class Proc>
__global__ void __launch_bounds__(kBlock)
qcd_colour64_kernel(const double* __restrict__ jbuf, const int64_t* __restrict__ list,
                    const unsigned long long* __restrict__ count, int64_t e0, int64_t nb,
                    const double* __restrict__ w_in, int64_t n, qcd_launch a, double* __restrict__ out,
                    double* __restrict__ me0_out) {
    constexpr int K = Proc::K, NH = Proc::NHEL, BS = kColourBlock;
    static_assert(K % BS == 0, "colour blocks");
    const int64_t el = int64_t(blockIdx.x) * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (el >= nb) return;   // whole wave
    if (count && e0 + el >= int64_t(count[0])) return;
    const int64_t e = list ? list[e0 + el] : e0 + el;
    const int lane = threadIdx.x & 63;
    const double w = (a.mode == 0 && w_in) ? w_in[e] : 1.0;
    double me0 = 0.0;
#pragma unroll 1
    for (int kp = 0; kp < a.npts; ++kp) {
        double acc = 0.0;
#pragma unroll 1
        for (int hc = 0; hc < NH; hc += 64) {
            const double* X = jbuf + (el * a.npts + kp) * int64_t(2 * K) * NH + hc + lane;
#pragma unroll 1
            for (int a0 = 0; a0 < K; a0 += BS) {
                double zr[BS], zi[BS];
#pragma unroll
                for (int q = 0; q < BS; ++q) zr[q] = zi[q] = 0.0;
#pragma unroll 2
                for (int t = 0; t < K; ++t) {
                    const double jr = X[(2 * t) * NH], ji = X[(2 * t + 1) * NH];
                    const double* cf = Proc::CF_DBL + t * K + a0;
#pragma unroll
                    for (int q = 0; q < BS; ++q) {
                        zr[q] = fma(cf[q], jr, zr[q]);
                        zi[q] = fma(cf[q], ji, zi[q]);
                    }
                }
#pragma unroll
                for (int q = 0; q < BS; ++q)
                    acc += zr[q] * X[(2 * (a0 + q)) * NH] + zi[q] * X[(2 * (a0 + q) + 1) * NH];
            }
        }
        const double me = wave_sum(acc) * Proc::point_norm(a.pts[kp].gs);
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

template <class Proc, int C, int R>
hipError_t launch_fr(const event_data<Proc, double>* ev, const unsigned long long* count, int64_t e0, int64_t nb,
                     double* jbuf, const qcd_launch& a, hipStream_t s) {
    const dim3 grid(unsigned((nb + kBlock / 64 - 1) / (kBlock / 64)));
    hipLaunchKernelGGL((qcd_fr_kernel<Proc, C, R>), grid, dim3(kBlock), 0, s, ev, count, e0, nb, jbuf, a);
    return hipGetLastError();
}

// Kernel launchers of a split program, one translation unit each.
template <class Proc>
struct split_launchers {
    using part_fn = hipError_t (*)(const event_data<Proc, float>*, int64_t, int64_t, float*, const double*, int64_t,
                                   const qcd_launch&, double*, double*, hipStream_t);
    using fr_fn = hipError_t (*)(const event_data<Proc, double>*, const unsigned long long*, int64_t, int64_t,
                                 double*, const qcd_launch&, hipStream_t);
    part_fn part[Proc::NCHUNK];
    fr_fn fr[Proc::NCHUNK64 * Proc::NFR];
};

// Events per batch of the split programs: the buffer that carries J between
// the parts holds batch x points x 2K x NHEL values of T, about 16 GiB at most.
constexpr int64_t kPartBatch = 8192;
constexpr size_t kJBufBytes = size_t(16) << 30;
template <class Proc, typename T>
int64_t part_batch(int64_t n, int npts) {
    const size_t per_event = size_t(npts) * 2 * Proc::K * Proc::NHEL * sizeof(T);
    int64_t b = int64_t(kJBufBytes / per_event);
    b = b > kPartBatch ? kPartBatch : (b < 64 ? 64 : b);
    return n < b ? n : b;
}

// Double-precision pipeline over `slots` slots: per-slot data, then batches
// through the (chunk, range) kernels and the colour sum.  list == NULL: slot
// i is event i; otherwise slot i is event list[i] for i < count[0].
template <class Proc>
hipError_t launch_split64(const split_launchers<Proc>& L, const double* mom, int64_t n, const int64_t* list,
                          const unsigned long long* count, int64_t slots, const double* w_in, const qcd_launch& a,
                          double* out, double* me0, hipStream_t s, bool timed) {
    using ED = event_data<Proc, double>;
    const int64_t B = part_batch<Proc, double>(slots, a.npts);
    ED* ev = nullptr;
    double* jbuf = nullptr;
    hipError_t err = hipMallocAsync(reinterpret_cast<void**>(&ev), sizeof(ED) * size_t(slots), s);
    if (err != hipSuccess) return err;
    err = hipMallocAsync(reinterpret_cast<void**>(&jbuf),
                         sizeof(double) * size_t(B) * a.npts * 2 * Proc::K * Proc::NHEL, s);
    if (err != hipSuccess) {
        (void)hipFreeAsync(ev, s);
        return err;
    }
    hipLaunchKernelGGL((qcd_setup64_kernel<Proc>), dim3(unsigned((slots + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       mom, n, a.mt, list, count, slots, ev);
    err = hipGetLastError();
    if (timed) mark(a.t0, s);
    // One (chunk, range) kernel at one wave per SIMD leaves SIMDs idle: with
    // few events per batch (re-evaluating listed events) most of them, and in
    // the last round of waves of a full batch nearly all.  The ranges of a
    // chunk write disjoint parts of jbuf, so they run side by side, range 0
    // on the caller's stream and the others on library streams, joined per
    // chunk.
    constexpr int NFR = Proc::NFR;
    const bool side = NFR - 1 <= kAuxStreams;
    hipStream_t aux[kAuxStreams] = {};
    hipEvent_t fork = nullptr, join[kAuxStreams] = {};
    if (err == hipSuccess && side) {
        err = aux_streams(aux);
        if (err == hipSuccess) err = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        for (int r = 1; r < NFR && err == hipSuccess; ++r) err = hipEventCreateWithFlags(&join[r - 1], hipEventDisableTiming);
    }
    for (int64_t e0 = 0; e0 < slots && err == hipSuccess; e0 += B) {
        const int64_t nb = slots - e0 < B ? slots - e0 : B;
        for (int c = 0; c < Proc::NCHUNK64 && err == hipSuccess; ++c) {
            if (!side) {
                for (int r = 0; r < NFR && err == hipSuccess; ++r) err = L.fr[c * NFR + r](ev, count, e0, nb, jbuf, a, s);
                continue;
            }
            err = hipEventRecord(fork, s);
            for (int r = 1; r < NFR && err == hipSuccess; ++r) err = hipStreamWaitEvent(aux[r - 1], fork, 0);
            if (err == hipSuccess) err = L.fr[c * NFR](ev, count, e0, nb, jbuf, a, s);
            bool used[kAuxStreams] = {};
            for (int r = 1; r < NFR && err == hipSuccess; ++r) {
                used[r - 1] = true;   // a failed launch may still have queued work
                err = L.fr[c * NFR + r](ev, count, e0, nb, jbuf, a, aux[r - 1]);
            }
            // join every library stream that received work, also after an
            // error, before the buffers are released on the caller's stream
            for (int r = 1; r < NFR; ++r) {
                if (!used[r - 1]) continue;
                hipError_t j = hipEventRecord(join[r - 1], aux[r - 1]);
                if (j == hipSuccess) j = hipStreamWaitEvent(s, join[r - 1], 0);
                if (j != hipSuccess) (void)hipStreamSynchronize(aux[r - 1]);
                if (err == hipSuccess) err = j;
            }
        }
        if (err == hipSuccess) {
            hipLaunchKernelGGL((qcd_colour64_kernel<Proc>), dim3(unsigned((nb + kBlock / 64 - 1) / (kBlock / 64))),
                               dim3(kBlock), 0, s, jbuf, list, count, e0, nb, w_in, n, a, out, me0);
            err = hipGetLastError();
        }
    }
    if (timed) mark(a.t1, s);
    // the events are released once their pending work has completed
    if (fork) (void)hipEventDestroy(fork);
    for (int r = 0; r < kAuxStreams; ++r)
        if (join[r]) (void)hipEventDestroy(join[r]);
    hipError_t f1 = hipFreeAsync(jbuf, s), f2 = hipFreeAsync(ev, s);
    return err != hipSuccess ? err : (f1 != hipSuccess ? f1 : f2);
}

// A split program: FP64 runs the double-precision pipeline over all events;
// mixed precision runs the per-event data (listing ill-conditioned events
// when the re-evaluation is on), batches through the single-precision parts
// (and the matrix-core colour sum when selected), then the listed events
// through the double-precision pipeline.
template <class Proc>
hipError_t launch_split(const split_launchers<Proc>& L, int fp64, const double* mom, const double* w_in, int64_t n,
                        const qcd_launch& a, double* out, double* me0, hipStream_t s) {
    if (a.scratch.ptr) return hipErrorNotSupported;   // J buffers of MBs per event: always allocated
    if (fp64) return launch_split64<Proc>(L, mom, n, nullptr, nullptr, n, w_in, a, out, me0, s, true);
    using ED = event_data<Proc, float>;
    const bool rescue = a.rescue_tau > 0.0;
    const int64_t B = part_batch<Proc, float>(n, a.npts);
    ED* ev = nullptr;
    float* jbuf = nullptr;
    int64_t* buf = nullptr;
    hipError_t err = hipMallocAsync(reinterpret_cast<void**>(&ev), sizeof(ED) * size_t(n), s);
    if (err != hipSuccess) return err;
    err = hipMallocAsync(reinterpret_cast<void**>(&jbuf), sizeof(float) * size_t(B) * a.npts * 2 * Proc::K * Proc::NHEL,
                         s);
    if (err == hipSuccess && rescue)
        err = hipMallocAsync(reinterpret_cast<void**>(&buf), sizeof(int64_t) * size_t(n + 1), s);
    if (err != hipSuccess) {
        if (jbuf) (void)hipFreeAsync(jbuf, s);
        (void)hipFreeAsync(ev, s);
        return err;
    }
    unsigned long long* count = rescue ? reinterpret_cast<unsigned long long*>(buf) : nullptr;
    int64_t* list = rescue ? buf + 1 : nullptr;
    if (rescue) hipLaunchKernelGGL((rescue_reset_kernel<Proc>), dim3(1), dim3(64), 0, s, count);
    hipLaunchKernelGGL((qcd_setup_kernel<Proc, float>), dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       mom, n, int64_t(0), n, a.mt, ev, rescue ? a.rescue_tau : 0.0, count, list);
    err = hipGetLastError();
    mark(a.t0, s);
    for (int64_t e0 = 0; e0 < n && err == hipSuccess; e0 += B) {
        const int64_t nb = n - e0 < B ? n - e0 : B;
        for (int c = 0; c < Proc::NCHUNK && err == hipSuccess; ++c)
            err = L.part[c](ev, e0, nb, jbuf, w_in, n, a, out, me0, s);
        if (err == hipSuccess) err = launch_colour_mfma<Proc>(jbuf, e0, nb, w_in, n, a, out, me0, s);
    }
    mark(a.t1, s);
    hipError_t f1 = hipFreeAsync(jbuf, s), f2 = hipFreeAsync(ev, s);
    if (err == hipSuccess && rescue)
        err = launch_split64<Proc>(L, mom, n, list, count, n, w_in, a, out, me0, s, false);
    hipError_t f3 = rescue ? hipFreeAsync(buf, s) : hipSuccess;
    return err != hipSuccess ? err : (f1 != hipSuccess ? f1 : (f2 != hipSuccess ? f2 : f3));
}

// Launch the reweight (mode 0) or single-point (mode 1) kernels of Proc at the
// requested arithmetic; returns the launch status.
template <class Proc, typename T>
hipError_t launch_wave(const double* mom, const double* w_in, int64_t n, const qcd_launch& a, double* out,
                       double* me0, hipStream_t s) {
    if constexpr (Proc::NHEL % 64 != 0)
        return hipErrorInvalidConfiguration;
    else
        return launch_wave_pipeline<Proc, T, false>(mom, w_in, n, a, out, me0, s);
}

template <class Proc>
hipError_t launch_main(int fp64, const double* mom, const double* w_in, int64_t n, const qcd_launch& a,
                       double* out, double* me0, hipStream_t s) {
    if (a.kpoly)
        return fp64 ? launch_kpoly<Proc, double>(mom, w_in, n, a, out, me0, s)
                    : launch_kpoly<Proc, float>(mom, w_in, n, a, out, me0, s);
    if (a.mapping == MGRW_MAP_EVENT_PER_WAVE)
        return fp64 ? launch_wave<Proc, double>(mom, w_in, n, a, out, me0, s)
                    : launch_wave<Proc, float>(mom, w_in, n, a, out, me0, s);
    constexpr int NBD = lane_block<Proc, double>(), NBF = lane_block<Proc, float>();
    mark(a.t0, s);
    if (fp64)
        hipLaunchKernelGGL((qcd_kernel<Proc, double>), dim3(unsigned((n + NBD - 1) / NBD)), dim3(NBD), 0, s, mom, w_in,
                           n, a, out, me0);
    else
        hipLaunchKernelGGL((qcd_kernel<Proc, float>), dim3(unsigned((n + NBF - 1) / NBF)), dim3(NBF), 0, s, mom, w_in,
                           n, a, out, me0);
    mark(a.t1, s);
    return hipGetLastError();
}

template <class Proc>
hipError_t launch_qcd(int fp64, const double* mom, const double* w_in, int64_t n, const qcd_launch& a,
                      double* out, double* me0, hipStream_t s) {
    hipError_t err = launch_main<Proc>(fp64, mom, w_in, n, a, out, me0, s);
    if (err != hipSuccess || fp64 || !(a.rescue_tau > 0.0)) return err;
    // the one-event-per-wave pipelines re-evaluate their listed events themselves
    const bool wave = a.kpoly ? Proc::NHEL % 64 == 0 : a.mapping == MGRW_MAP_EVENT_PER_WAVE;
    if (wave) return err;
    return launch_rescue<Proc>(mom, w_in, n, a, out, me0, s);
}

}  // namespace mgrw
