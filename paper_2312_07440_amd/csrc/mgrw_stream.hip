// Reweighting of events held in host memory (the paper's timings include the
// transfers, and for small samples the transfers dominate: Sec. 3.3).  The
// batch is cut into chunks; each chunk's host-to-device copy, reweight and
// device-to-host copy are queued on one of two streams in turn, so the copies
// of one chunk overlap the kernels of the other.  The host arrays keep the
// layouts of mgrw_reweight (structure of arrays over all n events): a chunk is
// a 2-D copy (rows of n doubles, m of them per row).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string>

#include "../../include/mgrw.h"
#include "mgrw_internal.h"

namespace {

constexpr int64_t kDefaultChunk = int64_t(1) << 18;

}  // namespace

// Two streams and two staging slots, kept by the handle between calls (the
// slots grow to the largest chunk seen; freed with the handle).
struct mgrw::host_pipeline {
    hipStream_t s[2] = {nullptr, nullptr};
    double* buf[2] = {nullptr, nullptr};
    size_t doubles = 0;   // per slot
};

void mgrw::host_pipeline_destroy(host_pipeline* h) {
    if (!h) return;
    for (int i = 0; i < 2; ++i) {
        if (h->s[i]) (void)hipStreamSynchronize(h->s[i]);
        if (h->buf[i]) (void)hipFree(h->buf[i]);
        if (h->s[i]) (void)hipStreamDestroy(h->s[i]);
    }
    delete h;
}

extern "C" mgrw_status mgrw_reweight_host(mgrw_process* p, const double* mom, const double* w_in, int64_t n_events,
                                          double* w_out, double* me_base_out, int64_t chunk) {
    using mgrw::set_error;
    if (!p) return set_error(MGRW_ERR_ARG, "process is NULL");
    if (p->n_points == 0) return set_error(MGRW_ERR_STATE, "no parameter points set");
    if (n_events < 0) return set_error(MGRW_ERR_ARG, "n_events < 0");
    if (chunk < 0) return set_error(MGRW_ERR_ARG, "chunk < 0");
    if (n_events == 0) return MGRW_OK;
    if (!mom || !w_out) return set_error(MGRW_ERR_ARG, "mom or w_out is NULL");
    int n_ext = 0;
    mgrw_status st = mgrw_process_info(p, &n_ext, nullptr, nullptr, nullptr);
    if (st != MGRW_OK) return st;
    const int P = p->n_points;
    const int64_t c = std::min(chunk == 0 ? kDefaultChunk : chunk, n_events);
    auto dev_fail = [](hipError_t err) {
        return set_error(MGRW_ERR_DEVICE, std::string("host reweight: ") + hipGetErrorString(err));
    };
    // per slot: momenta [n_ext*4][c], input weights [c], outputs [P][c], base |M|^2 [c]
    const size_t per_slot = size_t(c) * (size_t(n_ext) * 4 + 1 + size_t(P) + 1);
    if (!p->hp) {
        p->hp = new (std::nothrow) mgrw::host_pipeline;
        if (!p->hp) return set_error(MGRW_ERR_ALLOC, "out of host memory");
        for (int i = 0; i < 2; ++i) {
            hipError_t err = hipStreamCreateWithFlags(&p->hp->s[i], hipStreamNonBlocking);
            if (err != hipSuccess) {
                p->hp->s[i] = nullptr;
                return dev_fail(err);
            }
        }
    }
    mgrw::host_pipeline& h = *p->hp;
    if (h.doubles < per_slot) {
        for (int i = 0; i < 2; ++i) {
            (void)hipStreamSynchronize(h.s[i]);
            if (h.buf[i]) (void)hipFree(h.buf[i]);
            h.buf[i] = nullptr;
        }
        h.doubles = 0;
        for (int i = 0; i < 2; ++i) {
            hipError_t err = hipMalloc(reinterpret_cast<void**>(&h.buf[i]), per_slot * sizeof(double));
            if (err != hipSuccess) {
                h.buf[i] = nullptr;
                return err == hipErrorOutOfMemory ? set_error(MGRW_ERR_ALLOC, "host reweight: out of device memory")
                                                  : dev_fail(err);
            }
        }
        h.doubles = per_slot;
    }
    // on an error, let what is queued finish before the caller's buffers may go away
    auto drain = [&h](mgrw_status status) {
        for (int i = 0; i < 2; ++i) (void)hipStreamSynchronize(h.s[i]);
        return status;
    };
    const size_t row = size_t(n_events) * sizeof(double);
    int slot = 0;
    for (int64_t e0 = 0; e0 < n_events; e0 += c, slot ^= 1) {
        const int64_t m = std::min(c, n_events - e0);
        const size_t w = size_t(m) * sizeof(double);
        double* mom_d = h.buf[slot];
        double* w_d = mom_d + size_t(c) * n_ext * 4;
        double* out_d = w_d + c;
        double* me0_d = out_d + size_t(c) * P;
        hipStream_t s = h.s[slot];
        // the slot's previous chunk is ordered before this one on the same stream
        hipError_t err = hipMemcpy2DAsync(mom_d, w, mom + e0, row, w, size_t(n_ext) * 4, hipMemcpyHostToDevice, s);
        if (err == hipSuccess && w_in) err = hipMemcpyAsync(w_d, w_in + e0, w, hipMemcpyHostToDevice, s);
        if (err != hipSuccess) return drain(dev_fail(err));
        st = mgrw_reweight(p, mom_d, w_in ? w_d : nullptr, m, out_d, me_base_out ? me0_d : nullptr, s);
        if (st != MGRW_OK) return drain(st);
        err = hipMemcpy2DAsync(w_out + e0, row, out_d, w, w, size_t(P), hipMemcpyDeviceToHost, s);
        if (err == hipSuccess && me_base_out) err = hipMemcpyAsync(me_base_out + e0, me0_d, w, hipMemcpyDeviceToHost, s);
        if (err != hipSuccess) return drain(dev_fail(err));
    }
    for (int i = 0; i < 2; ++i) {
        hipError_t err = hipStreamSynchronize(h.s[i]);
        if (err != hipSuccess) return dev_fail(err);
    }
    return MGRW_OK;
}
