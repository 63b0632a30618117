// One reweight call over a sample that mixes processes, e.g. the Born
// g g -> t tbar and its real emission g g -> t tbar g (the tree-level pieces
// of an NLO sample, which the same machinery evaluates: Sec. 4).  Each
// event carries the index of its process; the events of every process are
// gathered into a contiguous batch, reweighted by that process's kernels and
// their results scattered back to the events' places.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/mgrw.h"
#include "mgrw_internal.h"

namespace {

constexpr int kMultiBlock = 256;
constexpr int kMaxProcs = 8;

__global__ void __launch_bounds__(kMultiBlock)
count_kernel(const int32_t* __restrict__ idx, int64_t n, int n_procs, unsigned long long* __restrict__ counts) {
    const int64_t e = int64_t(blockIdx.x) * kMultiBlock + threadIdx.x;
    if (e >= n) return;
    const int p = idx[e];
    // counts[n_procs] collects indices out of range
    atomicAdd(&counts[(p >= 0 && p < n_procs) ? p : n_procs], 1ull);
}

// Events of process p: momenta rows 0..n_ext-1, input weight and origin.
__global__ void __launch_bounds__(kMultiBlock)
gather_kernel(const double* __restrict__ mom, const int32_t* __restrict__ idx, const double* __restrict__ w_in,
              int64_t n, int p, int n_ext, int64_t np, unsigned long long* __restrict__ fill,
              double* __restrict__ mom_p, double* __restrict__ w_p, int64_t* __restrict__ origin) {
    const int64_t e = int64_t(blockIdx.x) * kMultiBlock + threadIdx.x;
    if (e >= n || idx[e] != p) return;
    const int64_t k = int64_t(atomicAdd(fill, 1ull));
    if (k >= np) return;   // cannot happen: np is this process's count
    for (int r = 0; r < n_ext * 4; ++r) mom_p[int64_t(r) * np + k] = mom[int64_t(r) * n + e];
    if (w_p) w_p[k] = w_in[e];
    origin[k] = e;
}

__global__ void __launch_bounds__(kMultiBlock)
scatter_kernel(const double* __restrict__ out_p, const double* __restrict__ me0_p, const int64_t* __restrict__ origin,
               int64_t np, int64_t n, int n_points, double* __restrict__ out, double* __restrict__ me0) {
    const int64_t k = int64_t(blockIdx.x) * kMultiBlock + threadIdx.x;
    if (k >= np) return;
    const int64_t e = origin[k];
    for (int q = 0; q < n_points; ++q) out[int64_t(q) * n + e] = out_p[int64_t(q) * np + k];
    if (me0) me0[e] = me0_p[k];
}

__global__ void zero_kernel(unsigned long long* c, int m) {
    if (int(threadIdx.x) < m) c[threadIdx.x] = 0;
}

unsigned grid(int64_t n) { return unsigned((n + kMultiBlock - 1) / kMultiBlock); }

// Arrays the kernels here touch directly must be device memory.
bool on_device(const void* ptr) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

}  // namespace

extern "C" mgrw_status mgrw_multi_reweight(mgrw_process* const* procs, int n_procs, const double* mom, int n_ext_max,
                                           const int32_t* proc_index, const double* w_in, int64_t n_events,
                                           double* w_out, double* me_base_out, void* stream) {
    using mgrw::set_error;
    if (!procs || n_procs < 1 || n_procs > kMaxProcs) return set_error(MGRW_ERR_ARG, "need 1..8 processes");
    if (n_events < 0) return set_error(MGRW_ERR_ARG, "n_events < 0");
    if (!mom || !proc_index || !w_out) return set_error(MGRW_ERR_ARG, "mom, proc_index or w_out is NULL");
    int n_points = -1;
    std::vector<int> n_ext(static_cast<size_t>(n_procs));
    for (int p = 0; p < n_procs; ++p) {
        if (!procs[p]) return set_error(MGRW_ERR_ARG, "process is NULL");
        if (procs[p]->n_points == 0) return set_error(MGRW_ERR_STATE, "no parameter points set");
        if (n_points >= 0 && procs[p]->n_points != n_points)
            return set_error(MGRW_ERR_ARG, "every process needs the same number of parameter points");
        n_points = procs[p]->n_points;
        int fl, nh, nd;
        mgrw_status st = mgrw_process_info(procs[p], &n_ext[size_t(p)], &fl, &nh, &nd);
        if (st != MGRW_OK) return st;
        if (n_ext[size_t(p)] > n_ext_max) return set_error(MGRW_ERR_ARG, "n_ext_max smaller than a process's");
    }
    if (n_events == 0) return MGRW_OK;
    if ((n_events + kMultiBlock - 1) / kMultiBlock > 0x7fffffffLL) return set_error(MGRW_ERR_ARG, "n_events too large");
    if (!on_device(mom) || !on_device(proc_index) || !on_device(w_out) || (w_in && !on_device(w_in)) ||
        (me_base_out && !on_device(me_base_out)))
        return set_error(MGRW_ERR_ARG, "mom, proc_index, w_in, w_out and me_base_out must be device memory");
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto dev_fail = [](hipError_t err) {
        return set_error(MGRW_ERR_DEVICE, std::string("multi-process reweight: ") + hipGetErrorString(err));
    };
    // per-process counts (the call synchronises once to size the batches)
    unsigned long long* counts = nullptr;
    hipError_t err = hipMallocAsync(reinterpret_cast<void**>(&counts), sizeof(unsigned long long) * 2 * (kMaxProcs + 1), s);
    if (err != hipSuccess) return dev_fail(err);
    unsigned long long* fill = counts + kMaxProcs + 1;
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, counts, 2 * (kMaxProcs + 1));
    err = hipGetLastError();
    if (err == hipSuccess) {
        hipLaunchKernelGGL(count_kernel, dim3(grid(n_events)), dim3(kMultiBlock), 0, s, proc_index, n_events, n_procs,
                           counts);
        err = hipGetLastError();
    }
    unsigned long long h_counts[kMaxProcs + 1] = {};
    if (err == hipSuccess) err = hipMemcpyAsync(h_counts, counts, sizeof h_counts, hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) {
        (void)hipFreeAsync(counts, s);
        return dev_fail(err);
    }
    if (h_counts[n_procs] != 0) {
        (void)hipFreeAsync(counts, s);
        return set_error(MGRW_ERR_ARG, "proc_index holds values outside [0, n_procs)");
    }
    mgrw_status result = MGRW_OK;
    for (int p = 0; p < n_procs && result == MGRW_OK; ++p) {
        const int64_t np = int64_t(h_counts[p]);
        if (np == 0) continue;
        const int ne = n_ext[size_t(p)];
        // one allocation: momenta, weights, outputs, base |M|^2, origins
        const size_t doubles = size_t(np) * (size_t(ne) * 4 + 1 + size_t(n_points) + 1);
        double* buf = nullptr;
        err = hipMallocAsync(reinterpret_cast<void**>(&buf), sizeof(double) * doubles + sizeof(int64_t) * size_t(np), s);
        if (err != hipSuccess) {
            result = dev_fail(err);
            break;
        }
        double* mom_p = buf;
        double* w_p = mom_p + size_t(np) * ne * 4;
        double* out_p = w_p + np;
        double* me0_p = out_p + size_t(np) * n_points;
        int64_t* origin = reinterpret_cast<int64_t*>(me0_p + np);
        hipLaunchKernelGGL(gather_kernel, dim3(grid(n_events)), dim3(kMultiBlock), 0, s, mom, proc_index, w_in,
                           n_events, p, ne, np, fill + p, mom_p, w_in ? w_p : nullptr, origin);
        err = hipGetLastError();
        if (err != hipSuccess) {
            result = dev_fail(err);
        } else {
            result = mgrw_reweight(procs[p], mom_p, w_in ? w_p : nullptr, np, out_p, me0_p, stream);
            if (result == MGRW_OK) {
                hipLaunchKernelGGL(scatter_kernel, dim3(grid(np)), dim3(kMultiBlock), 0, s, out_p, me0_p, origin, np,
                                   n_events, n_points, w_out, me_base_out);
                err = hipGetLastError();
                if (err != hipSuccess) result = dev_fail(err);
            }
        }
        (void)hipFreeAsync(buf, s);
    }
    err = hipFreeAsync(counts, s);
    if (result == MGRW_OK && err != hipSuccess) return dev_fail(err);
    return result;
}
