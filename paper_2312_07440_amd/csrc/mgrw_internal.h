// Internal declarations shared by the translation units of libmgrw.
#pragma once

#include <string>

#include <hip/hip_runtime.h>

#include "../../include/mgrw.h"

namespace mgrw {
struct surrogate;                       // MLP state (mgrw_mlp.hip)
void surrogate_destroy(surrogate* s);
struct host_pipeline;                   // streams and staging of mgrw_reweight_host (mgrw_stream.hip)
void host_pipeline_destroy(host_pipeline* h);
mgrw_status set_error(mgrw_status code, const std::string& msg);
// MGRW_OK if ptr is device (or managed) memory, or NULL with allow_null;
// else MGRW_ERR_ARG naming `what`.
mgrw_status check_device_ptr(const void* ptr, const char* what, bool allow_null);
}  // namespace mgrw

struct mgrw_process {
    int proc;
    int prec;
    mgrw_params base;
    mgrw_params points[MGRW_MAX_POINTS];
    int n_points;
    int mapping;                        // MGRW_MAP_*
    double rescue_tau;                  // FP64 rescue threshold on |2 p_i.p_j|/s (0: off)
    mgrw::surrogate* sur;               // null until trained or loaded
    hipEvent_t t0, t1;                  // amplitude-kernel timestamps (timing option), else null
    int timed;                          // a launch has recorded t0/t1
    int colour_mfma;                    // g g -> t tbar g g g: colour sum on the matrix cores
    mgrw::host_pipeline* hp;            // null until mgrw_reweight_host is first called
    int sur_inputs;                     // surrogate input features: 53 (with pair invariants) or 25
};
