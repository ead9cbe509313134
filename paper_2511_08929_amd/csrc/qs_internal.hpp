// qs_internal.hpp -- host-side internals shared by the table builder and the step kernels.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "../../include/qedspin.h"
#include "qs_device.hpp"

// Device view of the tables: FP64 rate and inverse-CDF tables for the four channels
// (0 = NLC s_beta=-1, 1 = NLC s_beta=+1, 2 = NBW xi3=-1, 3 = NBW xi3=+1) and an FP32 copy
// of the rate tables for the single-precision path.
struct TablesDev {
    int n_chi[2];
    double lnchi0[2], dlnchi[2];
    int n_rho;
    double rho0, drho;
    const double *lnrate;     // [sum n_chi(channel)]
    const float *lnrate32;
    const double *nu;         // [sum n_chi(channel) * n_rho]
    const double *bn64;       // trapezoid nodes of the Bessel functions, FP64 levels
    const float *bn32;        // FP32 levels
    const double *lng;        // [kGfN] ln(a(chi)/a(0)) of the field-dependent anomalous moment
    const float *lng32;
    int off_rate[4];
    int64_t off_nu[4];
};

struct qed_tables_s {
    qed_table_params params;
    TablesDev dev;
    double *d_lnrate;
    float *d_lnrate32;
    double *d_nu;
    double *d_bn64;
    float *d_bn32;
    double *d_lng;
    float *d_lng32;
    int64_t n_rate, n_nu;
};

// Record the error text of a failed HIP call for qed_last_error() and map it to QED_ERR_HIP.
qed_status qs_fail(hipError_t e, const char *where);
// Record the text of a rejected call (a status other than QED_ERR_HIP) for qed_last_error().
qed_status qs_reject(qed_status st, const char *msg);
// Clear a stale error left in HIP's per-thread last-error slot by earlier, unrelated calls.
inline void qs_clear_error() { (void)hipGetLastError(); }
// Status after a sequence of launches.
inline qed_status qs_launch_status(const char *where)
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? QED_OK : qs_fail(e, where);
}

#define QS_CHECK(expr)                                   \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return qs_fail(e_, #expr); \
    } while (0)

// ---------------------------------------------------------------- kernel timing
// With profiling on (qed_profile_start), every launch goes through hipExtLaunchKernelGGL with a
// start and a stop event, which the runtime stamps with the begin and end of the kernel's own
// dispatch (the interval a kernel trace reports; events recorded around the launch would also
// take in the dispatch latency, ~2 us); qed_profile_stop synchronizes and reports per-kernel
// calls and time.
enum QsKernel {
    K_TABLES = 0, K_PUSH, K_LEPTON_MAIN, K_EMIT_PROCESS, K_PHOTON_MAIN, K_PAIR_PROCESS, K_MASK_EXPAND, K_SET_PREV,
    K_ALIVE_MASK, K_GATHER, K_SCATTER_BACK, K_PLAN_LEPTON, K_PLAN_PHOTON, K_PLAN_PROCESS, K_GRID_PACK, K_PLAN_SUB, K_NKERNELS
};
extern bool g_qs_profiling;
// a start and a stop event for one launch of kernel kid (both null if none could be made)
void qs_prof_events(int kid, hipEvent_t *start, hipEvent_t *stop);

#define QS_LAUNCH(kid, kernel, grid, block, lds, stream, ...)                                     \
    do {                                                                                         \
        if (g_qs_profiling) {                                                                    \
            hipEvent_t a_, b_;                                                                   \
            qs_prof_events(kid, &a_, &b_);                                                       \
            hipExtLaunchKernelGGL(kernel, grid, block, lds, stream, a_, b_, 0, __VA_ARGS__);     \
        } else {                                                                                 \
            hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);                   \
        }                                                                                        \
    } while (0)
