// qs_internal.hpp -- host-side internals shared by the table builder and the step kernels.
#pragma once
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
    int off_rate[4];
    int64_t off_nu[4];
};

struct qed_tables_s {
    qed_table_params params;
    TablesDev dev;
    double *d_lnrate;
    float *d_lnrate32;
    double *d_nu;
    int64_t n_rate, n_nu;
};

#define QS_CHECK(expr)                                 \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return QED_ERR_HIP;      \
    } while (0)
