// qs_profile.hip -- per-kernel timing with HIP events stamped by the kernel dispatch itself
// (qed_profile_start / qed_profile_stop).
// Single-threaded host use: the event records live in one process-wide list.
#include <string.h>

#include <vector>

#include "qs_internal.hpp"

bool g_qs_profiling = false;

namespace {
struct Rec {
    int kid;
    hipEvent_t a, b;
};
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

const char *const kNames[K_NKERNELS] = {"table_build", "push",       "lepton_main", "emit_process", "photon_main",
                                        "pair_process", "expand",    "clock",       "alive_mask",   "gather",
                                        "scatter_back", "plan_lepton", "plan_photon", "plan_process",
                                        "grid_pack", "plan_sub"};

hipEvent_t take()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

void qs_prof_events(int kid, hipEvent_t *start, hipEvent_t *stop)
{
    hipEvent_t a = take(), b = a ? take() : nullptr;
    if (!b) {
        if (a) g_pool.push_back(a);
        *start = *stop = nullptr;                // launched untimed
        return;
    }
    g_recs.push_back({kid, a, b});
    *start = a;
    *stop = b;
}

extern "C" qed_status qed_profile_start(void)
{
    for (Rec &r : g_recs) {
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    g_qs_profiling = true;
    return QED_OK;
}

extern "C" qed_status qed_profile_stop(qed_kernel_time *out, int max_entries, int *n_entries)
{
    g_qs_profiling = false;
    double ms[K_NKERNELS] = {0};
    long long calls[K_NKERNELS] = {0};
    for (Rec &r : g_recs) {
        QS_CHECK(hipEventSynchronize(r.b));
        float t = 0.0f;
        QS_CHECK(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.kid] += t;
        calls[r.kid] += 1;
    }
    int n = 0;
    for (int k = 0; k < K_NKERNELS; ++k) {
        if (!calls[k]) continue;
        if (out && n < max_entries) {
            out[n].name = kNames[k];
            out[n].calls = calls[k];
            out[n].total_ms = ms[k];
        }
        ++n;
    }
    if (n_entries) *n_entries = n;
    return QED_OK;
}
