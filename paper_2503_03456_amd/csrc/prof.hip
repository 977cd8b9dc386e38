// Per-kernel event timing (see prof.hpp).
#include "prof.hpp"
#include "../../include/sylv.h"

#include <atomic>
#include <mutex>
#include <vector>

namespace sylv {

static std::atomic<int> g_target{KID_NONE};
static std::mutex g_pmu;
static std::vector<hipEvent_t> g_pool;   // free events
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_live;
static thread_local hipEvent_t g_open = nullptr;
static double g_work = 0.0;

bool prof_armed(int id) { return g_target.load(std::memory_order_relaxed) == id; }
bool prof_any_armed() { return g_target.load(std::memory_order_relaxed) != KID_NONE; }

static hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}

void prof_begin(int id, hipStream_t s) {
    (void)id;
    std::lock_guard<std::mutex> lk(g_pmu);
    g_open = take_event();
    hipEventRecord(g_open, s);
}

void prof_add_work(int id, double work) {
    if (!prof_armed(id)) return;
    std::lock_guard<std::mutex> lk(g_pmu);
    g_work += work;
}

void prof_end(int id, hipStream_t s) {
    (void)id;
    std::lock_guard<std::mutex> lk(g_pmu);
    hipEvent_t e = take_event();
    hipEventRecord(e, s);
    g_live.push_back({g_open, e});
    g_open = nullptr;
}

}  // namespace sylv

using namespace sylv;

extern "C" int sylv_profile_begin(int kernel_id) {
    if (kernel_id < 0 || kernel_id >= KID_COUNT) return -1;
    std::lock_guard<std::mutex> lk(g_pmu);
    for (auto &p : g_live) { g_pool.push_back(p.first); g_pool.push_back(p.second); }
    g_live.clear();
    g_work = 0.0;
    g_target.store(kernel_id);
    return 0;
}

extern "C" int sylv_profile_end(long *launches, double *total_ms, double *work) {
    g_target.store(KID_NONE);
    std::lock_guard<std::mutex> lk(g_pmu);
    double tot = 0.0;
    for (auto &p : g_live) {
        hipEventSynchronize(p.second);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) tot += ms;
        g_pool.push_back(p.first);
        g_pool.push_back(p.second);
    }
    if (launches) *launches = (long)g_live.size();
    if (total_ms) *total_ms = tot;
    if (work) *work = g_work;
    g_live.clear();
    return 0;
}

extern "C" const char *sylv_kernel_name(int kernel_id) {
    static const char *names[KID_COUNT] = {"none", "gemm_kernel", "k_hess_col", "k_hess_gemv",
                                           "k_aed", "k_chase", "k_trsyl_diag", "k_find_ktop",
                                           "k_cast", "k_sumsq_partial", "k_bhess", "k_bschur",
                                           "k_btrsyl", "gemm_batched_kernel", "k_jac_pairs",
                                           "k_jac_apply", "k_win_update"};
    if (kernel_id < 0 || kernel_id >= KID_COUNT) return "unknown";
    return names[kernel_id];
}
