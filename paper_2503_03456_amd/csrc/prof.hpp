// Optional per-kernel timing with HIP events on the launch stream.
// sylv_profile_begin(id) arms one kernel family; every launch of that family
// is then bracketed by a pair of events; sylv_profile_end() synchronises and
// returns the launch count and the summed durations.
#pragma once
#include <hip/hip_runtime.h>

namespace sylv {

enum KernelId {
    KID_NONE = 0, KID_GEMM = 1, KID_HESS_COL = 2, KID_HESS_GEMV = 3, KID_AED = 4, KID_CHASE = 5,
    KID_TRSYL = 6, KID_FIND_KTOP = 7, KID_CAST = 8, KID_NORM = 9, KID_BHESS = 10,
    KID_BSCHUR = 11, KID_BTRSYL = 12, KID_BGEMM = 13, KID_JAC_PAIRS = 14, KID_JAC_APPLY = 15,
    KID_WIN = 16, KID_COUNT = 17
};

bool prof_armed(int id);
bool prof_any_armed();
void prof_begin(int id, hipStream_t s);
void prof_end(int id, hipStream_t s);
// algorithmic work (flops or bytes) of the armed kernel family, summed over launches
void prof_add_work(int id, double work);

// RAII bracket around one launch
struct ProfScope {
    int id;
    hipStream_t s;
    bool on;
    ProfScope(int id_, hipStream_t s_) : id(id_), s(s_), on(prof_armed(id_)) {
        if (on) prof_begin(id, s);
    }
    ~ProfScope() {
        if (on) prof_end(id, s);
    }
};

}  // namespace sylv
