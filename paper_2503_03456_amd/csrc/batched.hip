// Batched entry point and selector state.
//
// sylv_solve_batched currently runs the equations one after another through
// the single-equation path (each equation on the caller's stream).
#include "common.hpp"
#include "kernels.hpp"
#include "../../include/sylv.h"

#include <vector>
#include <cstring>
#include <mutex>

static std::mutex g_sel_mu;
static std::vector<float> g_selector;  // 5443 params + 16 means + 16 stds

extern "C" int sylv_solve_batched(int batch, const int *kind, const int *m, const int *n,
                                  const double *const *A, const int *lda, const double *const *B,
                                  const int *ldb, const double *const *C, const int *ldc,
                                  double *const *X, const int *ldx, const sylv_opts *opts,
                                  sylv_info *infos, void *work, size_t work_bytes, void *stream) {
    if (batch < 0) return -1;
    if (batch == 0) return 0;
    if (!kind) return -2;
    if (!m) return -3;
    if (!n) return -4;
    if (!A) return -5;
    if (!lda) return -6;
    if (!C) return -9;
    if (!ldc) return -10;
    if (!X) return -11;
    if (!ldx) return -12;
    for (int i = 0; i < batch; ++i)
        if (kind[i] == SYLV_KIND_SYLV && (!B || !ldb)) return -7;
    for (int i = 0; i < batch; ++i) {
        int rc;
        sylv_info *inf = infos ? infos + i : nullptr;
        if (kind[i] == SYLV_KIND_LYAP)
            rc = lyap_solve(m[i], A[i], lda[i], C[i], ldc[i], X[i], ldx[i], opts, inf, work, work_bytes,
                            stream);
        else
            rc = sylv_solve(m[i], n[i], A[i], lda[i], B[i], ldb[i], C[i], ldc[i], X[i], ldx[i], opts,
                            inf, work, work_bytes, stream);
        if (rc) return rc;
    }
    return 0;
}

extern "C" int sylv_selector_set(const float *blob, int nvalues) {
    if (!blob) return -1;
    if (nvalues != SYLV_MLP_NPARAM + 2 * SYLV_NFEAT) return -2;
    std::lock_guard<std::mutex> lk(g_sel_mu);
    g_selector.assign(blob, blob + nvalues);
    return 0;
}

extern "C" int sylv_selector_features(int m, int n, const double *A, int lda, const double *B, int ldb,
                                      const double *C, int ldc, float *feats, void *stream) {
    (void)m; (void)n; (void)A; (void)lda; (void)B; (void)ldb; (void)C; (void)ldc; (void)feats;
    (void)stream;
    return -1;
}
