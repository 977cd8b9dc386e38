// Batched entry point and selector state.
//
// Lyapunov equations of order 1..256 with a binary32 low precision (binary32,
// or bfloat16 / binary16 operands in the transforms) run
// through the batched kernels (one workgroup per equation and stage, all
// equations in flight together, longest first); an equation whose
// refinement does not reach the tolerance is re-solved in binary64 when the
// options allow the fallback.  Every other equation goes through the
// single-equation path one after another.
#include "common.hpp"
#include "kernels.hpp"
#include "../../include/sylv.h"

#include <algorithm>
#include <vector>
#include <cstring>
#include <mutex>
#include <thread>

namespace sylv {
int lyap_batched(hipStream_t s, int batch, const int *nn, const double *const *A, const int *lda,
                 const double *const *C, const int *ldc, double *const *X, const int *ldx,
                 const sylv_opts &o, sylv_info *infos, void *work, size_t work_bytes, char *hbuf);
}
using namespace sylv;

static size_t pool_slice(size_t bytes) { return (bytes + 4095) & ~(size_t)4095; }

// One single-equation solve of a batched call (a binary64 re-solve, a
// selector class-2 equation, or an equation outside the batched kernels).
struct SingleJob {
    int i;             // equation index
    sylv_opts o;       // options of this solve
    sylv_info prev;    // batched result it follows (fell_back / chosen bookkeeping)
    int kind;          // 0 plain, 1 fallback after the batched pass, 2 selector class 2
};

// Runs the jobs on the pooled contexts from up to kSolvePool host threads.
// With a caller workspace of at least kSolvePool slices each thread takes one
// slice; a smaller caller workspace runs the jobs one after another in it;
// without one every pooled context keeps its own.
static int run_single_jobs(const std::vector<SingleJob> &jobs, const int *kind, const int *m, const int *n,
                           const double *const *A, const int *lda, const double *const *B, const int *ldb,
                           const double *const *C, const int *ldc, double *const *X, const int *ldx,
                           sylv_info *infos, void *work, size_t work_bytes) {
    if (jobs.empty()) return 0;
    size_t single = 0;
    for (const SingleJob &j : jobs) {
        const int lyap = kind[j.i] == SYLV_KIND_LYAP;
        single = std::max(single, sylv_workspace_size(m[j.i], lyap ? m[j.i] : n[j.i], lyap, &j.o));
    }
    const size_t slice = pool_slice(single);
    int threads = std::min<int>(kSolvePool, (int)jobs.size());
    if (work && work_bytes < slice * threads) threads = 1;
    std::vector<int> rcs(threads, 0);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SYLV_ERR_NOGPU;
    auto worker = [&](int t) {
        hipSetDevice(dev);
        void *w = work ? (char *)work + (threads > 1 ? slice * t : 0) : nullptr;
        const size_t wb = work ? (threads > 1 ? slice : work_bytes) : 0;
        for (size_t k = t; k < jobs.size(); k += threads) {
            const SingleJob &j = jobs[k];
            const int i = j.i;
            const bool lyap = kind[i] == SYLV_KIND_LYAP;
            sylv_info g;
            const int rc = solve_pooled(t, m[i], n[i], A[i], lda[i], lyap ? nullptr : B[i], lyap ? 1 : ldb[i],
                                        C[i], ldc[i], X[i], ldx[i], &j.o, &g, w, wb);
            if (rc) { rcs[t] = rc; return; }
            if (j.kind == 2) {
                g.chosen = 2;
                g.orth_u = j.prev.orth_u;
                g.orth_v = j.prev.orth_v;
            } else if (j.kind == 1) {
                g.fell_back = 1;
                g.iterations += j.prev.iterations;
                g.chosen = j.prev.chosen;
            }
            if (infos) infos[i] = g;
        }
    };
    if (threads == 1) worker(0);
    else {
        std::vector<std::thread> pool;
        for (int t = 0; t < threads; ++t) pool.emplace_back(worker, t);
        for (auto &th : pool) th.join();
    }
    for (int rc : rcs)
        if (rc) return rc;
    return 0;
}

static bool batched_eligible(int kind, int n, const sylv_opts &o) {
    return kind == SYLV_KIND_LYAP && n >= 1 && n <= 256 && o.alg == SYLV_ALG_ORIG &&
           (o.low == SYLV_PREC_FP32 || o.low == SYLV_PREC_BF16 || o.low == SYLV_PREC_FP16 ||
            (o.low == SYLV_PREC_AUTO && selector_installed()));
}

extern "C" size_t sylv_batched_workspace_size(int batch, const int *kind, const int *m, const int *n,
                                              const sylv_opts *opts) {
    if (batch < 0 || (batch > 0 && (!kind || !m || !n))) return 0;
    sylv_opts o;
    sylv_default_opts(&o);
    if (opts) o = *opts;
    std::vector<int> nb;
    size_t single = 0;
    for (int i = 0; i < batch; ++i) {
        if (batched_eligible(kind[i], m[i], o)) {
            nb.push_back(m[i]);
            if (o.fallback || o.low == SYLV_PREC_AUTO) {
                // binary64 re-solves: fallback, or the selector's class 2
                sylv_opts f = o;
                f.low = SYLV_PREC_FP64;
                single = std::max(single, sylv_workspace_size(m[i], m[i], 1, &f));
            }
        } else {
            const int lyap = kind[i] == SYLV_KIND_LYAP;
            single = std::max(single, sylv_workspace_size(m[i], lyap ? m[i] : n[i], lyap, &o));
        }
    }
    const size_t b = nb.empty() ? 0 : lyap_batched_bytes((int)nb.size(), nb.data());
    // single-equation solves run side by side, one workspace slice each
    return std::max(b, pool_slice(single) * kSolvePool);
}

static int solve_batched_impl(int batch, const int *kind, const int *m, const int *n,
                              const double *const *A, const int *lda, const double *const *B,
                              const int *ldb, const double *const *C, const int *ldc,
                              double *const *X, const int *ldx, const sylv_opts *opts,
                              sylv_info *infos, void *work, size_t work_bytes, void *stream);

extern "C" int sylv_solve_batched(int batch, const int *kind, const int *m, const int *n,
                                  const double *const *A, const int *lda, const double *const *B,
                                  const int *ldb, const double *const *C, const int *ldc,
                                  double *const *X, const int *ldx, const sylv_opts *opts,
                                  sylv_info *infos, void *work, size_t work_bytes, void *stream) {
    if (batch <= 0) return batch < 0 ? -1 : 0;
    InfoSink sink(infos, batch);
    const int rc = solve_batched_impl(batch, kind, m, n, A, lda, B, ldb, C, ldc, X, ldx, opts, sink.host(), work,
                                      work_bytes, stream);
    return sink.finish(rc, (hipStream_t)stream);
}

static int solve_batched_impl(int batch, const int *kind, const int *m, const int *n,
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
    sylv_opts o;
    sylv_default_opts(&o);
    if (opts) o = *opts;
    if (!(o.tol >= 0.0) || o.max_iter < 0) return -13;
    hipStream_t s = (hipStream_t)stream;
    if (const int cap = stream_capture_code(s, work == nullptr)) return cap;

    std::vector<SingleJob> jobs;
    // equations for the batched kernels (validated like the single path)
    std::vector<int> idx, bn, blda, bldc, bldx;
    std::vector<const double *> bA, bC;
    std::vector<double *> bX;
    for (int i = 0; i < batch; ++i) {
        if (!batched_eligible(kind[i], m[i], o)) continue;
        if (lda[i] < m[i] || ldc[i] < m[i] || ldx[i] < m[i]) return -6;
        if (!A[i] || !C[i] || !X[i]) return -5;
        idx.push_back(i);
        bn.push_back(m[i]);
        bA.push_back(A[i]); blda.push_back(lda[i]);
        bC.push_back(C[i]); bldc.push_back(ldc[i]);
        bX.push_back(X[i]); bldx.push_back(ldx[i]);
    }
    if (!idx.empty()) {
        const int nb = (int)idx.size();
        std::vector<sylv_info> binf(nb);
        int rc;
        {
            std::lock_guard<std::mutex> lk(lib_mutex());
            const size_t need = lyap_batched_bytes(nb, bn.data());
            void *ws = nullptr;
            char *hbuf = nullptr;
            rc = device_work(work ? 0 : need, &ws, &hbuf);
            if (rc) return rc;
            if (work) {
                if (work_bytes < need) return -15;
                ws = work;
            }
            rc = lyap_batched(s, nb, bn.data(), bA.data(), blda.data(), bC.data(), bldc.data(),
                              bX.data(), bldx.data(), o, binf.data(), ws, work ? work_bytes : need, hbuf);
            hipError_t e = hipGetLastError();
            if (rc == 0 && e != hipSuccess) rc = SYLV_ERR_HIP - (int)e;
        }
        if (rc) return rc;
        for (int t = 0; t < nb; ++t) {
            const int i = idx[t];
            const sylv_info &f = binf[t];
            if (o.low == SYLV_PREC_AUTO && f.chosen == 2) {
                // the selector sent the equation to the plain binary64 path
                sylv_opts f64 = o;
                f64.low = SYLV_PREC_FP64;
                jobs.push_back({i, f64, f, 2});
                continue;
            }
            const bool ok = f.status == SYLV_OK || f.status == SYLV_ST_PERTURBED;
            if (!ok && o.fallback) {
                // next rung of the ladder: bfloat16 / binary16 updates ->
                // binary32 (which itself falls back to binary64); binary32 ->
                // binary64
                sylv_opts f64 = o;
                const bool narrow = o.low == SYLV_PREC_BF16 || o.low == SYLV_PREC_FP16 ||
                                    (o.low == SYLV_PREC_AUTO && f.chosen == 0);
                f64.low = narrow ? SYLV_PREC_FP32 : SYLV_PREC_FP64;
                jobs.push_back({i, f64, f, 1});
                continue;
            }
            if (infos) infos[i] = f;
        }
    }
    for (int i = 0; i < batch; ++i) {
        if (batched_eligible(kind[i], m[i], o)) continue;
        jobs.push_back({i, o, sylv_info{}, 0});
    }
    // the single solves run on the pooled contexts' own streams: finish the
    // caller's stream first (its earlier work may produce their inputs)
    if (!jobs.empty()) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    }
    return run_single_jobs(jobs, kind, m, n, A, lda, B, ldb, C, ldc, X, ldx, infos, work, work_bytes);
}

extern "C" int sylv_batched_tune(int hess_hi, int hess_lo, int band1, int band2, int band3, int graph_passes) {
    const int band[3] = {band1, band2, band3};
    return batch_tune_set(hess_hi, hess_lo, band, graph_passes);
}

extern "C" int sylv_batched_tune_get(int *vals) {
    if (!vals) return -1;
    batch_tune_get(vals);
    return 0;
}
