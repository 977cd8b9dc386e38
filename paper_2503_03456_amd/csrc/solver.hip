// Solver orchestration and the C ABI of libsylv.so.
//
// sylv_solve / lyap_solve run, on one GPU:
//   low precision (binary32):  Schur(A), Schur(B) -> first iterate by the
//       Bartels-Stewart transform / tri-solve / back-transform (Sec. 2.2.1);
//   refinement (Alg. 3.1 in the original basis): R = C - AX - XB in binary64
//       against the original coefficients, correction D from the binary32
//       Schur factors (U^T R V -> tri-solve -> U D V^T), X += D in binary64,
//       until the relative residual of eq. (2.1) is below tol;
//   fallback / baseline: the same stages instantiated in binary64 (plain
//       Bartels-Stewart).
// Lyapunov (eq. (1.3), real): one Schur form A = U T U^T; the right
// coefficient T^T is lower quasi-triangular, so the tri-solve is run on the
// equivalent upper form T Y' + Y' (P T^T P) = C~ P with P the reversal
// permutation, i.e. with V = U P.
#include "common.hpp"
#include "kernels.hpp"
#include "schur.hpp"
#include "../../include/sylv.h"

#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>
#include <new>
#include <vector>
#include <algorithm>

namespace sylv {

// ------------------------------------------------------------ device context
struct DevCtx {
    bool ok = false;
    bool checked = false;
    int dev = 0;
    char *hbuf = nullptr;       // pinned host staging, 64 KiB
    char *hbuf2 = nullptr;      // second staging buffer (concurrent Schur of B)
    hipStream_t s2 = nullptr;   // internal stream for the Schur form of B
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    void *work = nullptr;       // cached internal workspace
    size_t work_bytes = 0;
    hipStream_t own = nullptr;  // pooled contexts: the stream their solves run on
};

static std::mutex g_mu;
static DevCtx g_ctx[64];

// One-time set-up of a context on device dev (own: also a stream of its own
// for the pooled solves).
static int init_ctx(DevCtx &c, int dev, bool own) {
    if (!c.checked) {
        c.checked = true;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return SYLV_ERR_NOGPU;
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SYLV_ERR_NOGPU;
        if (hipHostMalloc((void **)&c.hbuf, 65536, hipHostMallocDefault) != hipSuccess) return SYLV_ERR_ALLOC;
        if (hipHostMalloc((void **)&c.hbuf2, 65536, hipHostMallocDefault) != hipSuccess) return SYLV_ERR_ALLOC;
        if (hipStreamCreateWithFlags(&c.s2, hipStreamNonBlocking) != hipSuccess) return SYLV_ERR_NOGPU;
        if (own && hipStreamCreateWithFlags(&c.own, hipStreamNonBlocking) != hipSuccess) return SYLV_ERR_NOGPU;
        if (hipEventCreateWithFlags(&c.ev_in, hipEventDisableTiming) != hipSuccess) return SYLV_ERR_NOGPU;
        if (hipEventCreateWithFlags(&c.ev_out, hipEventDisableTiming) != hipSuccess) return SYLV_ERR_NOGPU;
        c.dev = dev;
        c.ok = true;
    }
    return c.ok ? 0 : SYLV_ERR_NOGPU;
}

static int device_ctx(DevCtx **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SYLV_ERR_NOGPU;
    DevCtx &c = g_ctx[dev];
    const int rc = init_ctx(c, dev, false);
    if (rc) return rc;
    *out = &c;
    return 0;
}

// Pool of contexts for independent solves run side by side from several host
// threads (the binary64 re-solves and single-equation members of a batched
// call): each has its own stream, pinned staging and workspace cache, and a
// lock of its own instead of the library lock.
static DevCtx g_pool[64][kSolvePool];
static std::mutex g_pool_mu[64][kSolvePool];

static int ensure_work(DevCtx *c, size_t bytes, void **out) {
    if (c->work_bytes < bytes) {
        if (c->work) hipFree(c->work);
        c->work = nullptr;
        c->work_bytes = 0;
        if (hipMalloc(&c->work, bytes) != hipSuccess) return SYLV_ERR_ALLOC;
        c->work_bytes = bytes;
    }
    *out = c->work;
    return 0;
}

// Library lock and per-device staging/workspace for the batched entry point
// (the caller holds the lock while it uses them).
std::mutex &lib_mutex() { return g_mu; }
int device_work(size_t bytes, void **work, char **hbuf) {
    DevCtx *c = nullptr;
    int rc = device_ctx(&c);
    if (rc) return rc;
    *hbuf = c->hbuf;
    if (bytes == 0) { *work = nullptr; return 0; }
    return ensure_work(c, bytes, work);
}

// SYLV_ERR_CAPTURE_ALLOC (work == NULL) or SYLV_ERR_CAPTURE when `s` is being
// captured into a graph, else 0
int stream_capture_code(hipStream_t s, bool needs_alloc) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return 0;
    if (cs == hipStreamCaptureStatusNone) return 0;
    return needs_alloc ? SYLV_ERR_CAPTURE_ALLOC : SYLV_ERR_CAPTURE;
}

// True when p is device memory (an info array the caller keeps on the GPU);
// host memory, pinned or pageable, is written directly.  Any error the query
// leaves behind is cleared.
bool is_device_pointer(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    std::memset(&at, 0, sizeof(at));
    const hipError_t e = hipPointerGetAttributes(&at, p);
    (void)hipGetLastError();
    return e == hipSuccess && at.type == hipMemoryTypeDevice;
}

InfoSink::InfoSink(sylv_info *user, int count) : user_(user), count_(count) {
    if (user && count > 0 && is_device_pointer(user)) local_.resize((size_t)count);
}
sylv_info *InfoSink::host() { return local_.empty() ? user_ : local_.data(); }
int InfoSink::finish(int rc, hipStream_t s) {
    if (rc != 0 || local_.empty()) return rc;
    hipError_t e = hipMemcpyAsync(user_, local_.data(), sizeof(sylv_info) * local_.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? 0 : SYLV_ERR_HIP - (int)e;
}

// ----------------------------------------------------------- workspace plan
struct Arena {
    char *base;
    size_t off = 0;
    explicit Arena(void *b) : base((char *)b) {}
    template <typename T>
    T *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

template <typename T>
struct Stage {  // buffers of one precision's Bartels-Stewart pipeline
    T *TA, *UA, *TB, *UB, *W1, *Y;
    T *W2;            // Lyapunov: the symmetric second product of the forward transform
    char *schur_ws;   // Schur workspace for A
    char *schur_ws2;  // Schur workspace for B (the two run concurrently)
    int diag;         // symmetric coefficients: TA, TB diagonal (eigen-decompositions)
    int lsym;         // Lyapunov with symmetric C: symmetric iterate, half tri-solve
    T *Pinv;          // binary32: block-pair inverse rows of the tri-solve (4 m n), set by mixed_forms
    int *pflag;       // their pivot-perturbation flag
};

// Alg. 4.1 buffers (binary64): orthonormalised factors, the triangular-basis
// coefficients M = Q^T A Q (= T + L), the binary64 copies of T, F = QA^T C QB,
// the triangular-basis iterate Y, and two scratch matrices.
struct OrthStage {
    double *QA, *QB, *MA, *MB, *TA, *TB, *F, *Y, *W, *E;
    double *UA, *UB;  // Alg. 4.2: binary64 copies of the low-precision factors (QA, QB hold their inverses)
};

// random probe vectors of the orthogonality estimate
constexpr int kProbes = 8;
constexpr int kProbeSlices = 32;  // contraction slices of the probe product U Z

// Narrow operand format of the GEMM-shaped updates for a precision option:
// 0 binary32 inputs, 1 bfloat16, 2 binary16 (the code the GEMM wrappers take)
static int narrow_of(int low) {
    return low == SYLV_PREC_BF16 ? 1 : low == SYLV_PREC_FP16 ? 2 : 0;
}
static int prec_of_narrow(int nf) {
    return nf == 1 ? SYLV_PREC_BF16 : nf == 2 ? SYLV_PREC_FP16 : SYLV_PREC_FP32;
}

struct Plan {
    Stage<float> lo;
    Stage<double> hi;
    OrthStage o;
    double *R;        // m x n residual
    double *G;        // orthogonality check scratch (full: 2 max(m,n)^2, probe: 24 max(m,n))
    double *scal;     // 64 device scalars
    double *nscr;     // 512-entry reduction scratch
    int *flag;        // tri-solve perturbation flag
    float *eig;       // eigenvalue scratch for sep_est (4 * max(m,n))
};

// orth: 0 no orthogonality check, 1 probe (three n x 8 binary64 blocks),
// 2 full product (two n x n binary64 matrices)
static void plan(Arena &a, int m, int n, bool lyap, bool need_lo, bool need_hi, int orth, Plan &p,
                 bool alg41 = false) {
    const int mx = std::max(m, n);
    std::memset(&p, 0, sizeof(p));
    if (alg41) {
        const size_t mm = (size_t)m * m, nn = (size_t)n * n, mn = (size_t)m * n, xx = (size_t)mx * mx;
        p.o.QA = a.take<double>(mm);
        p.o.QB = a.take<double>(nn);
        p.o.MA = a.take<double>(mm);
        p.o.MB = a.take<double>(nn);
        p.o.TA = a.take<double>(mm);
        p.o.TB = a.take<double>(nn);
        p.o.F = a.take<double>(mn);
        p.o.Y = a.take<double>(mn);
        p.o.W = a.take<double>(std::max(xx, mn));
        p.o.E = a.take<double>(xx);
        p.o.UA = a.take<double>(mm);
        p.o.UB = a.take<double>(nn);
    }
    if (need_lo) {
        p.lo.TA = a.take<float>((size_t)m * m);
        p.lo.UA = a.take<float>((size_t)m * m);
        p.lo.TB = a.take<float>((size_t)n * n);
        p.lo.UB = a.take<float>((size_t)n * n);
        p.lo.W1 = a.take<float>((size_t)m * n);
        p.lo.Y = a.take<float>((size_t)m * n);
        if (lyap) p.lo.W2 = a.take<float>((size_t)m * n);
        p.lo.Pinv = a.take<float>((size_t)4 * m * n);
        p.lo.pflag = a.take<int>(64);
        p.lo.schur_ws = a.take<char>(std::max(schur_work_bytes<float>(m), sym_eig_work_bytes<float>(m)));
        if (!lyap)
            p.lo.schur_ws2 = a.take<char>(std::max(schur_work_bytes<float>(n), sym_eig_work_bytes<float>(n)));
    }
    if (need_hi) {
        p.hi.TA = a.take<double>((size_t)m * m);
        p.hi.UA = a.take<double>((size_t)m * m);
        p.hi.TB = a.take<double>((size_t)n * n);
        p.hi.UB = a.take<double>((size_t)n * n);
        p.hi.W1 = a.take<double>((size_t)m * n);
        p.hi.Y = a.take<double>((size_t)m * n);
        if (lyap) p.hi.W2 = a.take<double>((size_t)m * n);
        p.hi.schur_ws = a.take<char>(std::max(schur_work_bytes<double>(m), sym_eig_work_bytes<double>(m)));
        if (!lyap)
            p.hi.schur_ws2 = a.take<char>(std::max(schur_work_bytes<double>(n), sym_eig_work_bytes<double>(n)));
    }
    p.R = a.take<double>((size_t)m * n);
    if (orth == 2) p.G = a.take<double>((size_t)2 * mx * mx);
    else if (orth == 1) p.G = a.take<double>((size_t)(3 + kProbeSlices) * kProbes * mx);
    p.scal = a.take<double>(64);
    p.nscr = a.take<double>(512);
    p.flag = a.take<int>(64);
    p.eig = a.take<float>((size_t)4 * mx + 64);
}

static size_t plan_bytes(int m, int n, bool lyap, bool need_lo, bool need_hi, int orth,
                         bool alg41 = false) {
    Arena a(nullptr);
    Plan p;
    plan(a, m, n, lyap, need_lo, need_hi, orth, p, alg41);
    return a.off + 256;
}

// --------------------------------------------------------------- kernels
// eigenvalues of an upper quasi-triangular float/double matrix -> (wr, wi)
template <typename T>
__global__ void k_quasi_eigs(int n, const T *Tm, int ld, float *wr, float *wi) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        bool lower = (i > 0) && CM(Tm, i, i - 1, ld) != T(0);
        bool upper = (i + 1 < n) && CM(Tm, i + 1, i, ld) != T(0);
        if (!lower && !upper) { wr[i] = (float)CM(Tm, i, i, ld); wi[i] = 0.f; continue; }
        int k = upper ? i : i - 1;
        double a = CM(Tm, k, k, ld), b = CM(Tm, k, k + 1, ld), c = CM(Tm, k + 1, k, ld), d = CM(Tm, k + 1, k + 1, ld);
        double p = 0.5 * (a - d), disc = p * p + b * c, mid = 0.5 * (a + d);
        if (disc >= 0) { double r = sqrt(disc); wr[i] = (float)(upper ? mid + r : mid - r); wi[i] = 0.f; }
        else { double r = sqrt(-disc); wr[i] = (float)mid; wi[i] = (float)(upper ? r : -r); }
    }
}

// min and max over i, j of |lambda_i + mu_j|: per-workgroup extremes into
// part[0..nb) (min) and part[SEP_BLOCKS..SEP_BLOCKS+nb) (max), then one
// workgroup folds them (fixed order, deterministic)
constexpr int SEP_BLOCKS = 256;
__global__ __launch_bounds__(256) void k_sep_range(int m, int n, const float *wra, const float *wia,
                                                   const float *wrb, const float *wib, double *part) {
    __shared__ double rlo[256], rhi[256];
    double lo = 1e300, hi = 0.0;
    const size_t total = (size_t)m * n;
    for (size_t e = blockIdx.x * (size_t)256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const int i = (int)(e % m), j = (int)(e / m);
        const double re = (double)wra[i] + wrb[j], im = (double)wia[i] + wib[j];
        const double a = sqrt(re * re + im * im);
        lo = fmin(lo, a);
        hi = fmax(hi, a);
    }
    rlo[threadIdx.x] = lo;
    rhi[threadIdx.x] = hi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            rlo[threadIdx.x] = fmin(rlo[threadIdx.x], rlo[threadIdx.x + s]);
            rhi[threadIdx.x] = fmax(rhi[threadIdx.x], rhi[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = rlo[0];
        part[SEP_BLOCKS + blockIdx.x] = rhi[0];
    }
}

// out[0] = min of part[0..cnt), out[1] = max of part[SEP_BLOCKS..SEP_BLOCKS+cnt)
__global__ __launch_bounds__(256) void k_range_final(int cnt, const double *part, double *out) {
    __shared__ double rlo[256], rhi[256];
    double lo = 1e300, hi = 0.0;
    for (int i = threadIdx.x; i < cnt; i += 256) {
        lo = fmin(lo, part[i]);
        hi = fmax(hi, part[SEP_BLOCKS + i]);
    }
    rlo[threadIdx.x] = lo;
    rhi[threadIdx.x] = hi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            rlo[threadIdx.x] = fmin(rlo[threadIdx.x], rlo[threadIdx.x + s]);
            rhi[threadIdx.x] = fmax(rhi[threadIdx.x], rhi[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = rlo[0];
        out[1] = rhi[0];
    }
}

// -------------------------------------------------------- pipeline stages
// Lyapunov: TB = P TA^T P, UB = UA P
template <typename T>
static void lyap_right_factor(hipStream_t s, int n, Stage<T> &st) {
    transpose<T>(s, n, n, st.TA, n, st.TB, n, 1);
    revcols<T, T>(s, n, n, st.UA, n, st.UB, n, T(1));
}

// Cap on the block-Jacobi sweeps of the symmetric eigen-decomposition.
constexpr int kSymSweeps = 60;

// Schur form of A into (Tm, Um); with sym, the eigen-decomposition of the
// symmetric part of A (Tm diagonal).  *qr = 1 when the iteration cap ran out.
template <typename T>
static int schur_stage(hipStream_t s, int n, const double *A, int lda, T *Tm, T *Um, char *ws,
                       char *hbuf, int *qr, int bf16, int sym = 0) {
    if (sym) {
        sym_part<double, T>(s, n, A, lda, Tm, n);
        int sweeps = 0;
        const int rc = sym_eig<T>(s, n, Tm, n, Um, n, ws, hbuf, kSymSweeps, &sweeps);
        if (rc < 0) return rc;
        *qr = rc;
        return 0;
    }
    if (bf16 == 2) {
        // binary16 operands: A is brought to max|a_ij| in [1/2, 1) by a power
        // of two before the factorisation (exact; U unchanged, T scaled by
        // the same power, undone afterwards)
        double *mx = reinterpret_cast<double *>(ws);
        matnorm<double>(s, n, n, A, lda, mx, mx + 1, 1);
        hipError_t e = hipMemcpyAsync(hbuf, mx, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
        double amax = 0.0;
        std::memcpy(&amax, hbuf, sizeof(double));
        int ex = 0;
        std::frexp((amax > 0 && std::isfinite(amax)) ? amax : 1.0, &ex);
        cast<double, T>(s, n, n, A, lda, Tm, n, std::ldexp(1.0, -ex));
        const int rc = schur_run<T>(s, n, Tm, n, Um, n, ws, hbuf, qr, bf16);
        if (rc) return rc;
        cast<T, T>(s, n, n, Tm, n, Tm, n, (T)std::ldexp(1.0, ex));
        return 0;
    }
    cast<double, T>(s, n, n, A, lda, Tm, n, 1.0);
    return schur_run<T>(s, n, Tm, n, Um, n, ws, hbuf, qr, bf16);
}

// Schur forms of A (and of B for Sylvester).  The two factorisations are
// independent and each is a chain of latency-bound single-workgroup kernels,
// so B runs concurrently on the context's second stream, driven by a second
// host thread; the caller's stream waits for it at the end.
template <typename T>
static int schur_pair(hipStream_t s, DevCtx *c, int m, int n, const double *A, int lda,
                      const double *B, int ldb, bool lyap, Stage<T> &st, int *qa, int *qb,
                      int bf16 = 0) {
    if (lyap) {
        int rc = schur_stage<T>(s, m, A, lda, st.TA, st.UA, st.schur_ws, c->hbuf, qa, bf16, st.diag);
        if (!rc) lyap_right_factor<T>(s, m, st);
        return rc;
    }
    hipError_t e = hipEventRecord(c->ev_in, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->s2, c->ev_in, 0);
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    int rcb = 0;
    std::thread tb([&]() {
        hipSetDevice(c->dev);
        rcb = schur_stage<T>(c->s2, n, B, ldb, st.TB, st.UB, st.schur_ws2, c->hbuf2, qb, bf16, st.diag);
    });
    int rca = schur_stage<T>(s, m, A, lda, st.TA, st.UA, st.schur_ws, c->hbuf, qa, bf16, st.diag);
    tb.join();
    e = hipEventRecord(c->ev_out, c->s2);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->ev_out, 0);
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    return rca ? rca : rcb;
}


// X (binary64) <- alpha * UA * tri-solve(UA^T op(Rin) UB) * UB^T (+ X when accumulate)
// Rin is binary64 (C or the residual); bscale scales it before the cast.
// nf (binary32 stage only): narrow operand format of the four transforms,
// 1 bfloat16, 2 binary16.  With binary16 the tri-solve output Y is brought
// to max|y_ij| in [1/2, 1) by a power of two before the back-transform (one
// scalar read; yscr is a device scalar, hbuf pinned host staging), and the
// power is undone on the binary64 result.
template <typename T>
static void correction(hipStream_t s, int m, int n, Stage<T> &st, const double *Rin, int ldr,
                       double bscale, double *X, int ldx, bool accumulate, const double *maxab,
                       int *flag, int nf = 0, double *yscr = nullptr, double *nscr = nullptr,
                       char *hbuf = nullptr);

template <>
void correction<float>(hipStream_t s, int m, int n, Stage<float> &st, const double *Rin, int ldr,
                       double bscale, double *X, int ldx, bool accumulate, const double *maxab,
                       int *flag, int nf, double *yscr, double *nscr, char *hbuf) {
    gemm<float, double, float, float>(s, 1, 0, m, n, m, 1.0, st.UA, m, Rin, ldr, 0.0f, st.W1, m, bscale,
                                      nf);
    if (st.lsym) {
        // Lyapunov with a symmetric right-hand side: U^T R U is symmetric, so
        // the second product forms only the tiles on or above the diagonal
        // and Y = (U^T R U) P is read off their mirror (V = U P)
        gemm<float, float, float, float>(s, 0, 0, m, n, n, 1.0, st.W1, m, st.UA, n, 0.0f, st.W2, m, 1.0f, nf, 1);
        mirror_reverse<float>(s, m, st.W2, m, st.Y, m);
    } else {
        gemm<float, float, float, float>(s, 0, 0, m, n, n, 1.0, st.W1, m, st.UB, n, 0.0f, st.Y, m, 1.0f, nf);
    }
    if (st.diag) diag_solve<float>(s, m, n, st.TA, m, st.TB, n, st.Y, m, maxab, flag);
    else trsyl<float>(s, m, n, st.TA, m, st.TB, n, st.Y, m, maxab, flag, st.lsym, st.Pinv, st.pflag);
    double ys = 1.0;
    if (nf == 2 && yscr && nscr && hbuf) {
        matnorm<float>(s, m, n, st.Y, m, yscr, nscr, 1);
        if (hipMemcpyAsync(hbuf, yscr, sizeof(double), hipMemcpyDeviceToHost, s) == hipSuccess &&
            hipStreamSynchronize(s) == hipSuccess) {
            double ymax = 0.0;
            std::memcpy(&ymax, hbuf, sizeof(double));
            int ex = 0;
            std::frexp((ymax > 0 && std::isfinite(ymax)) ? ymax : 1.0, &ex);
            ys = std::ldexp(1.0, -ex);
        }
    }
    gemm<float, float, float, float>(s, 0, 0, m, n, m, 1.0, st.UA, m, st.Y, m, 0.0f, st.W1, m, (float)ys, nf);
    // the un-scaling powers of two are applied to the binary64 result
    // symmetric iterate: U Y V^T is symmetric, only its upper tiles are
    // formed and mirrored (X stays exactly symmetric)
    gemm<float, float, double, float>(s, 0, 1, m, n, n, 1.0 / (bscale * ys), st.W1, m, st.UB, n,
                                      accumulate ? 1.0f : 0.0f, X, ldx, 1.0f, nf, st.lsym ? 1 : 0);
    if (st.lsym) mirror_upper<double>(s, m, X, ldx);
}

template <>
void correction<double>(hipStream_t s, int m, int n, Stage<double> &st, const double *Rin, int ldr,
                        double bscale, double *X, int ldx, bool accumulate, const double *maxab,
                        int *flag, int, double *, double *, char *) {
    gemm<double, double, double, double>(s, 1, 0, m, n, m, 1.0, st.UA, m, Rin, ldr, 0.0, st.W1, m, bscale);
    if (st.lsym) {
        // symmetric U^T R U: tiles on or above the diagonal, then Y = S P
        gemm<double, double, double, double>(s, 0, 0, m, n, n, 1.0, st.W1, m, st.UA, n, 0.0, st.W2, m, 1.0, 0, 1);
        mirror_reverse<double>(s, m, st.W2, m, st.Y, m);
    } else {
        gemm<double, double, double, double>(s, 0, 0, m, n, n, 1.0, st.W1, m, st.UB, n, 0.0, st.Y, m);
    }
    if (st.diag) diag_solve<double>(s, m, n, st.TA, m, st.TB, n, st.Y, m, maxab, flag);
    else trsyl<double>(s, m, n, st.TA, m, st.TB, n, st.Y, m, maxab, flag, st.lsym);
    gemm<double, double, double, double>(s, 0, 0, m, n, m, 1.0, st.UA, m, st.Y, m, 0.0, st.W1, m);
    gemm<double, double, double, double>(s, 0, 1, m, n, n, 1.0 / bscale, st.W1, m, st.UB, n,
                                         accumulate ? 1.0 : 0.0, X, ldx, 1.0, 0, st.lsym ? 1 : 0);
    if (st.lsym) mirror_upper<double>(s, m, X, ldx);
}

// R = C - A X - X op(B); scal[slot] = ||R||_F, scal[slot+1] = max|R|, scal[slot+2] = ||X||_F.
// lsym (Lyapunov, X symmetric): X A^T = (A X)^T, one product.
static void residual(hipStream_t s, int m, int n, const double *A, int lda, const double *B, int ldb,
                     bool lyap, const double *C, int ldc, const double *X, int ldx, double *R,
                     double *scal, double *nscr, bool lsym = false) {
    if (lyap && lsym) {
        gemm<double, double, double, double>(s, 0, 0, m, n, m, -1.0, A, lda, X, ldx, 0.0, R, m);
        sym_residual(s, m, C, ldc, R, m);
    } else {
        cast<double, double>(s, m, n, C, ldc, R, m, 1.0);
        gemm<double, double, double, double>(s, 0, 0, m, n, m, -1.0, A, lda, X, ldx, 1.0, R, m);
        if (lyap) gemm<double, double, double, double>(s, 0, 1, m, n, n, -1.0, X, ldx, A, lda, 1.0, R, m);
        else gemm<double, double, double, double>(s, 0, 0, m, n, n, -1.0, X, ldx, B, ldb, 1.0, R, m);
    }
    matnorm<double>(s, m, n, R, m, scal + 0, nscr, 0);
    matnorm<double>(s, m, n, R, m, scal + 1, nscr, 1);
    matnorm<double>(s, m, n, X, ldx, scal + 2, nscr, 0);
}

static hipError_t read_scalars(hipStream_t s, DevCtx *c, const double *d, int cnt, double *h) {
    hipError_t e = hipMemcpyAsync(c->hbuf, d, sizeof(double) * cnt, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    std::memcpy(h, c->hbuf, sizeof(double) * cnt);
    return hipSuccess;
}

// ||U^T U - I||_F in binary64 for a float U (n x n)
static void orth_check(hipStream_t s, int n, const float *U, double *G, double *out, double *nscr) {
    double *Ud = G, *Gm = G + (size_t)n * n;
    cast<float, double>(s, n, n, U, n, Ud, n, 1.0f);
    gemm<double, double, double, double>(s, 1, 0, n, n, n, 1.0, Ud, n, Ud, n, 0.0, Gm, n);
    sub_identity(s, n, Gm, n);
    matnorm<double>(s, n, n, Gm, n, out, nscr, 0);
}

// Probe columns z_k (k < kProbes) with independent entries +-1/sqrt(kProbes)
// from a counter-based hash of (seed, i, k) (the splitmix64 finaliser).
__global__ void k_probe_vectors(int n, unsigned seed, double *Z) {
    const size_t total = (size_t)n * kProbes;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        unsigned long long x = ((unsigned long long)seed << 40) ^ (unsigned long long)e;
        x += 0x9e3779b97f4a7c15ull;
        x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
        x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
        x ^= x >> 31;
        Z[e] = (x & 1ull) ? 0.35355339059327373 : -0.35355339059327373;
    }
}

// Slice z of W = U Z (U: n x n binary32, Z: n x kProbes binary64, both
// ld n): Wp_z(i, p) = sum_{k in [z kc, (z + 1) kc)} U(i, k) Z(k, p), one
// thread per row i (coalesced column reads of U), Z staged 128 rows at a time
__global__ __launch_bounds__(256) void k_probe_uz(int n, int kc, const float *__restrict__ U,
                                                  const double *__restrict__ Z, double *__restrict__ Wp) {
    __shared__ double zs[128 * kProbes];
    const int z = blockIdx.y, kb = z * kc, ke = min(n, kb + kc);
    const int i = blockIdx.x * 256 + threadIdx.x;
    double acc[kProbes];
#pragma unroll
    for (int q = 0; q < kProbes; ++q) acc[q] = 0.0;
    for (int c0 = kb; c0 < ke; c0 += 128) {
        const int cl = min(128, ke - c0);
        __syncthreads();
        for (int e = threadIdx.x; e < cl * kProbes; e += 256) {
            const int k = e / kProbes, q = e % kProbes;
            zs[e] = Z[(size_t)q * n + c0 + k];
        }
        __syncthreads();
        if (i < n)
            for (int k = 0; k < cl; ++k) {
                const double u = (double)U[(size_t)(c0 + k) * n + i];
#pragma unroll
                for (int q = 0; q < kProbes; ++q) acc[q] += u * zs[k * kProbes + q];
            }
    }
    if (i < n)
#pragma unroll
        for (int q = 0; q < kProbes; ++q) Wp[((size_t)z * kProbes + q) * n + i] = acc[q];
}

// W = sum_z Wp_z in slice order (n x kProbes, ld n)
__global__ void k_probe_sum(int n, int nz, const double *__restrict__ Wp, double *__restrict__ W) {
    const size_t total = (size_t)n * kProbes;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int z = 0; z < nz; ++z) v += Wp[(size_t)z * total + e];
        W[e] = v;
    }
}

// E(j, p) = sum_i U(i, j) W(i, p) - Z(j, p): one wavefront per column j of
// U (lanes along i, a fixed shuffle tree per probe)
__global__ __launch_bounds__(256) void k_probe_utw(int n, const float *__restrict__ U, const double *__restrict__ W,
                                                   const double *__restrict__ Z, double *__restrict__ E) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
    if (j >= n) return;
    double acc[kProbes];
#pragma unroll
    for (int q = 0; q < kProbes; ++q) acc[q] = 0.0;
    const float *uc = U + (size_t)j * n;
    for (int i = l; i < n; i += 64) {
        const double u = (double)uc[i];
#pragma unroll
        for (int q = 0; q < kProbes; ++q) acc[q] += u * W[(size_t)q * n + i];
    }
#pragma unroll
    for (int q = 0; q < kProbes; ++q) {
        double v = acc[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        acc[q] = v;
    }
    if (l == 0)
#pragma unroll
        for (int q = 0; q < kProbes; ++q) E[(size_t)q * n + j] = acc[q] - Z[(size_t)q * n + j];
}

// Randomised estimate of ||U^T U - I||_F (Hutchinson's trace estimator of
// ||E||_F^2 = tr(E^T E) with E = U^T U - I): for independent random sign
// vectors z, E ||E z||^2 = ||E||_F^2, so with Z = [z_1 .. z_k] / sqrt(k) the
// value ||U^T (U Z) - Z||_F estimates ||E||_F in O(k n^2) binary64 flops
// (binary32 U entries are exact in binary64).  G holds (3 + kProbeSlices)
// kProbes n doubles: Z, W, E and the slices of U Z.
static void orth_probe(hipStream_t s, int n, const float *U, double *G, double *out, double *nscr,
                       unsigned seed) {
    double *Z = G, *W = G + (size_t)kProbes * n, *E = G + (size_t)2 * kProbes * n;
    double *Wp = G + (size_t)3 * kProbes * n;
    const int nb = (int)std::min<size_t>(1024, ((size_t)n * kProbes + 255) / 256);
    hipLaunchKernelGGL(k_probe_vectors, dim3(nb), dim3(256), 0, s, n, seed, Z);
    const int nz = std::min(kProbeSlices, (n + 15) / 16);
    const int kc = (n + nz - 1) / nz;
    const int nzs = (n + kc - 1) / kc;   // every slice non-empty
    hipLaunchKernelGGL(k_probe_uz, dim3((n + 255) / 256, nzs), dim3(256), 0, s, n, kc, U, Z, Wp);
    hipLaunchKernelGGL(k_probe_sum, dim3(nb), dim3(256), 0, s, n, nzs, Wp, W);
    hipLaunchKernelGGL(k_probe_utw, dim3((n + 3) / 4), dim3(256), 0, s, n, U, W, Z, E);
    matnorm<double>(s, n, kProbes, E, n, out, nscr, 0);
}

// out[0] = sep_est = min |lambda_i + mu_j|, out[1] = max |lambda_i + mu_j|
// (kappa_est = out[1] / out[0]); scratch: 2 * SEP_BLOCKS doubles
template <typename T>
static void sep_estimate(hipStream_t s, int m, int n, const T *TA, const T *TB, float *eig, double *out,
                         double *scratch) {
    float *wra = eig, *wia = eig + m, *wrb = eig + 2 * m, *wib = eig + 2 * m + n;
    hipLaunchKernelGGL((k_quasi_eigs<T>), dim3((m + 255) / 256), dim3(256), 0, s, m, TA, m, wra, wia);
    hipLaunchKernelGGL((k_quasi_eigs<T>), dim3((n + 255) / 256), dim3(256), 0, s, n, TB, n, wrb, wib);
    const size_t total = (size_t)m * n;
    const int nb = (int)std::min<size_t>(SEP_BLOCKS, (total + 255) / 256);
    hipLaunchKernelGGL(k_sep_range, dim3(nb), dim3(256), 0, s, m, n, wra, wia, wrb, wib, scratch);
    hipLaunchKernelGGL(k_range_final, dim3(1), dim3(256), 0, s, nb, scratch, out);
}

// --------------------------------------------------------------- drivers
struct Norms { double a, b, c, cmax; };  // ||A||_F, ||B||_F, ||C||_F, max|C_ij|

// Plain binary64 Bartels-Stewart on the GPU.  Returns ABI code; fills info.
static int run_fp64(hipStream_t s, DevCtx *c, int m, int n, const double *A, int lda, const double *B,
                    int ldb, bool lyap, const double *C, int ldc, double *X, int ldx, Plan &p,
                    const Norms &nm, sylv_info *info) {
    int qa = 0, qb = 0, rc;
    rc = schur_pair<double>(s, c, m, n, A, lda, B, ldb, lyap, p.hi, &qa, &qb);
    if (rc) return rc;
    matnorm<double>(s, m, m, p.hi.TA, m, p.scal + 10, p.nscr, 1);
    matnorm<double>(s, n, n, p.hi.TB, n, p.scal + 11, p.nscr, 1);
    // maxab = max of both (computed on device by a max-norm over the two slots)
    matnorm<double>(s, 2, 1, p.scal + 10, 2, p.scal + 12, p.nscr, 1);
    hipMemsetAsync(p.flag, 0, sizeof(int), s);
    correction<double>(s, m, n, p.hi, C, ldc, 1.0, X, ldx, false, p.scal + 12, p.flag);
    sep_estimate<double>(s, m, n, p.hi.TA, p.hi.TB, p.eig, p.scal + 13, p.nscr);
    residual(s, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p.R, p.scal, p.nscr, p.hi.lsym);
    double h[16];
    hipError_t e = read_scalars(s, c, p.scal, 16, h);
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    int flag = 0;
    hipMemcpy(&flag, p.flag, sizeof(int), hipMemcpyDeviceToHost);
    if (info) {
        info->rel_res = h[0] / (nm.c + h[2] * (nm.a + nm.b));
        info->orth_u = 0.0;
        info->orth_v = 0.0;
        info->sep_est = h[13];
        info->corr_ratio = 0.0;
        info->iterations = 0;
        info->precision_used = SYLV_PREC_FP64;
        info->status = (qa || qb) ? SYLV_ST_QR_FAILED
                       : (!(std::isfinite(info->rel_res))) ? SYLV_ST_NAN
                       : flag ? SYLV_ST_PERTURBED : SYLV_OK;
    }
    return 0;
}

// Low-precision Schur forms of A (and B): binary32, with the GEMM-shaped
// updates on bfloat16 inputs when bf16 is set; then the orthogonality check
// (orth: 1 probe estimate, 2 full product), max|T| for the tri-solve pivot
// threshold and the sep estimate.
static int mixed_forms(hipStream_t s, DevCtx *c, int m, int n, const double *A, int lda,
                       const double *B, int ldb, bool lyap, Plan &p, int bf16, int orth, int *qa,
                       int *qb) {
    *qa = *qb = 0;
    int rc = schur_pair<float>(s, c, m, n, A, lda, B, ldb, lyap, p.lo, qa, qb, bf16);
    if (rc) return rc;
    if (orth == 2) {
        orth_check(s, m, p.lo.UA, p.G, p.scal + 20, p.nscr);
        if (!lyap) orth_check(s, n, p.lo.UB, p.G, p.scal + 21, p.nscr);
    } else if (orth == 1) {
        orth_probe(s, m, p.lo.UA, p.G, p.scal + 20, p.nscr, 1u);
        if (!lyap) orth_probe(s, n, p.lo.UB, p.G, p.scal + 21, p.nscr, 2u);
    }
    matnorm<float>(s, m, m, p.lo.TA, m, p.scal + 10, p.nscr, 1);
    matnorm<float>(s, n, n, p.lo.TB, n, p.scal + 11, p.nscr, 1);
    matnorm<double>(s, 2, 1, p.scal + 10, 2, p.scal + 12, p.nscr, 1);
    sep_estimate<float>(s, m, n, p.lo.TA, p.lo.TB, p.eig, p.scal + 13, p.nscr);
    // every binary32 tri-solve with these forms reuses the block-pair inverses
    if (!p.lo.diag && p.lo.Pinv)
        trsyl_prep<float>(s, m, n, p.lo.TA, m, p.lo.TB, n, p.scal + 12, p.lo.pflag, p.lo.Pinv, p.lo.lsym);
    return 0;
}

// Power of two 2^-e with 2^(e-1) <= mx < 2^e: scaling by it brings a binary64
// array with max-abs entry mx to [1/2, 1) exactly, ahead of a low-precision
// cast (the range of binary32 and of the narrower formats, Table 2.1).
static double pow2_scale(double mx) {
    int ex = 0;
    std::frexp((mx > 0 && std::isfinite(mx)) ? mx : 1.0, &ex);
    return std::ldexp(1.0, -ex);
}

// Binary64 refinement (Alg. 3.1 in the original basis) on the forms held in
// p.lo.  *ok = 1 on convergence.
//
// Stopping rule.  The iterate is accepted once the relative residual of
// eq. (2.1) is at most tol and, in addition, the forward error it implies is
// at the level the binary64 Bartels-Stewart solution reaches (the limiting
// accuracy of Thm 3.2): with R = C - AX - XB, ||X - X*||_F <= ||R||_F / sep,
// so the relative error of X is at most
//     rel_res * (||A||_F + ||B||_F + ||C||_F / ||X||_F) / sep,
// and the target is 100 u kappa with kappa = max|l_i + m_j| / sep (u = 2^-53,
// l, m the eigenvalues of the binary32 Schur forms).  sep cancels, so the
// extra test is rel_res * (||A||_F + ||B||_F + ||C||_F / ||X||_F)
// <= 100 u max|l_i + m_j|.  Steps past tol stop when the residual no longer
// halves (it has reached its floor) or at max_iter; the result is then still
// accepted because tol holds.
static int mixed_refine(hipStream_t s, DevCtx *c, int m, int n, const double *A, int lda,
                        const double *B, int ldb, bool lyap, const double *C, int ldc, double *X,
                        int ldx, Plan &p, const Norms &nm, const sylv_opts &o, int bf16, int qa, int qb,
                        sylv_info *info, int *ok) {
    *ok = 0;
    hipMemsetAsync(p.flag, 0, sizeof(int), s);
    // first iterate: X0 = U Y V^T from the low-precision factors, C brought to
    // unit size by a power of two before the cast
    const double sc0 = pow2_scale(nm.cmax);
    correction<float>(s, m, n, p.lo, C, ldc, sc0, X, ldx, false, p.scal + 12, p.flag, bf16, p.scal + 32,
                      p.nscr, c->hbuf);
    double prev = INFINITY, rel = INFINITY, corr = 0.0;
    int it = 0, stall = 0, status = SYLV_ST_NOT_CONVERGED;
    double h[32];
    for (;;) {
        residual(s, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p.R, p.scal, p.nscr, p.lo.lsym);
        hipError_t e = read_scalars(s, c, p.scal, 32, h);
        if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
        rel = h[0] / (nm.c + h[2] * (nm.a + nm.b));
        if (!std::isfinite(rel)) { status = SYLV_ST_NAN; break; }
        const bool at_tol = rel <= o.tol;
        const double growth = nm.a + nm.b + (h[2] > 0 ? nm.c / h[2] : 0.0);
        const bool fwd_ok = rel * growth <= 100.0 * 0x1p-53 * h[14];
        if (at_tol) status = SYLV_OK;
        if (at_tol && fwd_ok) break;
        if (it >= o.max_iter) break;
        if (rel > 0.5 * prev) { if (++stall >= (at_tol ? 1 : 2)) break; } else stall = 0;
        prev = rel;
        // scale R by 2^-e so that max|R| is O(1) before the low-precision cast
        const double sc = pow2_scale(h[1]);
        correction<float>(s, m, n, p.lo, p.R, m, sc, X, ldx, true, p.scal + 12, p.flag, bf16, p.scal + 32,
                          p.nscr, c->hbuf);
        // ||D||_F ~ ||Y||_F / sc (orthogonal factors to working accuracy)
        matnorm<float>(s, m, n, p.lo.Y, m, p.scal + 30, p.nscr, 0);
        ++it;
        double hy;
        e = read_scalars(s, c, p.scal + 30, 1, &hy);
        if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
        corr = hy / sc;
    }
    int flag = 0;
    hipMemcpy(&flag, p.flag, sizeof(int), hipMemcpyDeviceToHost);
    if (qa || qb) status = (status == SYLV_OK) ? SYLV_OK : SYLV_ST_QR_FAILED;
    if (status == SYLV_OK && flag) status = SYLV_ST_PERTURBED;
    *ok = (status == SYLV_OK || status == SYLV_ST_PERTURBED) ? 1 : 0;
    if (info) {
        info->rel_res = rel;
        info->orth_u = o.orth_check ? h[20] : 0.0;
        info->orth_v = o.orth_check ? (lyap ? h[20] : h[21]) : 0.0;
        info->sep_est = h[13];
        info->corr_ratio = (h[2] > 0) ? corr / h[2] : 0.0;
        info->iterations = it;
        info->precision_used = prec_of_narrow(bf16);
        info->status = status;
    }
    return 0;
}

// binary32 factors (GEMM-shaped updates with bfloat16 inputs when o.low is
// BF16) + binary64 refinement.  *ok = 1 on convergence.
static int run_mixed(hipStream_t s, DevCtx *c, int m, int n, const double *A, int lda,
                     const double *B, int ldb, bool lyap, const double *C, int ldc, double *X,
                     int ldx, Plan &p, const Norms &nm, const sylv_opts &o, sylv_info *info,
                     int *ok) {
    *ok = 0;
    int qa = 0, qb = 0;
    const int bf16 = narrow_of(o.low);
    int rc = mixed_forms(s, c, m, n, A, lda, B, ldb, lyap, p, bf16, o.orth_check, &qa, &qb);
    if (rc) return rc;
    return mixed_refine(s, c, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p, nm, o, bf16, qa, qb, info,
                        ok);
}

// -------------------------------------------------- learned precision choice
// Spectral statistics of a quasi-triangular T with eigenvalues (wr, wi):
// out[0] = number of eigenvalues in complex pairs, out[1] = squared Frobenius
// norm of the block-diagonal part, out[2] = min_{i != j} |l_i - l_j|,
// out[3] = max |l_i|.
template <typename T>
__global__ __launch_bounds__(1024) void k_spec_stats(int n, const T *Tm, int ld, const float *wr,
                                                     const float *wi, double *out) {
    __shared__ double r0[16], r1[16], r2[16], r3[16];
    double ncx = 0.0, bd = 0.0, gap = 1e300, mx = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        if (wi[i] != 0.f) ncx += 1.0;
        const double d = CM(Tm, i, i, ld);
        bd += d * d;
        if (i + 1 < n && CM(Tm, i + 1, i, ld) != T(0)) {
            const double b = CM(Tm, i, i + 1, ld), c = CM(Tm, i + 1, i, ld);
            bd += b * b + c * c;
        }
        mx = fmax(mx, sqrt((double)wr[i] * wr[i] + (double)wi[i] * wi[i]));
    }
    const size_t pairs = (size_t)n * n;
    for (size_t e = threadIdx.x; e < pairs; e += 1024) {
        const int i = (int)(e % n), j = (int)(e / n);
        if (i < j) {
            const double dr = (double)wr[i] - wr[j], di = (double)wi[i] - wi[j];
            gap = fmin(gap, sqrt(dr * dr + di * di));
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ncx += __shfl_xor(ncx, o);
        bd += __shfl_xor(bd, o);
        gap = fmin(gap, __shfl_xor(gap, o));
        mx = fmax(mx, __shfl_xor(mx, o));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { r0[w] = ncx; r1[w] = bd; r2[w] = gap; r3[w] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0, g = 1e300, x = 0;
        for (int k = 0; k < 16; ++k) { a += r0[k]; b += r1[k]; g = fmin(g, r2[k]); x = fmax(x, r3[k]); }
        out[0] = a; out[1] = b; out[2] = g; out[3] = x;
    }
}

// The 16 selector features from the low-precision forms in p.lo (mixed_forms
// with orth = 1 must have run).  Order:
//  0 log2 m, 1 log2 n, 2 log10(||A||_F/sqrt m), 3 log10(||B||_F/sqrt n),
//  4 log10(||C||_F/sqrt(mn)), 5 log10 sep_est, 6 log10 kappa_est
//  (= (||A||_F + ||B||_F)/sep_est), 7-8 Henrici departure ||N||_F/||T||_F of
//  T_A, T_B, 9-10 fraction of eigenvalues in complex pairs, 11-12 log10 of the
//  relative minimum eigenvalue gap, 13-14 log10 of the probe estimates of
//  ||U^T U - I||_F, ||V^T V - I||_F,
//  15 Lyapunov flag.
static int selector_features(hipStream_t s, DevCtx *c, int m, int n, bool lyap, Plan &p,
                             const Norms &nm, float *f) {
    float *wra = p.eig, *wia = p.eig + m, *wrb = p.eig + 2 * m, *wib = p.eig + 2 * m + n;
    hipLaunchKernelGGL((k_spec_stats<float>), dim3(1), dim3(1024), 0, s, m, p.lo.TA, m, wra, wia, p.scal + 40);
    hipLaunchKernelGGL((k_spec_stats<float>), dim3(1), dim3(1024), 0, s, n, p.lo.TB, n, wrb, wib, p.scal + 44);
    matnorm<float>(s, m, m, p.lo.TA, m, p.scal + 48, p.nscr, 0);
    matnorm<float>(s, n, n, p.lo.TB, n, p.scal + 49, p.nscr, 0);
    double h[64];
    hipError_t e = read_scalars(s, c, p.scal, 64, h);
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    auto lg = [](double x) { return std::log10(std::max(x, 1e-300)); };
    const double sep = std::max(h[13], 1e-300);
    f[0] = (float)std::log2((double)m);
    f[1] = (float)std::log2((double)n);
    f[2] = (float)lg(nm.a / std::sqrt((double)m));
    f[3] = (float)lg(nm.b / std::sqrt((double)n));
    f[4] = (float)lg(nm.c / std::sqrt((double)m * n));
    f[5] = (float)lg(sep);
    f[6] = (float)lg((nm.a + nm.b) / sep);
    auto henrici = [](double tf, double bd) {
        return tf > 0 ? std::sqrt(std::max(tf * tf - bd, 0.0)) / tf : 0.0;
    };
    f[7] = (float)henrici(h[48], h[41]);
    f[8] = (float)henrici(h[49], h[45]);
    f[9] = (float)(h[40] / m);
    f[10] = (float)(h[44] / n);
    f[11] = (float)lg(m > 1 ? h[42] / std::max(h[43], 1e-300) : 1.0);
    f[12] = (float)lg(n > 1 ? h[46] / std::max(h[47], 1e-300) : 1.0);
    f[13] = (float)lg(h[20]);
    f[14] = (float)lg(lyap ? h[20] : h[21]);
    f[15] = lyap ? 1.f : 0.f;
    return 0;
}

// Alg. 4.1 (Sec. 4.1): the Q factor, with positive diag(R), of the binary64
// copy of the low-precision Schur vectors, by CholQR2 in binary64 (G = U^T U,
// R = chol(G), Q = U R^{-1}, twice; FP64 MFMA for the products, LDS kernels
// for the diagonal blocks).  Then the triangular-basis coefficients
// T + L = Q^T A Q and F = QA^T C QB in binary64, Y0 from the low-precision
// tri-solve, the stationary iteration of Alg. 3.1 in the triangular basis
// with binary64 residuals and a binary64 tri-solve, and X = QA Y QB^T.
// Returns 0 or a negative ABI code; *bad = 1 when a Cholesky pivot was not
// positive (U too far from orthogonal for the method).
static int orthonormalize(hipStream_t s, DevCtx *c, int n, const float *U, double *Q, double *E, int *dfail,
                          int *bad) {
    cast<float, double>(s, n, n, U, n, Q, n, 1.0f);
    hipError_t e = hipMemsetAsync(dfail, 0, sizeof(int), s);
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    cholqr2(s, n, Q, n, E, nullptr, dfail);
    e = hipMemcpyAsync(c->hbuf, dfail, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    std::memcpy(bad, c->hbuf, sizeof(int));
    return 0;
}

// Alg. 4.2 needs U^{-1} in binary64: Newton-Schulz steps for the inverse,
// Z <- Z - Z (U Z - I) from Z = U^T, until ||U Z - I||_F <= 8 n u_64 (at most
// 8 steps; quadratic convergence from ||U U^T - I|| ~ u_low).  Returns the
// number of steps or a negative ABI code.
static int invert_nearly_orthogonal(hipStream_t s, DevCtx *c, int n, const double *U, double *Z, double *E,
                                    double *W, double *scal, double *nscr) {
    transpose<double>(s, n, n, U, n, Z, n, 0);
    const double target = 8.0 * n * 1.1102230246251565e-16;
    for (int it = 0; it <= 8; ++it) {
        gemm<double, double, double, double>(s, 0, 0, n, n, n, 1.0, U, n, Z, n, 0.0, E, n);
        sub_identity(s, n, E, n);
        matnorm<double>(s, n, n, E, n, scal, nscr, 0);
        double h;
        hipError_t e = read_scalars(s, c, scal, 1, &h);
        if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
        if (!(h > target) || it == 8) return it;
        cast<double, double>(s, n, n, Z, n, W, n, 1.0);
        gemm<double, double, double, double>(s, 0, 0, n, n, n, -1.0, Z, n, E, n, 1.0, W, n);
        cast<double, double>(s, n, n, W, n, Z, n, 1.0);
    }
    return 8;
}

// inv = false: Alg. 4.1 (orthonormalised factors Q); inv = true: Alg. 4.2
// (the low-precision factors U themselves, with their binary64 inverses):
//   F = U_A^T C U_B,  M_A = U_A^T A U_A^{-T},  M_B = U_B^{-1} B U_B,
//   X = U_A^{-T} Y U_B^{-1}.
static int run_alg41(hipStream_t s, DevCtx *c, int m, int n, const double *A, int lda, const double *B,
                     int ldb, bool lyap, const double *C, int ldc, double *X, int ldx, Plan &p,
                     const Norms &nm, const sylv_opts &o, sylv_info *info, int *ok, bool inv = false) {
    *ok = 0;
    int qa = 0, qb = 0;
    const int bf16 = narrow_of(o.low);
    int rc = mixed_forms(s, c, m, n, A, lda, B, ldb, lyap, p, bf16, o.orth_check, &qa, &qb);
    if (rc) return rc;
    OrthStage &q = p.o;
    if (!inv) {
        // Q_A, Q_B
        int bad_a = 0, bad_b = 0;
        if ((rc = orthonormalize(s, c, m, p.lo.UA, q.QA, q.E, p.flag + 1, &bad_a)) < 0) return rc;
        if (lyap) revcols<double, double>(s, n, n, q.QA, n, q.QB, n, 1.0);  // V = U P
        else if ((rc = orthonormalize(s, c, n, p.lo.UB, q.QB, q.E, p.flag + 1, &bad_b)) < 0) return rc;
        if (bad_a || bad_b) {
            // the binary32 factor is not orthogonal enough for a Cholesky QR:
            // report failure (the caller's fallback takes over)
            if (info) {
                std::memset(info, 0, sizeof(*info));
                info->status = SYLV_ST_NOT_CONVERGED;
                info->rel_res = INFINITY;
                info->precision_used = prec_of_narrow(bf16);
            }
            return 0;
        }
        // M_A = Q_A^T A Q_A, M_B = Q_B^T B Q_B (B = A^T for Lyapunov)
        gemm<double, double, double, double>(s, 0, 0, m, m, m, 1.0, A, lda, q.QA, m, 0.0, q.W, m);
        gemm<double, double, double, double>(s, 1, 0, m, m, m, 1.0, q.QA, m, q.W, m, 0.0, q.MA, m);
        if (lyap) gemm<double, double, double, double>(s, 1, 0, n, n, n, 1.0, A, lda, q.QB, n, 0.0, q.W, n);
        else gemm<double, double, double, double>(s, 0, 0, n, n, n, 1.0, B, ldb, q.QB, n, 0.0, q.W, n);
        gemm<double, double, double, double>(s, 1, 0, n, n, n, 1.0, q.QB, n, q.W, n, 0.0, q.MB, n);
        // F = Q_A^T C Q_B
        gemm<double, double, double, double>(s, 1, 0, m, n, m, 1.0, q.QA, m, C, ldc, 0.0, q.W, m);
        gemm<double, double, double, double>(s, 0, 0, m, n, n, 1.0, q.W, m, q.QB, n, 0.0, q.F, m);
    } else {
        // binary64 U_A, U_B and Z_A = U_A^{-1}, Z_B = U_B^{-1} (in QA, QB)
        cast<float, double>(s, m, m, p.lo.UA, m, q.UA, m, 1.0f);
        cast<float, double>(s, n, n, p.lo.UB, n, q.UB, n, 1.0f);
        if ((rc = invert_nearly_orthogonal(s, c, m, q.UA, q.QA, q.E, q.W, p.scal + 53, p.nscr)) < 0) return rc;
        if ((rc = invert_nearly_orthogonal(s, c, n, q.UB, q.QB, q.E, q.W, p.scal + 53, p.nscr)) < 0) return rc;
        // M_A = U_A^T (A Z_A^T)
        gemm<double, double, double, double>(s, 0, 1, m, m, m, 1.0, A, lda, q.QA, m, 0.0, q.W, m);
        gemm<double, double, double, double>(s, 1, 0, m, m, m, 1.0, q.UA, m, q.W, m, 0.0, q.MA, m);
        // M_B = Z_B (B U_B), B = A^T for Lyapunov
        if (lyap) gemm<double, double, double, double>(s, 1, 0, n, n, n, 1.0, A, lda, q.UB, n, 0.0, q.W, n);
        else gemm<double, double, double, double>(s, 0, 0, n, n, n, 1.0, B, ldb, q.UB, n, 0.0, q.W, n);
        gemm<double, double, double, double>(s, 0, 0, n, n, n, 1.0, q.QB, n, q.W, n, 0.0, q.MB, n);
        // F = U_A^T C U_B
        gemm<double, double, double, double>(s, 1, 0, m, n, m, 1.0, q.UA, m, C, ldc, 0.0, q.W, m);
        gemm<double, double, double, double>(s, 0, 0, m, n, n, 1.0, q.W, m, q.UB, n, 0.0, q.F, m);
    }
    cast<float, double>(s, m, m, p.lo.TA, m, q.TA, m, 1.0f);
    cast<float, double>(s, n, n, p.lo.TB, n, q.TB, n, 1.0f);
    // Y0: low-precision solve of T_A Y + Y T_B = F
    hipMemsetAsync(p.flag, 0, sizeof(int), s);
    cast<double, float>(s, m, n, q.F, m, p.lo.Y, m, 1.0);
    trsyl<float>(s, m, n, p.lo.TA, m, p.lo.TB, n, p.lo.Y, m, p.scal + 12, p.flag, 0, p.lo.Pinv, p.lo.pflag);
    cast<float, double>(s, m, n, p.lo.Y, m, q.Y, m, 1.0f);
    // Alg. 3.1 in the triangular basis
    double hsep[2];
    hipError_t es = read_scalars(s, c, p.scal + 13, 2, hsep);
    if (es != hipSuccess) return SYLV_ERR_HIP - (int)es;
    double prev = INFINITY, rel = INFINITY, corr = 0.0, h[4];
    int it = 0, stall = 0, status = SYLV_ST_NOT_CONVERGED;
    for (;;) {
        cast<double, double>(s, m, n, q.F, m, p.R, m, 1.0);
        gemm<double, double, double, double>(s, 0, 0, m, n, m, -1.0, q.MA, m, q.Y, m, 1.0, p.R, m);
        gemm<double, double, double, double>(s, 0, 0, m, n, n, -1.0, q.Y, m, q.MB, n, 1.0, p.R, m);
        matnorm<double>(s, m, n, p.R, m, p.scal + 50, p.nscr, 0);
        matnorm<double>(s, m, n, q.Y, m, p.scal + 51, p.nscr, 0);
        hipError_t e = read_scalars(s, c, p.scal + 50, 2, h);
        if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
        rel = h[0] / (nm.c + h[1] * (nm.a + nm.b));
        if (!std::isfinite(rel)) { status = SYLV_ST_NAN; break; }
        // the stopping rule of the original-basis refinement (tol, then the
        // forward-error level 100 u kappa_est); ||Y||_F = ||X||_F up to the
        // binary64 orthogonality of the basis
        const bool at_tol = rel <= o.tol;
        const double growth = nm.a + nm.b + (h[1] > 0 ? nm.c / h[1] : 0.0);
        if (at_tol) status = SYLV_OK;
        if (at_tol && rel * growth <= 100.0 * 0x1p-53 * hsep[1]) break;
        if (it >= o.max_iter) break;
        if (rel > 0.5 * prev) { if (++stall >= (at_tol ? 1 : 2)) break; } else stall = 0;
        prev = rel;
        // D from T_A D + D T_B = R (binary64 tri-solve), Y += D
        trsyl<double>(s, m, n, q.TA, m, q.TB, n, p.R, m, p.scal + 12, p.flag);
        axpy<double>(s, m, n, 1.0, p.R, m, q.Y, m);
        matnorm<double>(s, m, n, p.R, m, p.scal + 52, p.nscr, 0);
        ++it;
        e = read_scalars(s, c, p.scal + 52, 1, h + 2);
        if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
        corr = h[2];
    }
    // X = Q_A Y Q_B^T (Alg. 4.1) or Z_A^T Y Z_B (Alg. 4.2), then the residual
    // against the original coefficients
    gemm<double, double, double, double>(s, inv ? 1 : 0, 0, m, n, m, 1.0, q.QA, m, q.Y, m, 0.0, q.W, m);
    gemm<double, double, double, double>(s, 0, inv ? 0 : 1, m, n, n, 1.0, q.W, m, q.QB, n, 0.0, X, ldx);
    residual(s, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p.R, p.scal, p.nscr);
    double hr[32];
    hipError_t e = read_scalars(s, c, p.scal, 32, hr);
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    const double rel_true = hr[0] / (nm.c + hr[2] * (nm.a + nm.b));
    int flag = 0;
    hipMemcpy(&flag, p.flag, sizeof(int), hipMemcpyDeviceToHost);
    if (status == SYLV_OK && !(rel_true <= o.tol)) status = SYLV_ST_NOT_CONVERGED;
    if (!std::isfinite(rel_true)) status = SYLV_ST_NAN;
    if (qa || qb) status = (status == SYLV_OK) ? SYLV_OK : SYLV_ST_QR_FAILED;
    if (status == SYLV_OK && flag) status = SYLV_ST_PERTURBED;
    *ok = (status == SYLV_OK || status == SYLV_ST_PERTURBED) ? 1 : 0;
    if (info) {
        info->rel_res = rel_true;
        info->orth_u = o.orth_check ? hr[20] : 0.0;
        info->orth_v = o.orth_check ? (lyap ? hr[20] : hr[21]) : 0.0;
        info->sep_est = hr[13];
        info->corr_ratio = (h[1] > 0) ? corr / h[1] : 0.0;
        info->iterations = it;
        info->precision_used = prec_of_narrow(bf16);
        info->status = status;
    }
    return 0;
}

// SYLV_PREC_AUTO: binary32 forms, their 16 features, the selector's class,
// then the chosen refinement on those same forms:
//   0: transforms on bfloat16 inputs, 1: binary32 transforms, 2: plain binary64;
// a failing class escalates (0 -> 1 on the same forms -> 2).
static int run_auto(hipStream_t s, DevCtx *c, int m, int n, const double *A, int lda,
                    const double *B, int ldb, bool lyap, const double *C, int ldc, double *X,
                    int ldx, Plan &p, const Norms &nm, const sylv_opts &o, sylv_info *info) {
    int qa = 0, qb = 0;
    int rc = mixed_forms(s, c, m, n, A, lda, B, ldb, lyap, p, 0, 1, &qa, &qb);
    if (rc) return rc;
    float f[SYLV_NFEAT], pr[SYLV_NCLASS];
    rc = selector_features(s, c, m, n, lyap, p, nm, f);
    if (rc) return rc;
    int cls = 1;
    rc = selector_choose(s, c->hbuf, f, &cls, pr);
    if (rc) return rc;
    sylv_opts oo = o;
    oo.orth_check = 1;
    sylv_info tmp;
    sylv_info *inf = info ? info : &tmp;
    int ok = 0, iters = 0, esc = 0;
    if (cls == 0) {
        rc = mixed_refine(s, c, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p, nm, oo, 1, qa, qb, inf, &ok);
        if (rc) return rc;
        iters += inf->iterations;
        if (!ok && o.fallback) esc = 1;
    }
    if (cls == 1 || (cls == 0 && esc)) {
        rc = mixed_refine(s, c, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p, nm, oo, 0, qa, qb, inf, &ok);
        if (rc) return rc;
        iters += inf->iterations;
        if (!ok && o.fallback) esc = 1;
    }
    if (cls == 2 || (!ok && o.fallback)) {
        rc = run_fp64(s, c, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p, nm, inf);
        if (rc) return rc;
        if (cls != 2) esc = 1;
    }
    inf->iterations = iters;
    inf->fell_back = esc;
    inf->chosen = cls;
    return 0;
}

// pc: a pooled context whose lock the caller holds (the library lock is
// then not taken); nullptr: the device's own context under the library lock.
static int solve_common_impl(int m, int n, const double *A, int lda, const double *B, int ldb,
                        const double *C, int ldc, double *X, int ldx, bool lyap,
                        const sylv_opts *opts, sylv_info *info, void *work, size_t work_bytes,
                        void *stream, DevCtx *pc = nullptr) {
    sylv_opts o;
    sylv_default_opts(&o);
    if (opts) o = *opts;
    // argument checks (ABI: -i for the i-th argument)
    if (m < 0) return -1;
    if (!lyap && n < 0) return -2;
    if (lyap) n = m;
    const int ai = lyap ? 2 : 3;  // position of A
    if (lda < std::max(1, m)) return -(ai + 1);
    if (!lyap && ldb < std::max(1, n)) return -6;
    const int ci = lyap ? 4 : 7;
    if (ldc < std::max(1, m)) return -(ci + 1);
    if (ldx < std::max(1, m)) return -(ci + 3);
    if (m > 0 && (A == nullptr)) return -ai;
    if (!lyap && n > 0 && B == nullptr) return -5;
    if (m > 0 && n > 0 && (C == nullptr)) return -ci;
    if (m > 0 && n > 0 && (X == nullptr)) return -(ci + 2);
    const bool autosel = o.low == SYLV_PREC_AUTO;
    if (o.low != SYLV_PREC_FP64 && o.low != SYLV_PREC_FP32 && o.low != SYLV_PREC_BF16 &&
        o.low != SYLV_PREC_FP16 && !autosel)
        return -(ci + 4);
    if (autosel && !selector_installed()) return -(ci + 4);
    if (!(o.tol >= 0.0) || o.max_iter < 0) return -(ci + 4);
    if (o.alg != SYLV_ALG_ORIG && o.alg != SYLV_ALG_ORTH && o.alg != SYLV_ALG_INV && o.alg != SYLV_ALG_SYM)
        return -(ci + 4);
    if (o.orth_check < 0 || o.orth_check > 2) return -(ci + 4);
    if (info) std::memset(info, 0, sizeof(*info));
    if (m == 0 || n == 0) {
        if (info) {
            info->precision_used = o.low;
            info->chosen = -1;
        }
        return 0;
    }
    {
        // the solve reads device results on the host between its stages, so
        // it cannot be recorded into a graph; with work == NULL it would also
        // allocate.  Refuse before any other call on the stream.
        const int cap = stream_capture_code((hipStream_t)stream, work == nullptr);
        if (cap) return cap;
    }
    std::unique_lock<std::mutex> lk(g_mu, std::defer_lock);
    DevCtx *c = pc;
    int rc = 0;
    if (!c) {
        lk.lock();
        rc = device_ctx(&c);
        if (rc) return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    const bool mixed = o.low != SYLV_PREC_FP64;
    const bool need_hi = !mixed || o.fallback || autosel;
    const int orth = !mixed ? 0 : autosel ? 1 : o.orth_check;
    const bool alg41 = mixed && !autosel && (o.alg == SYLV_ALG_ORTH || o.alg == SYLV_ALG_INV);
    const size_t need = plan_bytes(m, n, lyap, mixed, need_hi, orth, alg41);
    void *base = work;
    if (work) {
        if (work_bytes < need) return lyap ? -11 : -15;
    } else {
        rc = ensure_work(c, need, &base);
        if (rc) return rc;
    }
    Arena ar(base);
    Plan p;
    plan(ar, m, n, lyap, mixed, need_hi, orth, p, alg41);
    // norms of the coefficients (eq. (2.1) denominators)
    matnorm<double>(s, m, m, A, lda, p.scal + 40, p.nscr, 0);
    if (!lyap) matnorm<double>(s, n, n, B, ldb, p.scal + 41, p.nscr, 0);
    matnorm<double>(s, m, n, C, ldc, p.scal + 42, p.nscr, 0);
    const bool sym = !autosel && o.alg == SYLV_ALG_SYM;
    if (sym) {
        asym_norm(s, m, A, lda, p.scal + 43, p.nscr);
        if (!lyap) asym_norm(s, n, B, ldb, p.scal + 44, p.nscr);
    }
    if (lyap) asym_norm(s, m, C, ldc, p.scal + 45, p.nscr);
    matnorm<double>(s, m, n, C, ldc, p.scal + 46, p.nscr, 1);
    double hn[7] = {0, 0, 0, 0, 0, 0, 0};
    hipError_t e = read_scalars(s, c, p.scal + 40, 7, hn);
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    Norms nm{hn[0], lyap ? hn[0] : hn[1], hn[2], hn[6]};
    if (sym) {
        // symmetric coefficients are required up to rounding: ||A - A^T||_F
        // <= sqrt(u) ||A||_F (u = 2^-53), below binary32 resolution
        const double tol_sym = 1.4901161193847656e-08;
        if (!(hn[3] <= tol_sym * hn[0])) return -ai;
        if (!lyap && !(hn[4] <= tol_sym * hn[1])) return -5;
    }
    p.lo.diag = sym ? 1 : 0;
    p.hi.diag = sym ? 1 : 0;
    // Lyapunov with C symmetric to 2u ||C||_F: the solution is symmetric;
    // the iterate is kept symmetric, the residual takes one product and the
    // tri-solve one tile of each mirror pair (Alg. 4.1/4.2 keep the general
    // forms)
    const bool lsym = lyap && !alg41 && hn[5] <= 0x1p-52 * hn[2];
    p.lo.lsym = lsym ? 1 : 0;
    p.hi.lsym = lsym ? 1 : 0;
    if (info) info->chosen = -1;
    if (!mixed) return run_fp64(s, c, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p, nm, info);
    if (autosel) return run_auto(s, c, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p, nm, o, info);
    int ok = 0;
    if (alg41)
        rc = run_alg41(s, c, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p, nm, o, info, &ok,
                       o.alg == SYLV_ALG_INV);
    else rc = run_mixed(s, c, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p, nm, o, info, &ok);
    if (rc) return rc;
    int escalated = 0, iters = info ? info->iterations : 0;
    if (!ok && o.fallback && (o.low == SYLV_PREC_BF16 || o.low == SYLV_PREC_FP16)) {
        // escalation ladder: bfloat16 / binary16 updates -> binary32 -> plain binary64
        sylv_opts o32 = o;
        o32.low = SYLV_PREC_FP32;
        rc = run_mixed(s, c, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p, nm, o32, info, &ok);
        if (rc) return rc;
        escalated = 1;
        if (info) iters += info->iterations;
    }
    if (escalated && info) {
        info->fell_back = 1;
        info->iterations = iters;
    }
    if (!ok && o.fallback) {
        sylv_info keep;
        if (info) keep = *info;
        p.hi.diag = 0;  // the fallback is the general binary64 Bartels-Stewart
        rc = run_fp64(s, c, m, n, A, lda, B, ldb, lyap, C, ldc, X, ldx, p, nm, info);
        if (rc) return rc;
        if (info) {
            info->fell_back = 1;
            info->iterations = keep.iterations;
            info->orth_u = keep.orth_u;
            info->orth_v = keep.orth_v;
        }
    }
    return 0;
}

// Runs the solve and converts any pending HIP error (launch failures are
// reported asynchronously through hipGetLastError) into an ABI code, so no
// error is left behind for the caller's next HIP call.
static int solve_common(int m, int n, const double *A, int lda, const double *B, int ldb,
                        const double *C, int ldc, double *X, int ldx, bool lyap,
                        const sylv_opts *opts, sylv_info *info, void *work, size_t work_bytes,
                        void *stream, DevCtx *pc = nullptr) {
    int rc = solve_common_impl(m, n, A, lda, B, ldb, C, ldc, X, ldx, lyap, opts, info, work,
                               work_bytes, stream, pc);
    // invalid sizes and empty problems return before any HIP call
    if (m <= 0 || (!lyap && n <= 0)) return rc;
    hipError_t e = hipGetLastError();
    if (rc == 0 && e != hipSuccess) rc = SYLV_ERR_HIP - (int)e;
    if (rc == -1 && m >= 0) rc = SYLV_ERR_HIP;  // internal launch failure
    return rc;
}

// A solve on pooled context `slot` of the current device, on that
// context's own stream (independent of the caller's stream, which must not
// hold unfinished work the solve depends on).  B == nullptr: Lyapunov.
int solve_pooled(int slot, int m, int n, const double *A, int lda, const double *B, int ldb, const double *C,
                 int ldc, double *X, int ldx, const sylv_opts *opts, sylv_info *info, void *work,
                 size_t work_bytes) {
    if (slot < 0 || slot >= kSolvePool) return -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SYLV_ERR_NOGPU;
    std::lock_guard<std::mutex> lk(g_pool_mu[dev][slot]);
    DevCtx &c = g_pool[dev][slot];
    int rc = init_ctx(c, dev, true);
    if (rc) return rc;
    const bool lyap = B == nullptr;
    try {
        return solve_common(m, lyap ? m : n, A, lda, B, lyap ? 1 : ldb, C, ldc, X, ldx, lyap, opts, info, work,
                            work_bytes, (void *)c.own, &c);
    } catch (const std::bad_alloc &) {
        return SYLV_ERR_ALLOC;
    }
}

// ------------------------------------------------ allocation-free scratch
// Device scratch of sylv_solve_noalloc: a file-scope device array (each GPU
// holds its own copy for the life of the process).  Host code never uses the
// array's name as an address: sylv_init looks the copy of the current device
// up once and keeps it in g_scratch[dev].
constexpr size_t kScratchBytes = (size_t)SYLV_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];
static void *g_scratch[64];

}  // namespace sylv

using namespace sylv;

extern "C" {

void sylv_default_opts(sylv_opts *o) {
    if (!o) return;
    o->low = SYLV_PREC_FP32;
    o->alg = SYLV_ALG_ORIG;
    o->tol = 1e-14;
    o->max_iter = 20;
    o->fallback = 1;
    o->orth_check = 1;
}

size_t sylv_workspace_size(int m, int n, int lyap, const sylv_opts *opts) {
    sylv_opts o;
    sylv_default_opts(&o);
    if (opts) o = *opts;
    if (m < 0 || (!lyap && n < 0)) return 0;
    if (o.orth_check < 0 || o.orth_check > 2) return 0;
    if (lyap) n = m;
    const bool mixed = o.low != SYLV_PREC_FP64;
    const bool autosel = o.low == SYLV_PREC_AUTO;
    return plan_bytes(m, n, lyap != 0, mixed, !mixed || o.fallback || autosel,
                      !mixed ? 0 : (o.low == SYLV_PREC_AUTO) ? 1 : o.orth_check,
                      mixed && !autosel && (o.alg == SYLV_ALG_ORTH || o.alg == SYLV_ALG_INV));
}

int sylv_schur_tune(int prec, int nsmall, int nw, int nb, int adv, int nibble, int aed_waves,
                    int chase_waves, int chains) {
    if (prec != SYLV_PREC_FP64 && prec != SYLV_PREC_FP32) return -1;
    const bool f = prec == SYLV_PREC_FP32;
    SchurTune t = f ? schur_tune<float>() : schur_tune<double>();
    if (nsmall > 0) t.nsmall = nsmall;
    if (nw > 0) t.nw = nw;
    if (nb > 0) t.nb = nb;
    if (adv > 0) t.adv = adv;
    if (nibble >= 0) t.nibble = nibble;
    if (aed_waves > 0) t.aedw = aed_waves;
    if (chase_waves > 0) t.chasew = chase_waves;
    if (chains > 0) t.chains = chains;
    std::lock_guard<std::mutex> lk(g_mu);
    return (f ? schur_tune_set<float>(t) : schur_tune_set<double>(t)) ? -2 : 0;
}

int sylv_schur_tune_get(int prec, int *vals) {
    if (prec != SYLV_PREC_FP64 && prec != SYLV_PREC_FP32) return -1;
    if (!vals) return -2;
    const SchurTune t = prec == SYLV_PREC_FP32 ? schur_tune<float>() : schur_tune<double>();
    vals[0] = t.nsmall; vals[1] = t.nw; vals[2] = t.nb; vals[3] = t.adv; vals[4] = t.nibble;
    vals[5] = t.aedw; vals[6] = t.chasew; vals[7] = t.chains;
    return 0;
}

int sylv_selector_features(int m, int n, const double *A, int lda, const double *B, int ldb,
                           const double *C, int ldc, float *feats, void *stream) {
    const bool lyap = (B == nullptr);
    if (lyap) n = m;
    if (m < 1) return -1;
    if (n < 1) return -2;
    if (!A) return -3;
    if (lda < m) return -4;
    if (!lyap && ldb < n) return -6;
    if (!C) return -7;
    if (ldc < m) return -8;
    if (!feats) return -9;
    try {
        std::lock_guard<std::mutex> lk(g_mu);
        DevCtx *c = nullptr;
        int rc = device_ctx(&c);
        if (rc) return rc;
        hipStream_t s = (hipStream_t)stream;
        void *base = nullptr;
        rc = ensure_work(c, plan_bytes(m, n, lyap, true, false, 1), &base);
        if (rc) return rc;
        Arena ar(base);
        Plan p;
        plan(ar, m, n, lyap, true, false, 1, p);
        matnorm<double>(s, m, m, A, lda, p.scal + 40, p.nscr, 0);
        if (!lyap) matnorm<double>(s, n, n, B, ldb, p.scal + 41, p.nscr, 0);
        matnorm<double>(s, m, n, C, ldc, p.scal + 42, p.nscr, 0);
        matnorm<double>(s, m, n, C, ldc, p.scal + 43, p.nscr, 1);
        double hn[4];
        hipError_t e = read_scalars(s, c, p.scal + 40, 4, hn);
        if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
        Norms nm{hn[0], lyap ? hn[0] : hn[1], hn[2], hn[3]};
        int qa = 0, qb = 0;
        rc = mixed_forms(s, c, m, n, A, lda, B, ldb, lyap, p, 0, 1, &qa, &qb);
        if (rc) return rc;
        rc = selector_features(s, c, m, n, lyap, p, nm, feats);
        if (rc) return rc;
        e = hipGetLastError();
        return e == hipSuccess ? 0 : SYLV_ERR_HIP - (int)e;
    } catch (const std::bad_alloc &) {
        return SYLV_ERR_ALLOC;
    }
}

int sylv_solve(int m, int n, const double *A, int lda, const double *B, int ldb, const double *C,
               int ldc, double *X, int ldx, const sylv_opts *opts, sylv_info *info, void *work,
               size_t work_bytes, void *stream) {
    try {
        InfoSink sink(info, 1);
        const int rc = solve_common(m, n, A, lda, B, ldb, C, ldc, X, ldx, false, opts, sink.host(), work,
                                    work_bytes, stream);
        return sink.finish(rc, (hipStream_t)stream);
    } catch (const std::bad_alloc &) {
        return SYLV_ERR_ALLOC;
    }
}

int lyap_solve(int n, const double *A, int lda, const double *C, int ldc, double *X, int ldx,
               const sylv_opts *opts, sylv_info *info, void *work, size_t work_bytes, void *stream) {
    try {
        InfoSink sink(info, 1);
        const int rc = solve_common(n, n, A, lda, nullptr, 1, C, ldc, X, ldx, true, opts, sink.host(), work,
                                    work_bytes, stream);
        return sink.finish(rc, (hipStream_t)stream);
    } catch (const std::bad_alloc &) {
        return SYLV_ERR_ALLOC;
    }
}

int sylv_init(void) {
    try {
        std::lock_guard<std::mutex> lk(g_mu);
        DevCtx *c = nullptr;
        int rc = device_ctx(&c);
        if (rc) return rc;
        if (!g_scratch[c->dev]) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) return SYLV_ERR_HIP - (int)(e != hipSuccess ? e : hipErrorUnknown);
            g_scratch[c->dev] = ptr;
        }
        return 0;
    } catch (const std::bad_alloc &) {
        return SYLV_ERR_ALLOC;
    }
}

int sylv_solve_noalloc(int m, int n, const double *A, int lda, const double *B, int ldb, const double *C,
                       int ldc, double *X, int ldx, const sylv_opts *opts, sylv_info *info, void *stream) {
    sylv_opts o;
    sylv_default_opts(&o);
    if (opts) o = *opts;
    // the learned selector keeps a device copy of its weights, made on first use
    if (o.low == SYLV_PREC_AUTO) return -11;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SYLV_ERR_NOGPU;
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ptr = g_scratch[dev];
    }
    if (!ptr) return SYLV_ERR_NOINIT;
    if (const int cap = stream_capture_code((hipStream_t)stream, false)) return cap;
    const size_t need = sylv_workspace_size(m, n, 0, &o);
    if (need > kScratchBytes) return SYLV_ERR_SCRATCH;
    return sylv_solve(m, n, A, lda, B, ldb, C, ldc, X, ldx, &o, info, ptr, kScratchBytes, stream);
}

int sylv_cholqr(int n, double *Q, int ldq, double *R, int ldr, int *status, void *stream) {
    if (n < 0) return -1;
    if (ldq < std::max(1, n)) return -3;
    if (R && ldr < std::max(1, n)) return -5;
    if (n > 0 && !Q) return -2;
    if (status) *status = 0;
    if (n == 0) return 0;
    try {
        std::lock_guard<std::mutex> lk(g_mu);
        DevCtx *c = nullptr;
        int rc = device_ctx(&c);
        if (rc) return rc;
        void *base = nullptr;
        const size_t nn = (size_t)n * n;
        rc = ensure_work(c, sizeof(double) * (2 * nn + 64), &base);
        if (rc) return rc;
        hipStream_t s = (hipStream_t)stream;
        double *G = (double *)base, *R1 = G + nn;
        int *dfail = (int *)(R1 + nn);
        hipError_t e = hipMemsetAsync(dfail, 0, sizeof(int), s);
        if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
        cholqr2(s, n, Q, ldq, G, R ? R1 : nullptr, dfail);
        if (R) {
            // R = R2 R1 with the strict lower parts of both cleared first
            clear_lower(s, n, G, n);
            clear_lower(s, n, R1, n);
            gemm<double, double, double, double>(s, 0, 0, n, n, n, 1.0, G, n, R1, n, 0.0, R, ldr);
        }
        e = hipMemcpyAsync(c->hbuf, dfail, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
        int bad = 0;
        std::memcpy(&bad, c->hbuf, sizeof(int));
        if (status) *status = bad ? SYLV_ST_NOT_CONVERGED : SYLV_OK;
        e = hipGetLastError();
        return e == hipSuccess ? 0 : SYLV_ERR_HIP - (int)e;
    } catch (const std::bad_alloc &) {
        return SYLV_ERR_ALLOC;
    }
}

const char *sylv_status_string(int code) {
    switch (code) {
        case SYLV_OK: return "ok";
        case SYLV_ST_PERTURBED: return "near-singular pivot perturbed in the quasi-triangular solve";
        case SYLV_ST_NOT_CONVERGED: return "refinement did not reach the tolerance";
        case SYLV_ST_NAN: return "NaN or Inf encountered";
        case SYLV_ST_QR_FAILED: return "QR algorithm (or symmetric Jacobi) iteration cap reached";
        case SYLV_ERR_ALLOC: return "device allocation failed";
        case SYLV_ERR_NOGPU: return "no gfx950 device";
        case SYLV_ERR_NOINIT: return "sylv_init has not been called on this device";
        case SYLV_ERR_CAPTURE_ALLOC:
            return "the stream is being captured and work == NULL asks the library to allocate";
        case SYLV_ERR_CAPTURE: return "the stream is being captured (the solve reads device results between stages)";
        case SYLV_ERR_SCRATCH: return "problem needs more than the static scratch of sylv_solve_noalloc";
        default:
            if (code <= SYLV_ERR_HIP && code > SYLV_ERR_ALLOC) return "HIP runtime error";
            if (code < 0) return "invalid argument";
            return "unknown status";
    }
}

// ---------------------------------------------------------- stage entry points
int sylv_schur(int n, const void *A, int lda, void *T, int ldt, void *U, int ldu, int prec,
               int *status, void *stream) {
    if (n < 0) return -1;
    if (lda < std::max(1, n)) return -3;
    if (ldt < std::max(1, n)) return -5;
    if (ldu < std::max(1, n)) return -7;
    if (prec != SYLV_PREC_FP64 && prec != SYLV_PREC_FP32) return -8;
    if (n > 0 && (!A || !T || !U)) return !A ? -2 : (!T ? -4 : -6);
    if (status) *status = 0;
    if (n == 0) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    DevCtx *c = nullptr;
    int rc = device_ctx(&c);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool f = prec == SYLV_PREC_FP32;
    const size_t es = f ? sizeof(float) : sizeof(double);
    size_t bytes = ((size_t)2 * n * n * es + 1024) + (f ? schur_work_bytes<float>(n) : schur_work_bytes<double>(n));
    void *base;
    rc = ensure_work(c, bytes, &base);
    if (rc) return rc;
    char *H = (char *)base;
    char *Uc = H + (((size_t)n * n * es + 255) & ~(size_t)255);
    char *ws = Uc + (((size_t)n * n * es + 255) & ~(size_t)255);
    int qr = 0;
    if (f) {
        cast<float, float>(s, n, n, (const float *)A, lda, (float *)H, n, 1.0f);
        rc = schur_run<float>(s, n, (float *)H, n, (float *)Uc, n, ws, c->hbuf, &qr);
        if (!rc) {
            cast<float, float>(s, n, n, (const float *)H, n, (float *)T, ldt, 1.0f);
            cast<float, float>(s, n, n, (const float *)Uc, n, (float *)U, ldu, 1.0f);
        }
    } else {
        cast<double, double>(s, n, n, (const double *)A, lda, (double *)H, n, 1.0);
        rc = schur_run<double>(s, n, (double *)H, n, (double *)Uc, n, ws, c->hbuf, &qr);
        if (!rc) {
            cast<double, double>(s, n, n, (const double *)H, n, (double *)T, ldt, 1.0);
            cast<double, double>(s, n, n, (const double *)Uc, n, (double *)U, ldu, 1.0);
        }
    }
    if (rc) { (void)hipGetLastError(); return rc < 0 && rc > -100 ? SYLV_ERR_HIP : rc; }
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    if (status) *status = qr ? SYLV_ST_QR_FAILED : SYLV_OK;
    return 0;
}

int sylv_sym_eig(int n, const void *S, int lds, void *d, void *Q, int ldq, int prec, int *sweeps,
                 int *status, void *stream) {
    if (n < 0) return -1;
    if (lds < std::max(1, n)) return -3;
    if (ldq < std::max(1, n)) return -6;
    if (prec != SYLV_PREC_FP64 && prec != SYLV_PREC_FP32) return -7;
    if (n > 0 && (!S || !d || !Q)) return !S ? -2 : (!d ? -4 : -5);
    if (sweeps) *sweeps = 0;
    if (status) *status = 0;
    if (n == 0) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    DevCtx *c = nullptr;
    int rc = device_ctx(&c);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool f = prec == SYLV_PREC_FP32;
    const size_t es = f ? sizeof(float) : sizeof(double);
    const size_t hb = ((size_t)n * n * es + 255) & ~(size_t)255;
    const size_t bytes = hb + 256 + (f ? sym_eig_work_bytes<float>(n) : sym_eig_work_bytes<double>(n));
    void *base;
    rc = ensure_work(c, bytes, &base);
    if (rc) return rc;
    char *H = (char *)base;
    char *ws = H + hb;
    int sw = 0;
    if (f) {
        sym_part<float, float>(s, n, (const float *)S, lds, (float *)H, n);
        rc = sym_eig<float>(s, n, (float *)H, n, (float *)Q, ldq, ws, c->hbuf, kSymSweeps, &sw);
        if (rc >= 0) get_diag<float>(s, n, (const float *)H, n, (float *)d);
    } else {
        sym_part<double, double>(s, n, (const double *)S, lds, (double *)H, n);
        rc = sym_eig<double>(s, n, (double *)H, n, (double *)Q, ldq, ws, c->hbuf, kSymSweeps, &sw);
        if (rc >= 0) get_diag<double>(s, n, (const double *)H, n, (double *)d);
    }
    if (rc < 0) { (void)hipGetLastError(); return rc; }
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    if (sweeps) *sweeps = sw;
    if (status) *status = rc ? SYLV_ST_QR_FAILED : SYLV_OK;
    return 0;
}

int sylv_trsyl(int m, int n, const void *TA, int ldta, const void *TB, int ldtb, int trans_b, void *Cp,
               int ldc, int prec, int *perturbed, void *stream) {
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (ldta < std::max(1, m)) return -4;
    if (ldtb < std::max(1, n)) return -6;
    if (ldc < std::max(1, m)) return -9;
    if (prec != SYLV_PREC_FP64 && prec != SYLV_PREC_FP32) return -10;
    if (m > 0 && !TA) return -3;
    if (n > 0 && !TB) return -5;
    if (m > 0 && n > 0 && !Cp) return -8;
    if (perturbed) *perturbed = 0;
    if (m == 0 || n == 0) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    DevCtx *c = nullptr;
    int rc = device_ctx(&c);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool f = prec == SYLV_PREC_FP32;
    const size_t es = f ? sizeof(float) : sizeof(double);
    // scratch: reversed TB (trans_b), reversed C, scalars, and in binary32
    // the block-pair inverse rows (4 m n)
    const size_t pinv_bytes = f ? (((size_t)4 * m * n * sizeof(float) + 255) & ~(size_t)255) : 0;
    size_t bytes = (size_t)n * n * es + (size_t)m * n * es + 8192 + pinv_bytes + 512;
    void *base;
    rc = ensure_work(c, bytes, &base);
    if (rc) return rc;
    char *TBr = (char *)base;
    char *Cr = TBr + (((size_t)n * n * es + 255) & ~(size_t)255);
    double *scal = (double *)(Cr + (((size_t)m * n * es + 255) & ~(size_t)255));
    double *nscr = scal + 8;
    int *flag = (int *)(nscr + 256);
    int *pflag = flag + 16;
    float *Pinv = f ? (float *)((char *)scal + 8192) : nullptr;
    hipMemsetAsync(flag, 0, sizeof(int), s);
    if (f) {
        const float *ta = (const float *)TA, *tb = (const float *)TB;
        matnorm<float>(s, m, m, ta, ldta, scal + 0, nscr, 1);
        matnorm<float>(s, n, n, tb, ldtb, scal + 1, nscr, 1);
        matnorm<double>(s, 2, 1, scal, 2, scal + 2, nscr, 1);
        if (!trans_b) {
            trsyl_prep<float>(s, m, n, ta, ldta, tb, ldtb, scal + 2, pflag, Pinv);
            trsyl<float>(s, m, n, ta, ldta, tb, ldtb, (float *)Cp, ldc, scal + 2, flag, 0, Pinv, pflag);
        } else {
            transpose<float>(s, n, n, tb, ldtb, (float *)TBr, n, 1);
            revcols<float, float>(s, m, n, (const float *)Cp, ldc, (float *)Cr, m, 1.0f);
            trsyl_prep<float>(s, m, n, ta, ldta, (const float *)TBr, n, scal + 2, pflag, Pinv);
            trsyl<float>(s, m, n, ta, ldta, (const float *)TBr, n, (float *)Cr, m, scal + 2, flag, 0, Pinv, pflag);
            revcols<float, float>(s, m, n, (const float *)Cr, m, (float *)Cp, ldc, 1.0f);
        }
    } else {
        const double *ta = (const double *)TA, *tb = (const double *)TB;
        matnorm<double>(s, m, m, ta, ldta, scal + 0, nscr, 1);
        matnorm<double>(s, n, n, tb, ldtb, scal + 1, nscr, 1);
        matnorm<double>(s, 2, 1, scal, 2, scal + 2, nscr, 1);
        if (!trans_b) trsyl<double>(s, m, n, ta, ldta, tb, ldtb, (double *)Cp, ldc, scal + 2, flag);
        else {
            transpose<double>(s, n, n, tb, ldtb, (double *)TBr, n, 1);
            revcols<double, double>(s, m, n, (const double *)Cp, ldc, (double *)Cr, m, 1.0);
            trsyl<double>(s, m, n, ta, ldta, (const double *)TBr, n, (double *)Cr, m, scal + 2, flag);
            revcols<double, double>(s, m, n, (const double *)Cr, m, (double *)Cp, ldc, 1.0);
        }
    }
    int hf = 0;
    hipError_t e = hipMemcpyAsync(c->hbuf, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    std::memcpy(&hf, c->hbuf, sizeof(int));
    if (perturbed) *perturbed = hf;
    e = hipGetLastError();
    return e == hipSuccess ? 0 : SYLV_ERR_HIP - (int)e;
}

int sylv_residual(int m, int n, const double *A, int lda, const double *B, int ldb, const double *C,
                  int ldc, const double *X, int ldx, double *R, int ldr, int lyap, double *rel_res,
                  void *stream) {
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (lyap && n != m) return -2;
    if (lda < std::max(1, m)) return -4;
    if (!lyap && ldb < std::max(1, n)) return -6;
    if (ldc < std::max(1, m)) return -8;
    if (ldx < std::max(1, m)) return -10;
    if (R && ldr < std::max(1, m)) return -12;
    if (m > 0 && !A) return -3;
    if (!lyap && n > 0 && !B) return -5;
    if (m > 0 && n > 0 && (!C || !X)) return !C ? -7 : -9;
    if (rel_res) *rel_res = 0.0;
    if (m == 0 || n == 0) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    DevCtx *c = nullptr;
    int rc = device_ctx(&c);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    size_t bytes = (size_t)m * n * sizeof(double) + 8192;
    void *base;
    rc = ensure_work(c, bytes, &base);
    if (rc) return rc;
    double *Rw = (double *)base;
    double *scal = (double *)((char *)base + (((size_t)m * n * sizeof(double) + 255) & ~(size_t)255));
    double *nscr = scal + 16;
    residual(s, m, n, A, lda, B, ldb, lyap != 0, C, ldc, X, ldx, Rw, scal, nscr);
    matnorm<double>(s, m, m, A, lda, scal + 4, nscr, 0);
    if (!lyap) matnorm<double>(s, n, n, B, ldb, scal + 5, nscr, 0);
    matnorm<double>(s, m, n, C, ldc, scal + 6, nscr, 0);
    if (R) cast<double, double>(s, m, n, Rw, m, R, ldr, 1.0);
    double h[8];
    hipError_t e = read_scalars(s, c, scal, 8, h);
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    double nb = lyap ? h[4] : h[5];
    if (rel_res) *rel_res = h[0] / (h[6] + h[2] * (h[4] + nb));
    e = hipGetLastError();
    return e == hipSuccess ? 0 : SYLV_ERR_HIP - (int)e;
}

int sylv_gemm(int prec, int ta, int tb, int m, int n, int k, double alpha, const void *A, int lda,
              const void *B, int ldb, double beta, void *C, int ldc, void *stream) {
    if (prec != SYLV_PREC_FP64 && prec != SYLV_PREC_FP32 && prec != SYLV_PREC_BF16 && prec != SYLV_PREC_FP16)
        return -1;
    if (m < 0) return -4;
    if (n < 0) return -5;
    if (k < 0) return -6;
    if (lda < std::max(1, ta ? k : m)) return -9;
    if (ldb < std::max(1, tb ? n : k)) return -11;
    if (ldc < std::max(1, m)) return -14;
    if (m == 0 || n == 0) return 0;
    if (!C) return -13;
    if (k > 0 && (!A || !B)) return !A ? -8 : -10;
    DevCtx *c = nullptr;
    int rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        rc = device_ctx(&c);
    }
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (prec == SYLV_PREC_FP64)
        gemm<double, double, double, double>(s, ta, tb, m, n, k, alpha, (const double *)A, lda,
                                             (const double *)B, ldb, beta, (double *)C, ldc);
    else
        gemm<float, float, float, float>(s, ta, tb, m, n, k, (float)alpha, (const float *)A, lda,
                                         (const float *)B, ldb, (float)beta, (float *)C, ldc, 1.0f,
                                         narrow_of(prec));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    return 0;
}

}  // extern "C"
