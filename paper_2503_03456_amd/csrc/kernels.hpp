// Internal launch wrappers (all enqueue on the given stream).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <mutex>
#include <vector>
#include "../../include/sylv.h"

namespace sylv {

// Per-equation descriptor of the batched Lyapunov path (device resident).
// ptr/ld fields: 0 A, 1 C, 2 X (binary64, caller's), 3 R (binary64
// workspace), 4 H/T, 5 U, 6 W, 7 Y, 8 V = U P (U with its columns reversed),
// 9 TB = P T^T P (binary32 workspace, column-major, ld n).
enum BatchField {
    BF_A = 0, BF_C = 1, BF_X = 2, BF_R = 3, BF_H = 4, BF_U = 5, BF_W = 6, BF_Y = 7, BF_V = 8, BF_TB = 9,
    BF_COUNT = 10
};
struct BatchEq {
    void *ptr[BF_COUNT];
    int ld[BF_COUNT];
    int n;
    int active;      // 1 while the equation still needs work
    int status;      // sylv_info.status
    int iterations;  // corrections applied
    int qr_fail;
    int flag;        // tri-solve pivot perturbed
    double scale;    // 2^-e applied to the residual before the binary32 cast
    double nA, nC;   // ||A||_F, ||C||_F
    double rel_res, prev_rel, corr;
    double tmax;     // max |T_ij| (pivot threshold of the tri-solve)
    double lmax;     // max |lambda_i| of the binary32 Schur form (max |l_i + l_j| = 2 lmax)
    double orth;     // randomised estimate of ||U^T U - I||_F (binary64)
    int stall;
    int steps;       // double-shift QR steps of the Schur kernel
    double napply;   // 3-element reflector applications of the Schur kernel
    long long cyc[4];  // Schur kernel cycles: total, sweeps, U updates, deflation scans
    int sweeps;
    int sym;         // C symmetric to rounding: X kept symmetric, one-product residual, half tri-solve
    int cls;         // selector class (SYLV_PREC_AUTO): 0 bfloat16 transforms, 1 binary32, 2 binary64; -1 none
    int narrow;      // operand format of this equation's transforms under the selector (1 bfloat16)
};

// mlp.hip: feature standardisation and mini-batch gathering
void mlp_feature_stats(hipStream_t s, int n, const float *F, float *mean, float *sd);
void mlp_standardize(hipStream_t s, int n, const float *F, const float *mean, const float *sd, float *Z);
void mlp_gather(hipStream_t s, int cnt, const int *perm, const float *Z, const int *y, float *Zb, int *yb);

// selector.hip
bool selector_installed();
// device copy of the installed selector blob (params | means | deviations),
// uploaded on `s` when stale; nullptr if none is installed
const float *selector_device_blob(hipStream_t s, int *rc);
int selector_choose(hipStream_t s, char *hbuf, const float *feats, int *cls, float *probs);

// solver.hip
std::mutex &lib_mutex();
// independent solves run side by side on pooled contexts (own stream,
// staging and lock each); B == nullptr selects the Lyapunov equation
constexpr int kSolvePool = 8;
int solve_pooled(int slot, int m, int n, const double *A, int lda, const double *B, int ldb, const double *C,
                 int ldc, double *X, int ldx, const sylv_opts *opts, sylv_info *info, void *work,
                 size_t work_bytes);
int stream_capture_code(hipStream_t s, bool needs_alloc);
bool is_device_pointer(const void *p);
// Per-equation results for a caller array that may live in device memory:
// host() is where the solver writes, finish() copies to the device array
// (and synchronises) when the caller's pointer is device memory.
class InfoSink {
  public:
    InfoSink(sylv_info *user, int count);
    sylv_info *host();
    int finish(int rc, hipStream_t s);
  private:
    sylv_info *user_;
    int count_;
    std::vector<sylv_info> local_;
};
int device_work(size_t bytes, void **work, char **hbuf);

// lyap_batch.hip: all equations Lyapunov of order 1..256
size_t lyap_batched_bytes(int batch, const int *n);
int batch_tune_set(int hess_hi, int hess_lo, const int *band, int gpasses);
void batch_tune_get(int *vals);

// trsyl.hip: batched tri-solve T Y + Y TB = W over every active equation
void trsyl_batched(hipStream_t s, BatchEq *eqs, const int *order, int batch, int nmax);

// gemm.hip
template <typename TA, typename TB, typename TC, typename ACC>
void gemm(hipStream_t s, int ta, int tb, int M, int N, int K, double alpha, const TA *A, int lda,
          const TB *B, int ldb, ACC beta, TC *C, int ldc, TB bscale = TB(1), int in_bf16 = 0,
          int upper = 0);

// split-K partial products op(A) op(B) of the contraction slices into
// P + z M N (ld M); returns the slice count nz (<= ksplit)
template <typename T>
int gemm_splitk(hipStream_t s, int ta, int tb, int M, int N, int K, const T *A, int lda, const T *B, int ldb,
                T *P, int ksplit);

template <typename TA, typename TB, typename TC, typename ACC>
void gemm_batched(hipStream_t s, const BatchEq *eqs, const int *order, int batch, int nmax, int fa,
                  int ta, int fb, int tb, int fc, double alpha, int amode, ACC beta, int in_bf16 = 0);

// blas.hip
template <typename TS, typename TD>
void cast(hipStream_t s, int r, int c, const TS *src, int lds, TD *dst, int ldd, TS scale);
template <typename T>
void transpose(hipStream_t s, int r, int c, const T *src, int lds, T *dst, int ldd, int reverse);
template <typename TS, typename TD>
void revcols(hipStream_t s, int r, int c, const TS *src, int lds, TD *dst, int ldd, TS scale);
template <typename T>
void identity(hipStream_t s, int n, T *U, int ldu);
template <typename T>
void matnorm(hipStream_t s, int r, int c, const T *a, int ld, double *out, double *scratch, int mode);
void sub_identity(hipStream_t s, int n, double *G, int ldg);
void sym_residual(hipStream_t s, int n, const double *C, int ldc, double *R, int ldr);
template <typename T>
void mirror_upper(hipStream_t s, int n, T *X, int ldx);
template <typename T>
void mirror_reverse(hipStream_t s, int n, const T *In, int ldi, T *Out, int ldo);
template <typename TS>
void axpy(hipStream_t s, int r, int c, double alpha, const TS *D, int ldd, double *X, int ldx);

// hessenberg.hip
template <typename T>
size_t hessenberg_work_elems(int n, int nb, int S);
template <typename T>
void hessenberg(hipStream_t s, int n, T *A, int lda, T *U, int ldu, T *work, int nb, int S,
                int bf16 = 0);

// hqr.hip
template <typename T>
size_t aed_smem(int nw);
template <typename T>
int aed_launch(hipStream_t s, int nw, T *H, int ldh, int kwtop, int spike_on, T *Zw, int *out, T *wr,
               T *wi, int waves = 7);
template <typename T>
size_t chase_smem(int W, int nbulge);
// One bulge-chain window of a chase phase: rows/cols [ws, ws + W) of H,
// the chain's time t0 at the phase start (negative before its first
// bulge enters), its bulge count and shifts (3 values per bulge), and the
// W x W output of the window's orthogonal factor.
template <typename T>
struct ChaseWin {
    int ws, W, t0, nbulge;
    const T *trd;
    T *Uw;
};
constexpr int kChaseMaxWin = 4;
template <typename T>
struct ChaseSet {
    ChaseWin<T> w[kChaseMaxWin];
};
// nwin disjoint windows chased side by side (one workgroup each), adv steps
template <typename T>
int chase_launch(hipStream_t s, T *H, int ldh, int ktop, int kbot, const ChaseSet<T> &set, int nwin, int adv,
                 int waves = 16);
template <typename T>
void find_ktop(hipStream_t s, T *H, int ldh, int klo, int kbot, int *out);
template <typename T>
void gather_sub(hipStream_t s, const T *H, int ldh, int i0, int m, T *out);
template <typename T>
void std2x2(hipStream_t s, int n, T *H, int ldh, T *U, int ldu, int k);
template <typename T>
void clean_lower(hipStream_t s, int n, T *H, int ldh);

// syevj.hip: symmetric eigen-decomposition (block Jacobi) and the
// elementwise solve of the symmetric-coefficient variant
template <typename T>
size_t sym_eig_work_bytes(int n);
template <typename T>
int sym_eig(hipStream_t s, int n, T *S, int lds, T *Q, int ldq, char *ws, char *hbuf, int max_sweeps,
            int *sweeps);
template <typename TS, typename T>
void sym_part(hipStream_t s, int n, const TS *A, int lda, T *D, int ldd);
template <typename T>
void diag_solve(hipStream_t s, int m, int n, const T *TA, int ldta, const T *TB, int ldtb, T *Y, int ldy,
                const double *maxab, int *flag);
template <typename T>
void get_diag(hipStream_t s, int n, const T *D, int ldd, T *d);
void asym_norm(hipStream_t s, int n, const double *A, int lda, double *out, double *scratch);

// cholqr.hip: binary64 CholQR2 of a nearly orthogonal square matrix
void chol_upper(hipStream_t s, int n, double *G, int ldg, int *fail);
void clear_lower(hipStream_t s, int n, double *A, int lda);
void trsm_right_upper(hipStream_t s, int m, int n, const double *R, int ldr, double *Q, int ldq);
void cholqr2(hipStream_t s, int n, double *Q, int ldq, double *G, double *R1, int *fail);

// trsyl.hip
// mirror: symmetric Lyapunov (m = n, TB = P TA^T P, C persymmetric up to
// rounding): one tile of each mirror pair is solved and stores the other
// Pinv, pflag (binary32 only, both or neither): the block-pair inverse rows
// and their perturbation flag from trsyl_prep for the same TA, TB and mirror
template <typename T>
void trsyl(hipStream_t s, int m, int n, const T *TA, int ldta, const T *TB, int ldtb, T *C, int ldc,
           const double *maxab, int *flag, int mirror = 0, const T *Pinv = nullptr, const int *pflag = nullptr);
// Pinv (4 m n elements, 16-byte aligned) <- the rows of the inverse of every
// block pair's embedded system, for repeated solves with the same TA, TB
template <typename T>
void trsyl_prep(hipStream_t s, int m, int n, const T *TA, int ldta, const T *TB, int ldtb, const double *maxab,
                int *pflag, T *Pinv, int mirror = 0);

}  // namespace sylv
