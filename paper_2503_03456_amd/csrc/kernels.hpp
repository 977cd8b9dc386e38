// Internal launch wrappers (all enqueue on the given stream).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace sylv {

// gemm.hip
template <typename TA, typename TB, typename TC, typename ACC>
void gemm(hipStream_t s, int ta, int tb, int M, int N, int K, ACC alpha, const TA *A, int lda,
          const TB *B, int ldb, ACC beta, TC *C, int ldc, TB bscale = TB(1));

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
template <typename TS>
void axpy(hipStream_t s, int r, int c, double alpha, const TS *D, int ldd, double *X, int ldx);

// hessenberg.hip
template <typename T>
size_t hessenberg_work_elems(int n, int nb, int S);
template <typename T>
void hessenberg(hipStream_t s, int n, T *A, int lda, T *U, int ldu, T *work, int nb, int S);

// hqr.hip
template <typename T>
size_t aed_smem(int nw);
template <typename T>
int aed_launch(hipStream_t s, int nw, T *H, int ldh, int kwtop, int spike_on, T *Zw, int *out, T *wr,
               T *wi);
template <typename T>
size_t chase_smem(int W, int nbulge);
template <typename T>
int chase_launch(hipStream_t s, T *H, int ldh, int ktop, int kbot, int ws, int W, int t0, int adv,
                 int nbulge, const T *trd, T *Uw);
template <typename T>
void find_ktop(hipStream_t s, T *H, int ldh, int klo, int kbot, int *out);
template <typename T>
void std2x2(hipStream_t s, int n, T *H, int ldh, T *U, int ldu, int k);
template <typename T>
void clean_lower(hipStream_t s, int n, T *H, int ldh);

// trsyl.hip
template <typename T>
void trsyl(hipStream_t s, int m, int n, const T *TA, int ldta, const T *TB, int ldtb, T *C, int ldc,
           const double *maxab, int *flag);

}  // namespace sylv
