// Binary64 QR factorisation of a nearly orthogonal square matrix by CholQR2:
// G = U^T U, R = chol(G) (upper, positive diagonal), Q = U R^{-1}, done twice
// (the second pass removes the loss of orthogonality of the first, which is
// about kappa(U)^2 u = O(u) here).  Q is the Q factor of U with positive
// diag(R) that Alg. 4.1 asks of its binary64 QR step.
//
// Cholesky: right-looking by blocks of NB = 64 columns on the upper
// triangle; each step factors its diagonal block in LDS (k_potrf_block),
// solves the row panel R_kk^T X = G_k,rest with one thread per column
// (k_trsm_rowpanel), and updates the trailing matrix with the MFMA GEMM.
// TRSM Q <- Q R^{-1}: by blocks of NB columns, Q_j <- (Q_j - Q_{<j} R_{<j,j})
// R_jj^{-1}, the GEMM first and then one thread per row (k_trsm_rows).
#include "common.hpp"
#include "kernels.hpp"

namespace sylv {

constexpr int CQ_NB = 64;

// In-place Cholesky of the nb x nb diagonal block at G (upper triangle read,
// G = R^T R, R written to the upper triangle, strict lower triangle zeroed).
// *fail = 1 on a non-positive pivot.
__global__ __launch_bounds__(256) void k_potrf_block(int nb, double *G, int ldg, int *fail) {
    __shared__ double a[CQ_NB][CQ_NB + 1];
    __shared__ double piv;
    const int t = threadIdx.x;
    for (int e = t; e < nb * nb; e += 256) {
        const int i = e % nb, j = e / nb;
        a[i][j] = (i <= j) ? G[(size_t)j * ldg + i] : 0.0;
    }
    __syncthreads();
    for (int c = 0; c < nb; ++c) {
        if (t == 0) {
            const double d = a[c][c];
            if (!(d > 0.0)) *fail = 1;
            piv = d > 0.0 ? sqrt(d) : 1.0;
            a[c][c] = piv;
        }
        __syncthreads();
        const double r = 1.0 / piv;
        for (int j = c + 1 + t; j < nb; j += 256) a[c][j] *= r;
        __syncthreads();
        // trailing block: a[i][j] -= a[c][i] a[c][j] for c < i <= j
        const int m = nb - c - 1;
        for (int e = t; e < m * m; e += 256) {
            const int i = c + 1 + e % m, j = c + 1 + e / m;
            if (i <= j) a[i][j] -= a[c][i] * a[c][j];
        }
        __syncthreads();
    }
    for (int e = t; e < nb * nb; e += 256) {
        const int i = e % nb, j = e / nb;
        G[(size_t)j * ldg + i] = (i <= j) ? a[i][j] : 0.0;
    }
}

// Row panel P (nb x ncols at P, ld ldg) <- R_kk^{-T} P, R_kk the factored
// upper block at Rkk: one thread per column, forward substitution with
// R_kk^T (lower triangular) staged in LDS.
__global__ __launch_bounds__(256) void k_trsm_rowpanel(int nb, int ncols, const double *Rkk, int ldg, double *P) {
    __shared__ double r[CQ_NB][CQ_NB + 1];
    for (int e = threadIdx.x; e < nb * nb; e += 256) {
        const int i = e % nb, j = e / nb;
        r[i][j] = Rkk[(size_t)j * ldg + i];
    }
    __syncthreads();
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= ncols) return;
    double *col = P + (size_t)j * ldg;
    double x[CQ_NB];
#pragma unroll
    for (int i = 0; i < CQ_NB; ++i) x[i] = (i < nb) ? col[i] : 0.0;
#pragma unroll
    for (int i = 0; i < CQ_NB; ++i) {
        if (i < nb) {
            double v = x[i];
#pragma unroll
            for (int l = 0; l < i; ++l) v -= r[l][i] * x[l];
            x[i] = v / r[i][i];
        }
    }
#pragma unroll
    for (int i = 0; i < CQ_NB; ++i)
        if (i < nb) col[i] = x[i];
}

// Rows of W (nrows x nb at W, ld ldw) <- W R_jj^{-1} for the upper nb x nb
// block Rjj: one thread per row, x R_jj = w by forward substitution.
__global__ __launch_bounds__(256) void k_trsm_rows(int nrows, int nb, const double *Rjj, int ldr, double *W,
                                                   int ldw) {
    __shared__ double r[CQ_NB][CQ_NB + 1];
    for (int e = threadIdx.x; e < nb * nb; e += 256) {
        const int i = e % nb, j = e / nb;
        r[i][j] = Rjj[(size_t)j * ldr + i];
    }
    __syncthreads();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nrows) return;
    double x[CQ_NB];
#pragma unroll
    for (int c = 0; c < CQ_NB; ++c) {
        if (c < nb) {
            double v = W[(size_t)c * ldw + i];
#pragma unroll
            for (int l = 0; l < c; ++l) v -= x[l] * r[l][c];
            x[c] = v / r[c][c];
        }
    }
#pragma unroll
    for (int c = 0; c < CQ_NB; ++c)
        if (c < nb) W[(size_t)c * ldw + i] = x[c];
}

// G (n x n, ldg; symmetric positive definite, upper triangle read) <- R with
// G = R^T R in the upper triangle, R upper triangular with a positive
// diagonal (the strict lower triangle of each diagonal block is zeroed; the
// blocks below them keep scratch values and are never read as part of R).
// *fail (device int) is set on a non-positive pivot.
void chol_upper(hipStream_t s, int n, double *G, int ldg, int *fail) {
    for (int k = 0; k < n; k += CQ_NB) {
        const int nb = std::min(CQ_NB, n - k);
        double *Gkk = G + (size_t)k * ldg + k;
        hipLaunchKernelGGL(k_potrf_block, dim3(1), dim3(256), 0, s, nb, Gkk, ldg, fail);
        const int rest = n - k - nb;
        if (rest <= 0) break;
        double *Pk = G + (size_t)(k + nb) * ldg + k;  // row panel R_k,rest (nb x rest)
        hipLaunchKernelGGL(k_trsm_rowpanel, dim3((rest + 255) / 256), dim3(256), 0, s, nb, rest, Gkk, ldg, Pk);
        // G_rest,rest -= P^T P
        double *Gr = G + (size_t)(k + nb) * ldg + (k + nb);
        gemm<double, double, double, double>(s, 1, 0, rest, rest, nb, -1.0, Pk, ldg, Pk, ldg, 1.0, Gr, ldg);
    }
}

// Q (m x n, ldq) <- Q R^{-1}, R upper triangular (n x n, ldr).
void trsm_right_upper(hipStream_t s, int m, int n, const double *R, int ldr, double *Q, int ldq) {
    for (int j = 0; j < n; j += CQ_NB) {
        const int nb = std::min(CQ_NB, n - j);
        double *Qj = Q + (size_t)j * ldq;
        if (j > 0)
            gemm<double, double, double, double>(s, 0, 0, m, nb, j, -1.0, Q, ldq, R + (size_t)j * ldr, ldr, 1.0,
                                                 Qj, ldq);
        hipLaunchKernelGGL(k_trsm_rows, dim3((m + 255) / 256), dim3(256), 0, s, m, nb, R + (size_t)j * ldr + j, ldr,
                           Qj, ldq);
    }
}

__global__ void k_clear_lower(int n, double *A, int lda) {
    const size_t total = (size_t)n * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        if (i > j) A[(size_t)j * lda + i] = 0.0;
    }
}

// strict lower triangle of A (n x n) <- 0
void clear_lower(hipStream_t s, int n, double *A, int lda) {
    const int nb = (int)std::min<size_t>(2048, ((size_t)n * n + 255) / 256);
    if (nb > 0) hipLaunchKernelGGL(k_clear_lower, dim3(nb), dim3(256), 0, s, n, A, lda);
}

// CholQR2 of the n x n binary64 matrix Q (ldq) in place (Q <- the Q factor
// with positive diag(R)); G: n x n scratch; R1 (n x n, may be NULL): the
// first pass's triangular factor is kept there so that the caller can form
// R = R2 R1 (R2 is left in G).  *fail (device int, cleared by the caller) is
// set when a Cholesky pivot was not positive.
void cholqr2(hipStream_t s, int n, double *Q, int ldq, double *G, double *R1, int *fail) {
    for (int pass = 0; pass < 2; ++pass) {
        gemm<double, double, double, double>(s, 1, 0, n, n, n, 1.0, Q, ldq, Q, ldq, 0.0, G, n);
        chol_upper(s, n, G, n, fail);
        trsm_right_upper(s, n, n, G, n, Q, ldq);
        if (pass == 0 && R1) cast<double, double>(s, n, n, G, n, R1, n, 1.0);
    }
}

}  // namespace sylv
