// Memory-bound helper kernels: casts, copies, identity, Frobenius norms,
// max-abs.  All reductions are deterministic (fixed-shape partial sums, then
// one workgroup combines them in a fixed order).
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace sylv {

// dst(i,j) = (TD)(scale * src(i,j)) for an r x c block.
template <typename TS, typename TD>
__global__ void k_cast(int r, int c, const TS *__restrict__ src, int lds, TD *__restrict__ dst,
                       int ldd, TS scale) {
    size_t total = (size_t)r * c;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(e % r), j = (int)(e / r);
        dst[(size_t)j * ldd + i] = (TD)(scale * src[(size_t)j * lds + i]);
    }
}

static inline int grid_for(size_t total) {
    size_t g = (total + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

template <typename TS, typename TD>
void cast(hipStream_t s, int r, int c, const TS *src, int lds, TD *dst, int ldd, TS scale) {
    if (r <= 0 || c <= 0) return;
    ProfScope ps(KID_CAST, s);
    hipLaunchKernelGGL((k_cast<TS, TD>), dim3(grid_for((size_t)r * c)), dim3(256), 0, s, r, c, src,
                       lds, dst, ldd, scale);
}
template void cast<double, float>(hipStream_t, int, int, const double *, int, float *, int, double);
template void cast<float, double>(hipStream_t, int, int, const float *, int, double *, int, float);
template void cast<double, double>(hipStream_t, int, int, const double *, int, double *, int, double);
template void cast<float, float>(hipStream_t, int, int, const float *, int, float *, int, float);

// dst = src^T (r x c source -> c x r destination), optionally reversing the
// order of rows and columns of the result: dst(i,j) = src(c-1-j', ...) —
// used to build P T^T P (reversal permutation P) for the Lyapunov solve.
template <typename T>
__global__ void k_transpose(int r, int c, const T *__restrict__ src, int lds, T *__restrict__ dst,
                            int ldd, int reverse) {
    size_t total = (size_t)r * c;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(e % c), j = (int)(e / c);  // destination (i, j), c x r
        int si = j, sj = i;                       // dst(i,j) = src(j,i)
        if (reverse) { si = r - 1 - j; sj = c - 1 - i; }
        dst[(size_t)j * ldd + i] = src[(size_t)sj * lds + si];
    }
}

template <typename T>
void transpose(hipStream_t s, int r, int c, const T *src, int lds, T *dst, int ldd, int reverse) {
    if (r <= 0 || c <= 0) return;
    hipLaunchKernelGGL((k_transpose<T>), dim3(grid_for((size_t)r * c)), dim3(256), 0, s, r, c, src,
                       lds, dst, ldd, reverse);
}
template void transpose<float>(hipStream_t, int, int, const float *, int, float *, int, int);
template void transpose<double>(hipStream_t, int, int, const double *, int, double *, int, int);

// dst(:, j) = src(:, c-1-j)  (column reversal, r x c)
template <typename TS, typename TD>
__global__ void k_revcols(int r, int c, const TS *__restrict__ src, int lds, TD *__restrict__ dst,
                          int ldd, TS scale) {
    size_t total = (size_t)r * c;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(e % r), j = (int)(e / r);
        dst[(size_t)j * ldd + i] = (TD)(scale * src[(size_t)(c - 1 - j) * lds + i]);
    }
}
template <typename TS, typename TD>
void revcols(hipStream_t s, int r, int c, const TS *src, int lds, TD *dst, int ldd, TS scale) {
    if (r <= 0 || c <= 0) return;
    hipLaunchKernelGGL((k_revcols<TS, TD>), dim3(grid_for((size_t)r * c)), dim3(256), 0, s, r, c,
                       src, lds, dst, ldd, scale);
}
template void revcols<float, float>(hipStream_t, int, int, const float *, int, float *, int, float);
template void revcols<double, double>(hipStream_t, int, int, const double *, int, double *, int, double);
template void revcols<double, float>(hipStream_t, int, int, const double *, int, float *, int, double);

template <typename T>
__global__ void k_identity(int n, T *__restrict__ U, int ldu) {
    size_t total = (size_t)n * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(e % n), j = (int)(e / n);
        U[(size_t)j * ldu + i] = (i == j) ? T(1) : T(0);
    }
}
template <typename T>
void identity(hipStream_t s, int n, T *U, int ldu) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_identity<T>), dim3(grid_for((size_t)n * n)), dim3(256), 0, s, n, U, ldu);
}
template void identity<float>(hipStream_t, int, float *, int);
template void identity<double>(hipStream_t, int, double *, int);

// ---------------------------------------------------------------- norms
// Partial sums of squares (binary64 accumulation) over fixed column slabs,
// then a single-workgroup final sum in a fixed order.
constexpr int NRM_BLOCKS = 256;

template <typename T>
__global__ __launch_bounds__(256) void k_sumsq_partial(int r, int c, const T *__restrict__ a,
                                                       int ld, double *__restrict__ part,
                                                       int mode /*0 sumsq, 1 maxabs*/) {
    __shared__ double red[256];
    double acc = 0.0;
    size_t total = (size_t)r * c;
    size_t per = (total + gridDim.x - 1) / gridDim.x;
    size_t e0 = blockIdx.x * per, e1 = e0 + per < total ? e0 + per : total;
    for (size_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        int i = (int)(e % r), j = (int)(e / r);
        double v = (double)a[(size_t)j * ld + i];
        if (mode == 0) acc += v * v;
        else acc = fmax(acc, fabs(v));
        if (v != v) acc = v;  // propagate NaN
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            double x = red[threadIdx.x], y = red[threadIdx.x + s];
            red[threadIdx.x] = (mode == 0) ? x + y : ((x != x || y != y) ? x + y : fmax(x, y));
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_reduce_final(int nparts, const double *__restrict__ part, double *__restrict__ out,
                               int mode) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        double v = part[i];
        acc = (mode == 0) ? acc + v : ((v != v || acc != acc) ? acc + v : fmax(acc, v));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            double x = red[threadIdx.x], y = red[threadIdx.x + s];
            red[threadIdx.x] = (mode == 0) ? x + y : ((x != x || y != y) ? x + y : fmax(x, y));
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (mode == 0) ? sqrt(red[0]) : red[0];
}

// *out (device) = ||a||_F (mode 0) or max|a_ij| (mode 1).  scratch >= NRM_BLOCKS doubles.
template <typename T>
void matnorm(hipStream_t s, int r, int c, const T *a, int ld, double *out, double *scratch, int mode) {
    if (r <= 0 || c <= 0) {
        hipMemsetAsync(out, 0, sizeof(double), s);
        return;
    }
    size_t total = (size_t)r * c;
    int nb = (int)((total + 4095) / 4096);
    if (nb > NRM_BLOCKS) nb = NRM_BLOCKS;
    if (nb < 1) nb = 1;
    {
        ProfScope ps(KID_NORM, s);
        hipLaunchKernelGGL((k_sumsq_partial<T>), dim3(nb), dim3(256), 0, s, r, c, a, ld, scratch, mode);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, nb, scratch, out, mode);
}
// Symmetric Lyapunov residual: on entry R = -A X with X = X^T, so
// X A^T = (A X)^T and C - A X - X A^T = C + R + R^T; and X <- (X + X^T)/2.
// One workgroup per 32 x 32 tile pair (sym_tile_pair).
__global__ __launch_bounds__(256) void k_sym_pairs(int n, const double *__restrict__ C, int ldc, double *R, int ldr,
                                                   int res) {
    __shared__ double sa[32][33], sb[32][33];
    int ti, tj;
    sym_pair_index(blockIdx.x, ti, tj);
    sym_tile_pair(res != 0, n, C, ldc, R, ldr, ti, tj, sa, sb);
}

static unsigned sym_grid(int n) {
    const unsigned nt = (unsigned)(n + 31) / 32;
    return nt * (nt + 1) / 2;
}

void sym_residual(hipStream_t s, int n, const double *C, int ldc, double *R, int ldr) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_sym_pairs, dim3(sym_grid(n)), dim3(256), 0, s, n, C, ldc, R, ldr, 1);
}

// Strict lower triangle of X <- the transpose of its strict upper triangle,
// one 32 x 32 tile pair (ti <= tj) per workgroup through LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_mirror_upper(int n, T *X, int ldx) {
    __shared__ T t[32][33];
    int ti, tj;
    sym_pair_index(blockIdx.x, ti, tj);
    const int r0 = 32 * ti, c0 = 32 * tj;
    for (int e = threadIdx.x; e < 1024; e += 256) {
        const int ii = e & 31, jj = e >> 5;
        if (r0 + ii < n && c0 + jj < n) t[jj][ii] = X[(size_t)(c0 + jj) * ldx + r0 + ii];  // X(r0+ii, c0+jj)
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256) {
        const int ii = e & 31, jj = e >> 5;
        // target X(c0 + ii, r0 + jj) = X(r0 + jj, c0 + ii), below the diagonal only
        const int gi = c0 + ii, gj = r0 + jj;
        if (gi < n && gj < n && gi > gj) X[(size_t)gj * ldx + gi] = t[ii][jj];
    }
}

template <typename T>
void mirror_upper(hipStream_t s, int n, T *X, int ldx) {
    if (n <= 1) return;
    hipLaunchKernelGGL((k_mirror_upper<T>), dim3(sym_grid(n)), dim3(256), 0, s, n, X, ldx);
}
template void mirror_upper<float>(hipStream_t, int, float *, int);
template void mirror_upper<double>(hipStream_t, int, double *, int);

// Out = S P with S the symmetric matrix whose upper triangle is that of In
// and P the reversal permutation: Out(i, j) = S(i, n-1-j).
template <typename T>
__global__ void k_mirror_reverse(int n, const T *__restrict__ In, int ldi, T *__restrict__ Out, int ldo) {
    const size_t total = (size_t)n * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        const int c = n - 1 - j;
        Out[(size_t)j * ldo + i] = (i <= c) ? In[(size_t)c * ldi + i] : In[(size_t)i * ldi + c];
    }
}

template <typename T>
void mirror_reverse(hipStream_t s, int n, const T *In, int ldi, T *Out, int ldo) {
    if (n <= 0) return;
    const int nb = (int)std::min<size_t>(2048, ((size_t)n * n + 255) / 256);
    hipLaunchKernelGGL((k_mirror_reverse<T>), dim3(nb), dim3(256), 0, s, n, In, ldi, Out, ldo);
}
template void mirror_reverse<float>(hipStream_t, int, const float *, int, float *, int);
template void mirror_reverse<double>(hipStream_t, int, const double *, int, double *, int);


template void matnorm<float>(hipStream_t, int, int, const float *, int, double *, double *, int);
template void matnorm<double>(hipStream_t, int, int, const double *, int, double *, double *, int);

// ||U^T U - I||_F for a float U (n x n) in binary64: G = U^T U by FP64 MFMA
// after an exact widening of U, then the norm of G - I.
__global__ void k_sub_identity(int n, double *__restrict__ G, int ldg) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        G[(size_t)i * ldg + i] -= 1.0;
}
void sub_identity(hipStream_t s, int n, double *G, int ldg) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_sub_identity, dim3((n + 255) / 256), dim3(256), 0, s, n, G, ldg);
}

// X(:, :) += alpha * D (binary64 accumulate of a float correction)
template <typename TS>
__global__ void k_axpy(int r, int c, double alpha, const TS *__restrict__ D, int ldd,
                       double *__restrict__ X, int ldx) {
    size_t total = (size_t)r * c;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(e % r), j = (int)(e / r);
        X[(size_t)j * ldx + i] += alpha * (double)D[(size_t)j * ldd + i];
    }
}
template <typename TS>
void axpy(hipStream_t s, int r, int c, double alpha, const TS *D, int ldd, double *X, int ldx) {
    if (r <= 0 || c <= 0) return;
    hipLaunchKernelGGL((k_axpy<TS>), dim3(grid_for((size_t)r * c)), dim3(256), 0, s, r, c, alpha, D,
                       ldd, X, ldx);
}
template void axpy<float>(hipStream_t, int, int, double, const float *, int, double *, int);
template void axpy<double>(hipStream_t, int, int, double, const double *, int, double *, int);

}  // namespace sylv
