// Batched Lyapunov solver AX + XA^T = C (eq. (1.3), real case) for many
// small equations (order <= 256): binary32 Schur forms + binary64
// refinement, one workgroup per equation, every stage covering the whole
// batch in one launch.  Equations are processed in decreasing order of size
// (longest first).
//
// Per equation:
//   1. k_bprep    ||A||_F, ||C||_F, control fields, symmetry test of C
//   2. k_bhess_reg Householder reduction of fl32(A) to Hessenberg form H and
//                 the orthogonal factor U0, both held in registers
//   3. k_bschur   Francis double-shift QR on the Hessenberg band held in LDS
//                 (3 subdiagonals: 33.7K floats at n = 256); the reflectors of
//                 a sweep are logged and applied to the rows of U once per
//                 sweep, each thread streaming one row through registers
//   4. transforms on MFMA (gemm_batched), tri-solve T Y + Y T^T = C~ as the
//      upper-triangular Sylvester form T Y' + Y' (P T^T P) = C~ P with the
//      tiled solver (one launch per tile anti-diagonal over all equations),
//      back-transform accumulated in binary64
//   5. refinement passes: R = C - AX - XA^T (binary64 MFMA), k_bnorm decides
//      per equation (converged / stalled / cap / NaN) and the scale 2^-e of R
//      for the binary32 correction.
// Symmetric specialisation (C symmetric to rounding, so X is symmetric):
// the iterate is kept exactly symmetric, the residual takes one product
// (C - W - W^T with W = A X), the second product of each transform forms
// only the tiles on or above the diagonal of its symmetric result (U^T R U,
// U Y U^T) and mirrors them, and the tri-solve computes one tile of each
// mirror pair of the persymmetric Y' = Y P and stores the other by mirroring.
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"
#include "../../include/sylv.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

namespace sylv {

constexpr int BNT = 256;   // threads of the per-equation kernels
constexpr int BSNT = 576;  // threads of the Schur kernel (9 waves: 4 left, 4 right, 1 overlap)

template <typename T>
SYLV_DEVINL T wg_sum(T v, T *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = T(0);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
}

// minimum over the workgroup (any sign)
template <typename T>
SYLV_DEVINL T wg_min(T v, T *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s = fmin(s, red[w]);
    __syncthreads();
    return s;
}

// maximum over the workgroup of non-negative values
template <typename T>
SYLV_DEVINL T wg_max(T v, T *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = T(0);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = fmax(s, red[w]);
    __syncthreads();
    return s;
}

// ------------------------------------------------------------ 1. prepare
// ||A||_F, ||C||_F, the symmetry test of C and the per-equation control
// fields.  With ||C - C^T||_F <= 2u ||C||_F (u = 2^-53) the solution is
// symmetric to working accuracy and the equation takes the symmetric
// specialisation (Lyapunov with symmetric right-hand side).
__global__ __launch_bounds__(BNT) void k_bprep(BatchEq *eqs, const int *order) {
    __shared__ double red[8];
    BatchEq &q = eqs[order[blockIdx.x]];
    const int n = q.n;
    const double *A = (const double *)q.ptr[BF_A];
    const double *C = (const double *)q.ptr[BF_C];
    const int lda = q.ld[BF_A], ldc = q.ld[BF_C];
    double sa = 0.0, sc = 0.0, sd = 0.0, mc = 0.0;
    for (int e = threadIdx.x; e < n * n; e += BNT) {
        const int i = e % n, j = e / n;
        const double a = A[(size_t)j * lda + i], c = C[(size_t)j * ldc + i];
        const double d = c - C[(size_t)i * ldc + j];
        sa += a * a;
        sc += c * c;
        sd += d * d;
        mc = fmax(mc, fabs(c));
    }
    sa = wg_sum(sa, red);
    sc = wg_sum(sc, red);
    sd = wg_sum(sd, red);
    mc = wg_max(mc, red);
    if (threadIdx.x == 0) {
        q.nA = sqrt(sa);
        q.nC = sqrt(sc);
        q.sym = sqrt(sd) <= 0x1p-52 * q.nC ? 1 : 0;
        q.active = 1;
        q.cls = -1;
        q.narrow = 0;
        q.status = SYLV_ST_NOT_CONVERGED;
        q.iterations = 0;
        q.qr_fail = 0;
        q.flag = 0;
        // C brought to [1/2, 1) by a power of two before the binary32 cast of
        // the first iterate (undone on the binary64 result)
        int ex = 0;
        frexp((mc > 0.0 && isfinite(mc)) ? mc : 1.0, &ex);
        q.scale = ldexp(1.0, -ex);
        q.rel_res = INFINITY;
        q.prev_rel = INFINITY;
        q.corr = 0.0;
        q.stall = 0;
    }
}

// ----------------------------------------------------------- 2. Hessenberg
// Householder reduction H = U0^T A U0 with the whole matrix held in
// registers: a G x G thread grid, thread (tx, ty) owning the R x R entries
// (tx + G a, ty + G b) (cyclic, so the shrinking trailing block stays spread
// over all threads; capacity G R).  For column c the G threads with
// ty = c mod G hold the column and build the reflector with lane shuffles;
// the left update P H needs column sums (a reduction over tx: lane shuffles
// inside a G-lane group), the right update H P row sums (a reduction over
// ty: shuffles inside the wave, then one pass through LDS).  Three barriers
// per column.  The reflectors go to global memory and U0 = P_0 ... P_{n-3}
// is accumulated backwards afterwards in the same registers (left updates
// only, no barrier).
template <int G, int R>
__global__ __launch_bounds__(G * G) void k_bhess_reg(BatchEq *eqs, const int *order, int first) {
    constexpr int NT = G * G, NW = NT / 64, NP = G * R, LDP = NP + 1;
    constexpr int TPW = 64 / G;  // ty rows per wave
    __shared__ float vs[2][NP];
    __shared__ float taus[2];
    __shared__ float zs[NP];
    __shared__ float P[NW][LDP];
    BatchEq &q = eqs[order[first + blockIdx.x]];
    const int n = q.n;
    const double *A = (const double *)q.ptr[BF_A];
    const int lda = q.ld[BF_A];
    float *Hg = (float *)q.ptr[BF_H];
    float *Ug = (float *)q.ptr[BF_U];
    float *Vg = (float *)q.ptr[BF_W];  // reflector c in column c, tau_c in column n-1
    const int t = threadIdx.x, tx = t % G, ty = t / G, lane = t & 63, wid = t >> 6;
    float h[R][R];
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) {
            const int i = tx + G * a, j = ty + G * b;
            h[a][b] = (i < n && j < n) ? (float)A[(size_t)j * lda + i] : 0.f;
        }
    for (int c = 0; c + 2 < n; ++c) {
        const int buf = c & 1;
        // ---- reflector from column c (owner group ty == c mod G)
        if (ty == c % G) {
            const int bc = c / G;
            float x[R];
#pragma unroll
            for (int a = 0; a < R; ++a) {
                x[a] = 0.f;
#pragma unroll
                for (int b = 0; b < R; ++b)
                    if (b == bc) x[a] = h[a][b];
            }
            float mx = 0.f, alpha = 0.f;
#pragma unroll
            for (int a = 0; a < R; ++a) {
                const int i = tx + G * a;
                if (i >= c + 2) mx = fmaxf(mx, fabsf(x[a]));
                if (i == c + 1) alpha = x[a];
            }
#pragma unroll
            for (int o = 1; o < G; o <<= 1) {
                mx = fmaxf(mx, __shfl_xor(mx, o));
                alpha += __shfl_xor(alpha, o);
            }
            float ss = 0.f;
            if (mx > 0.f) {
                const float rm = 1.f / mx;
#pragma unroll
                for (int a = 0; a < R; ++a) {
                    const int i = tx + G * a;
                    const float y = x[a] * rm;
                    if (i >= c + 2) ss += y * y;
                }
            }
#pragma unroll
            for (int o = 1; o < G; o <<= 1) ss += __shfl_xor(ss, o);
            float tau = 0.f, beta = alpha, scl = 0.f;
            if (mx > 0.f) {
                const float nrm = hypotf(alpha, mx * sqrtf(ss));
                beta = (alpha >= 0.f) ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scl = 1.f / (alpha - beta);
            }
#pragma unroll
            for (int a = 0; a < R; ++a) {
                const int i = tx + G * a;
                const float v = (i == c + 1) ? 1.f : (i >= c + 2 ? x[a] * scl : 0.f);
                vs[buf][i] = v;
                if (i < n) Vg[(size_t)c * n + i] = v;
                x[a] = (i == c + 1) ? beta : (i >= c + 2 ? 0.f : x[a]);
            }
#pragma unroll
            for (int a = 0; a < R; ++a)
#pragma unroll
                for (int b = 0; b < R; ++b)
                    if (b == bc) h[a][b] = x[a];
            if (tx == 0) {
                taus[buf] = tau;
                Vg[(size_t)(n - 1) * n + c] = tau;
            }
        }
        __syncthreads();
        const float tau = taus[buf];
        float vr[R], vc[R];
#pragma unroll
        for (int a = 0; a < R; ++a) vr[a] = vs[buf][tx + G * a];
#pragma unroll
        for (int b = 0; b < R; ++b) vc[b] = vs[buf][ty + G * b];
        // ---- left update on columns > c: column sums over the G-lane group
#pragma unroll
        for (int b = 0; b < R; ++b) {
            float p = 0.f;
#pragma unroll
            for (int a = 0; a < R; ++a) p += vr[a] * h[a][b];
#pragma unroll
            for (int o = 1; o < G; o <<= 1) p += __shfl_xor(p, o);
            const int j = ty + G * b;
            const float sj = (j > c) ? tau * p : 0.f;
#pragma unroll
            for (int a = 0; a < R; ++a) h[a][b] -= vr[a] * sj;
        }
        // ---- right update: row sums over ty (wave shuffles, then LDS)
        float zp[R];
#pragma unroll
        for (int a = 0; a < R; ++a) {
            float z = 0.f;
#pragma unroll
            for (int b = 0; b < R; ++b) z += h[a][b] * vc[b];
#pragma unroll
            for (int o = G; o < 64; o <<= 1) z += __shfl_xor(z, o);
            zp[a] = z;
        }
        if (lane < G) {
#pragma unroll
            for (int a = 0; a < R; ++a) P[wid][tx + G * a] = zp[a];
        }
        __syncthreads();
        if (t < NP) {
            float z = 0.f;
#pragma unroll
            for (int w = 0; w < NW; ++w) z += P[w][t];
            zs[t] = tau * z;
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < R; ++a) {
            const float zi = zs[tx + G * a];
#pragma unroll
            for (int b = 0; b < R; ++b) h[a][b] -= zi * vc[b];
        }
    }
    // Hessenberg form out (exact zeros below the subdiagonal)
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) {
            const int i = tx + G * a, j = ty + G * b;
            if (i < n && j < n) Hg[(size_t)j * n + i] = (i > j + 1) ? 0.f : h[a][b];
        }
    __syncthreads();  // reflectors written by other threads become visible
    // ---- U0 = P_0 P_1 ... P_{n-3}, accumulated backwards: U <- P_c U
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) h[a][b] = (tx + G * a == ty + G * b) ? 1.f : 0.f;
    for (int c = n - 3; c >= 0; --c) {
        float vr[R];
#pragma unroll
        for (int a = 0; a < R; ++a) {
            const int i = tx + G * a;
            vr[a] = (i > c && i < n) ? Vg[(size_t)c * n + i] : 0.f;
        }
        const float tau = Vg[(size_t)(n - 1) * n + c];
#pragma unroll
        for (int b = 0; b < R; ++b) {
            float p = 0.f;
#pragma unroll
            for (int a = 0; a < R; ++a) p += vr[a] * h[a][b];
#pragma unroll
            for (int o = 1; o < G; o <<= 1) p += __shfl_xor(p, o);
            const float sj = tau * p;
#pragma unroll
            for (int a = 0; a < R; ++a) h[a][b] -= vr[a] * sj;
        }
    }
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) {
            const int i = tx + G * a, j = ty + G * b;
            if (i < n && j < n) Ug[(size_t)j * n + i] = h[a][b];
        }
}

// ------------------------------------------------------ 3. band-LDS Schur
// Column j of the band holds rows 0..j+3 (the Hessenberg part plus the two
// extra subdiagonals a bulge occupies; slots past row n-1 in the last three
// columns are padding), so the offset is branch-free.
SYLV_DEVINL int band_off(int i, int j, int) { return ((j * (j + 7)) >> 1) + i; }
inline int band_size(int n) { return (n * (n + 7)) / 2; }
#define HB(i, j) Hb[band_off((i), (j), n)]

template <typename T>
SYLV_DEVINL void brefl(T v1, T v2, T tau, T &a0, T &a1, T &a2) {
    T s = (a0 + v1 * a1 + v2 * a2) * tau;
    a0 -= s;
    a1 -= s * v1;
    a2 -= s * v2;
}

__global__ __launch_bounds__(BSNT) void k_bschur(BatchEq *eqs, const int *order) {
    extern __shared__ unsigned char smem_raw[];
    float *Hb = reinterpret_cast<float *>(smem_raw);
    __shared__ float lv1[256], lv2[256], ltau[256];
    __shared__ int sint;
    BatchEq &q = eqs[order[blockIdx.x]];
    const int n = q.n;
    float *Hg = (float *)q.ptr[BF_H];
    float *U = (float *)q.ptr[BF_U];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    for (int j = 0; j < n; ++j) {
        const int rows = (j + 4 < n) ? j + 4 : n;
        for (int i = tid; i < rows; i += BSNT) HB(i, j) = (i <= j + 1) ? Hg[(size_t)j * n + i] : 0.f;
    }
    __syncthreads();
    const float ulp = num<float>::ulp, smlnum = num<float>::safmin * float(n) / num<float>::ulp;
    int ihi = n - 1, its = 0, total = 0, fail = 0, nsteps = 0, nsweeps = 0;
    double napply = 0.0;
    const long long c_start = clock64();
    long long c_sweep = 0, c_u = 0, c_scan = 0;
    const int itmax = 30 * (n > 10 ? n : 10);
    while (ihi >= 0) {
        const long long c0 = clock64();
        if (tid == 0) sint = 0;
        __syncthreads();
        // after 20 sweeps without a deflation the window is taken to have
        // stagnated (nearly coincident eigenvalues can hold binary32
        // subdiagonals near 1e-5 for hundreds of sweeps): subdiagonals below
        // sqrt(u) (|h_{k-1,k-1}| + |h_kk|) then deflate.  The backward error
        // of the form becomes ~sqrt(u); the binary64 refinement absorbs it.
        const float thr = (its >= 20) ? 2.44140625e-4f : ulp;  // 2^-12 = sqrt(2^-24)
        for (int k = 1 + tid; k <= ihi; k += BSNT) {
            float hk = fabsf(HB(k, k - 1));
            float tst = fabsf(HB(k - 1, k - 1)) + fabsf(HB(k, k));
            if (tst == 0.f) {
                if (k >= 2) tst += fabsf(HB(k - 1, k - 2));
                if (k + 1 <= ihi) tst += fabsf(HB(k + 1, k));
            }
            if (hk <= fmaxf(smlnum, thr * tst)) atomicMax(&sint, k);
        }
        __syncthreads();
        const int l = sint;
        __syncthreads();
        if (l > 0 && tid == 0) HB(l, l - 1) = 0.f;
        __syncthreads();
        c_scan += clock64() - c0;
        if (l == ihi) { ihi -= 1; its = 0; continue; }
        if (l == ihi - 1) {
            // converged 2x2 block: split it when its eigenvalues are real
            const int k = l;
            float a = HB(k, k), b = HB(k, k + 1), c = HB(k + 1, k), d = HB(k + 1, k + 1);
            __syncthreads();
            float p = 0.5f * (a - d), disc = p * p + b * c;
            if (c != 0.f && disc >= 0.f) {
                float e1 = p + copysignf(sqrtf(disc), p);
                float nv = hypotf(e1, c);
                float cs = e1 / nv, sn = c / nv;
                for (int j = k + tid; j < n; j += BSNT) {
                    float t1 = HB(k, j), t2 = HB(k + 1, j);
                    HB(k, j) = cs * t1 + sn * t2;
                    HB(k + 1, j) = cs * t2 - sn * t1;
                }
                __syncthreads();
                for (int i = tid; i <= k + 1; i += BSNT) {
                    float t1 = HB(i, k), t2 = HB(i, k + 1);
                    HB(i, k) = cs * t1 + sn * t2;
                    HB(i, k + 1) = cs * t2 - sn * t1;
                }
                for (int i = tid; i < n; i += BSNT) {
                    float *u0 = U + (size_t)k * n + i, *u1 = u0 + n;
                    const float t1 = *u0, t2 = *u1;
                    *u0 = cs * t1 + sn * t2;
                    *u1 = cs * t2 - sn * t1;
                }
                __syncthreads();
                if (tid == 0) HB(k + 1, k) = 0.f;
                __syncthreads();
            }
            ihi -= 2; its = 0;
            continue;
        }
        if (++total > itmax) { fail = 1; break; }
        ++its;
        ++nsweeps;
        const long long c1 = clock64();
        float h11 = HB(ihi - 1, ihi - 1), h12 = HB(ihi - 1, ihi);
        float h21 = HB(ihi, ihi - 1), h22 = HB(ihi, ihi);
        // exceptional shifts every 10 sweeps without a deflation, built from
        // the bottom of the window and, every 20, from its top (breaks the
        // cycles a stagnating window can fall into)
        if (its % 10 == 0) {
            const bool top = (its % 20 == 0);
            const float sx = top ? fabsf(HB(l + 1, l)) + fabsf(HB(l + 2, l + 1))
                                 : fabsf(HB(ihi, ihi - 1)) + fabsf(HB(ihi - 1, ihi - 2));
            h11 = 0.75f * sx + (top ? HB(l, l) : HB(ihi, ihi));
            h12 = -0.4375f * sx;
            h21 = sx;
            h22 = h11;
        }
        float x, y, z;
        {
            float sp, sq;
            bool cplx;
            shift_pair(h11, h12, h21, h22, sp, sq, cplx);
            shift_column(HB(l, l), HB(l, l + 1), HB(l + 1, l), HB(l + 1, l + 1), HB(l + 2, l + 1), sp, sq, cplx, x,
                         y, z);
        }
        __syncthreads();
        // The column a step reduces (k-1) is read by every thread at the top
        // of that step, so its final values (beta, 0, 0) are written one step
        // later, when no thread reads it.
        int pcol = -1, pk2 = 0;
        float pbeta = 0.f;
        for (int k = l; k <= ihi - 1; ++k) {
            const int len = (k <= ihi - 2) ? 3 : 2;
            const int k2 = (len == 3) ? k + 2 : k + 1;
            if (k > l) { x = HB(k, k - 1); y = HB(k + 1, k - 1); z = HB(k2, k - 1); }
            float v1, v2, tau, beta;
            reflector3(len, x, y, z, v1, v2, tau, beta);
            const int lc0 = (k > l) ? 1 : 0;
            // left on n-k-len+lc0+3 columns, right on k+3 (+1) rows, the orthogonal factor on n rows
            napply += double(2 * n + 6 - len + lc0 + ((len == 3 && k + 3 <= ihi) ? 1 : 0));
            ++nsteps;
            if (wv < 4) {
                // left: columns [k+len, n), rows k, k+1, k2, and the deferred
                // column of the previous step
                if (tid == 0 && pcol >= 0) {
                    HB(pk2, pcol) = 0.f;
                    HB(pcol + 2, pcol) = 0.f;
                    HB(pcol + 1, pcol) = pbeta;
                }
                const int nL = n - (k + len);
                for (int qq = tid; qq < nL; qq += 256) {
                    const int j = k + len + qq;
                    float a0 = HB(k, j), a1 = HB(k + 1, j), a2 = HB(k2, j);
                    brefl(v1, v2, tau, a0, a1, a2);
                    HB(k2, j) = a2; HB(k, j) = a0; HB(k + 1, j) = a1;
                }
            } else if (wv < 8) {
                // right: rows [0, k) u {k+3}, columns k, k+1, k2
                const int extra = (len == 3 && k + 3 <= ihi) ? 1 : 0;
                const int nR = k + extra;
                for (int qq = tid - 256; qq < nR; qq += 256) {
                    const int i = (qq < k) ? qq : k + 3;
                    float a0 = HB(i, k), a1 = HB(i, k + 1), a2 = HB(i, k2);
                    brefl(v1, v2, tau, a0, a1, a2);
                    HB(i, k2) = a2; HB(i, k) = a0; HB(i, k + 1) = a1;
                }
            } else if (lane == 0) {
                // overlap block rows/cols k, k+1, k2: left then right (k2 =
                // k+1 duplicates for a length-2 step: the duplicate is stored
                // first so the genuine value wins)
                const int ix[3] = {k, k + 1, k2};
                float b[3][3];
#pragma unroll
                for (int jj = 0; jj < 3; ++jj)
#pragma unroll
                    for (int ii = 0; ii < 3; ++ii) b[ii][jj] = HB(ix[ii], ix[jj]);
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) brefl(v1, v2, tau, b[0][jj], b[1][jj], b[2][jj]);
#pragma unroll
                for (int ii = 0; ii < 3; ++ii) brefl(v1, v2, tau, b[ii][0], b[ii][1], b[ii][2]);
#pragma unroll
                for (int jj = 2; jj >= 0; --jj)
#pragma unroll
                    for (int ii = 2; ii >= 0; --ii) HB(ix[ii], ix[jj]) = b[ii][jj];
                lv1[k] = v1; lv2[k] = v2; ltau[k] = tau;
            }
            __syncthreads();
            pcol = (k > l) ? k - 1 : -1;
            pbeta = beta;
            pk2 = k2;
        }
        if (tid == 0 && pcol >= 0) {
            HB(pk2, pcol) = 0.f;
            HB(pcol + 2, pcol) = 0.f;
            HB(pcol + 1, pcol) = pbeta;
        }
        const long long c2 = clock64();
        c_sweep += c2 - c1;
        // apply the sweep's reflectors to the rows of U (column-major: a
        // wave's loads and stores are contiguous), each thread streaming one
        // row through a three-entry register window; the entries ahead are
        // fetched 8 at a time so their loads overlap
        for (int i = tid; i < n; i += BSNT) {
            float *ur = U + i;
            float z0 = ur[(size_t)l * n], z1 = ur[(size_t)(l + 1) * n];
            for (int k0 = l; k0 <= ihi - 1; k0 += 8) {
                float ahead[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int c = k0 + 2 + r;
                    ahead[r] = (c <= ihi) ? ur[(size_t)c * n] : 0.f;
                }
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int k = k0 + r;
                    if (k <= ihi - 1) {
                        float z2 = ahead[r];
                        brefl(lv1[k], lv2[k], ltau[k], z0, z1, z2);
                        ur[(size_t)k * n] = z0;
                        z0 = z1;
                        z1 = z2;
                    }
                }
            }
            ur[(size_t)ihi * n] = z0;
        }
        __syncthreads();
        c_u += clock64() - c2;
    }
    __syncthreads();
    // T back to global (dense, exact zeros below the first subdiagonal)
    for (int e = tid; e < n * n; e += BSNT) {
        const int i = e % n, j = e / n;
        Hg[e] = (i <= j + 1) ? HB(i, j) : 0.f;
    }
    if (tid == 0) {
        q.steps = nsteps;
        q.napply = napply;
        q.sweeps = nsweeps;
        q.cyc[0] = clock64() - c_start;
        q.cyc[1] = c_sweep;
        q.cyc[2] = c_u;
        q.cyc[3] = c_scan;
    }
    if (tid == 0 && fail) {
        q.qr_fail = 1;
        q.status = SYLV_ST_QR_FAILED;
        q.active = 0;
    }
}
#undef HB

// ------------------------------------- 4. right factor of the tri-solve
// With the reversal permutation P, T Y + Y T^T = W becomes
// T Y' + Y' (P T^T P) = W P with Y = Y' P; P T^T P is upper quasi-triangular,
// so the Sylvester tile solver applies.  W P and Y' P are folded into the
// transforms by V = U P:  W P = U^T C V,  X = U Y' V^T.
// V = U P, TB = P T^T P, max |T_ij| and the largest eigenvalue modulus of T
// (from its 1x1 and 2x2 diagonal blocks)
__global__ __launch_bounds__(BNT) void k_bpost(BatchEq *eqs, const int *order) {
    __shared__ float red[8];
    BatchEq &q = eqs[order[blockIdx.x]];
    if (!q.active) return;
    const int n = q.n;
    const float *T = (const float *)q.ptr[BF_H];
    const float *U = (const float *)q.ptr[BF_U];
    float *V = (float *)q.ptr[BF_V];
    float *TB = (float *)q.ptr[BF_TB];
    float mx = 0.f;
    for (int e = threadIdx.x; e < n * n; e += BNT) {
        const int i = e % n, j = e / n;
        V[e] = U[(size_t)(n - 1 - j) * n + i];
        TB[e] = T[(size_t)(n - 1 - i) * n + (n - 1 - j)];
        mx = fmaxf(mx, fabsf(T[e]));
    }
    float lm = 0.f;
    for (int i = threadIdx.x; i < n; i += BNT) {
        const bool lower = i > 0 && T[(size_t)(i - 1) * n + i] != 0.f;
        const bool upper = i + 1 < n && T[(size_t)i * n + i + 1] != 0.f;
        if (!lower && !upper) { lm = fmaxf(lm, fabsf(T[(size_t)i * n + i])); continue; }
        const int k = upper ? i : i - 1;
        const double a = T[(size_t)k * n + k], b = T[(size_t)(k + 1) * n + k];
        const double c = T[(size_t)k * n + k + 1], d = T[(size_t)(k + 1) * n + k + 1];
        const double p = 0.5 * (a - d), disc = p * p + b * c, mid = 0.5 * (a + d);
        const double mod = disc >= 0.0 ? fabs(mid) + sqrt(disc) : sqrt(mid * mid - disc);
        lm = fmaxf(lm, (float)mod);
    }
    mx = wg_max(mx, red);
    lm = wg_max(lm, red);
    if (threadIdx.x == 0) {
        q.tmax = (double)mx;
        q.lmax = (double)lm;
    }
}

// Randomised estimate of ||U^T U - I||_F per equation (Hutchinson's trace
// estimator of ||E||_F^2, E = U^T U - I): 8 probe columns z_k with entries
// +-1/sqrt(8) from a counter-based hash (splitmix64 finaliser) of (equation,
// entry); w_k = U z_k, then ||U^T w_k - z_k|| summed over k, in binary64
// (binary32 U entries are exact in binary64).  O(16 n^2) flops per equation.
constexpr int BPROBES = 8;
__global__ __launch_bounds__(BNT) void k_borth(BatchEq *eqs, const int *order) {
    __shared__ double wz[BPROBES][256];
    __shared__ double red[8];
    const int slot = order[blockIdx.x];
    BatchEq &q = eqs[slot];
    if (!q.active) return;
    const int n = q.n;
    const float *U = (const float *)q.ptr[BF_U];
    auto z = [&](int i, int k) {
        unsigned long long x = ((unsigned long long)(slot + 1) << 24) ^ (unsigned long long)(i * BPROBES + k);
        x += 0x9e3779b97f4a7c15ull;
        x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
        x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
        x ^= x >> 31;
        return (x & 1ull) ? 0.35355339059327373 : -0.35355339059327373;
    };
    for (int i = threadIdx.x; i < n; i += BNT) {
        double w[BPROBES];
#pragma unroll
        for (int k = 0; k < BPROBES; ++k) w[k] = 0.0;
        for (int j = 0; j < n; ++j) {
            const double u = (double)U[(size_t)j * n + i];
#pragma unroll
            for (int k = 0; k < BPROBES; ++k) w[k] += u * z(j, k);
        }
#pragma unroll
        for (int k = 0; k < BPROBES; ++k) wz[k][i] = w[k];
    }
    __syncthreads();
    double acc = 0.0;
    for (int j = threadIdx.x; j < n; j += BNT) {
        double e[BPROBES];
#pragma unroll
        for (int k = 0; k < BPROBES; ++k) e[k] = -z(j, k);
        for (int i = 0; i < n; ++i) {
            const double u = (double)U[(size_t)j * n + i];
#pragma unroll
            for (int k = 0; k < BPROBES; ++k) e[k] += u * wz[k][i];
        }
#pragma unroll
        for (int k = 0; k < BPROBES; ++k) acc += e[k] * e[k];
    }
    acc = wg_sum(acc, red);
    if (threadIdx.x == 0) q.orth = sqrt(acc);
}

// --------------------------------------- 5. residual norms and loop control
// R = C (general), or R = 0 ahead of the one-product symmetric residual
__global__ __launch_bounds__(BNT) void k_bcopy_c(BatchEq *eqs, const int *order) {
    BatchEq &q = eqs[order[blockIdx.x]];
    if (!q.active) return;
    const int n = q.n;
    const double *C = (const double *)q.ptr[BF_C];
    double *R = (double *)q.ptr[BF_R];
    const int ldc = q.ld[BF_C];
    if (q.sym)
        for (int e = threadIdx.x; e < n * n; e += BNT) R[e] = 0.0;
    else
        for (int e = threadIdx.x; e < n * n; e += BNT) R[e] = C[(size_t)(e / n) * ldc + e % n];
}

// Symmetric specialisation: with X = X^T, X A^T = (A X)^T, so after
// R = -A X the residual is C - A X - X A^T = C + R + R^T (one product
// instead of two).  grid.x = tile pair, grid.y = equation slot.
__global__ __launch_bounds__(256) void k_bsymres(BatchEq *eqs, const int *order) {
    __shared__ double sa[32][33], sb[32][33];
    BatchEq &q = eqs[order[blockIdx.y]];
    if (!q.active || !q.sym) return;
    const int n = q.n;
    if ((int)blockIdx.x >= sym_pair_count(n)) return;
    int ti, tj;
    sym_pair_index(blockIdx.x, ti, tj);
    sym_tile_pair(true, n, (const double *)q.ptr[BF_C], q.ld[BF_C], (double *)q.ptr[BF_R], n, ti, tj, sa, sb);
}


__global__ __launch_bounds__(BNT) void k_bnorm(BatchEq *eqs, const int *order, double tol,
                                               int max_iter, int *nactive) {
    __shared__ double red[8];
    BatchEq &q = eqs[order[blockIdx.x]];
    if (!q.active) return;
    const int n = q.n;
    const double *R = (const double *)q.ptr[BF_R];
    const double *X = (const double *)q.ptr[BF_X];
    const int ldx = q.ld[BF_X];
    double sr = 0.0, mr = 0.0, sx = 0.0;
    for (int e = threadIdx.x; e < n * n; e += BNT) {
        const double r = R[e], x = X[(size_t)(e / n) * ldx + e % n];
        sr += r * r;
        mr = fmax(mr, fabs(r));
        sx += x * x;
        if (r != r) mr = r;
    }
    sr = wg_sum(sr, red);
    sx = wg_sum(sx, red);
    mr = wg_max(mr, red);
    if (threadIdx.x == 0) {
        // accepted when rel <= tol and the forward error it implies is at the
        // binary64 level: rel * (2||A||_F + ||C||_F / ||X||_F) <= 100 u max|l_i + l_j|
        // (the rule of the single-equation refinement; max|l_i + l_j| = 2 lmax)
        const double nx = sqrt(sx);
        const double rel = sqrt(sr) / (q.nC + nx * 2.0 * q.nA);
        const bool at_tol = rel <= tol;
        const double growth = 2.0 * q.nA + (nx > 0.0 ? q.nC / nx : 0.0);
        const bool fwd_ok = rel * growth <= 100.0 * 0x1p-53 * 2.0 * q.lmax;
        const int ok_status = q.flag ? SYLV_ST_PERTURBED : SYLV_OK;
        q.rel_res = rel;
        int done = 0;
        if (!(rel == rel) || !isfinite(rel) || !(mr == mr)) { q.status = SYLV_ST_NAN; done = 1; }
        else if (at_tol && fwd_ok) { q.status = ok_status; done = 1; }
        else if (q.iterations >= max_iter) { q.status = at_tol ? ok_status : SYLV_ST_NOT_CONVERGED; done = 1; }
        else {
            if (rel > 0.5 * q.prev_rel) {
                if (++q.stall >= (at_tol ? 1 : 2)) {
                    q.status = at_tol ? ok_status : SYLV_ST_NOT_CONVERGED;
                    done = 1;
                }
            } else {
                q.stall = 0;
            }
        }
        q.prev_rel = rel;
        if (done) q.active = 0;
        else {
            int ex = 0;
            frexp(mr > 0.0 ? mr : 1.0, &ex);
            q.scale = ldexp(1.0, -ex);
            q.iterations += 1;  // one correction is about to be applied
            atomicAdd(nactive, 1);
        }
    }
}

}  // namespace sylv

namespace sylv {

// ------------------------------------------------------- launch sequences
__global__ void k_bzero(int *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// 32 x 32 tile pairs (ti <= tj) of an order-n matrix
static int sym_pairs(int n) {
    const int nt = (n + 31) / 32;
    return nt * (nt + 1) / 2;
}

struct BatchPlan {
    BatchEq *deq;
    int *dord, *dcnt;
    int batch, nmax, bf16, max_iter;
    double tol;
    int h1, h2;       // Hessenberg buckets [0,h1) [h1,h2) [h2,batch)
    int orth;         // orthogonality probe of the binary32 Schur vectors
    int autosel;      // learned precision choice per equation (SYLV_PREC_AUTO)
    float *feat, *zfeat, *prob;  // selector features (batch x 16, raw and standardised), class probabilities
    const float *sel;            // device selector blob: params | means | standard deviations
    int nsb;          // band-QR buckets [sb[i], sb[i+1]), i < nsb
    int sb[5];
    size_t smem[4];   // their dynamic LDS
};

// Tunables of the batched path (process-wide; the defaults are what the
// project's autotuner measured best on MI355X for the 4096-equation
// Lyapunov batch): Hessenberg kernel buckets (orders > hess_hi take the
// 32 x 32-thread register kernel, orders in (hess_lo, hess_hi] the 16 x 16 one
// with 8 x 8 entries per thread, the rest 4 x 4), the band-QR LDS buckets
// (each bucket's launch reserves the band of its largest order: orders above
// band[0], then (band[1], band[0]], ...; a zero ends the list) and the passes
// per captured refinement graph.
struct BatchTune {
    int hess_hi = 64, hess_lo = 48;
    int band[3] = {180, 128, 0};
    int gpasses = 3;
};
static std::mutex g_btune_mu;
static BatchTune g_btune;

static BatchTune batch_tune() {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    return g_btune;
}

// Symmetric equations: lower triangle of X <- its upper triangle (the
// back-transform formed only the tiles on or above the diagonal).
// grid.x = 32 x 32 tile pair, grid.y = equation slot.
__global__ __launch_bounds__(256) void k_bmirror_x(BatchEq *eqs, const int *order) {
    __shared__ double t[32][33];
    BatchEq &q = eqs[order[blockIdx.y]];
    if (!q.active || !q.sym) return;
    const int n = q.n;
    if ((int)blockIdx.x >= sym_pair_count(n)) return;
    int ti, tj;
    sym_pair_index(blockIdx.x, ti, tj);
    double *X = (double *)q.ptr[BF_X];
    const int ldx = q.ld[BF_X];
    const int r0 = 32 * ti, c0 = 32 * tj;
    for (int e = threadIdx.x; e < 1024; e += 256) {
        const int ii = e & 31, jj = e >> 5;
        if (r0 + ii < n && c0 + jj < n) t[jj][ii] = X[(size_t)(c0 + jj) * ldx + r0 + ii];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256) {
        const int ii = e & 31, jj = e >> 5;
        const int gi = c0 + ii, gj = r0 + jj;
        if (gi < n && gj < n && gi > gj) X[(size_t)gj * ldx + gi] = t[ii][jj];
    }
}

// Symmetric equations: W = S P, S the symmetric matrix whose upper triangle
// is that of the binary32 product held in the R buffer (U^T R U, upper tiles
// only), P the reversal permutation.  One workgroup per equation.
__global__ __launch_bounds__(BNT) void k_bsym_fwd(BatchEq *eqs, const int *order) {
    BatchEq &q = eqs[order[blockIdx.x]];
    if (!q.active || !q.sym) return;
    const int n = q.n;
    const float *S = (const float *)q.ptr[BF_R];
    float *W = (float *)q.ptr[BF_W];
    for (int e = threadIdx.x; e < n * n; e += BNT) {
        const int i = e % n, j = e / n, c = n - 1 - j;
        W[e] = (i <= c) ? S[(size_t)c * n + i] : S[(size_t)i * n + c];
    }
}

// The 16 selector features of every equation (the single-equation
// definitions with B = A^T, so the two spectra are the same): log2 n twice,
// log10 ||A||_F / sqrt n twice, log10 ||C||_F / n, log10 sep_est with
// sep_est = min |l_i + l_j|, log10 (2 ||A||_F / sep_est), the Henrici
// departure ||N||_F / ||T||_F twice, the fraction of eigenvalues in complex
// pairs twice, log10 of min_{i != j} |l_i - l_j| / max |l_i| twice, log10 of
// the orthogonality probe twice, and the Lyapunov flag.  Eigenvalues from the
// 1x1 / 2x2 diagonal blocks of the binary32 T.  Row slot of the batch order.
__global__ __launch_bounds__(BNT) void k_bfeatures(BatchEq *eqs, const int *order, float *feat) {
    __shared__ float wr[256], wi[256];
    __shared__ double red[8];
    const int slot = blockIdx.x;
    BatchEq &q = eqs[order[slot]];
    float *f = feat + (size_t)slot * 16;
    const int n = q.n;
    const float *T = (const float *)q.ptr[BF_H];
    for (int i = threadIdx.x; i < n; i += BNT) {
        const bool lower = i > 0 && T[(size_t)(i - 1) * n + i] != 0.f;
        const bool upper = i + 1 < n && T[(size_t)i * n + i + 1] != 0.f;
        if (!lower && !upper) { wr[i] = T[(size_t)i * n + i]; wi[i] = 0.f; continue; }
        const int k = upper ? i : i - 1;
        const double a = T[(size_t)k * n + k], b = T[(size_t)(k + 1) * n + k];
        const double c = T[(size_t)k * n + k + 1], d = T[(size_t)(k + 1) * n + k + 1];
        const double p = 0.5 * (a - d), disc = p * p + b * c, mid = 0.5 * (a + d);
        if (disc >= 0.0) { const double r = sqrt(disc); wr[i] = (float)(upper ? mid + r : mid - r); wi[i] = 0.f; }
        else { const double r = sqrt(-disc); wr[i] = (float)mid; wi[i] = (float)(upper ? r : -r); }
    }
    __syncthreads();
    double sep = 1e300, gap = 1e300, mx = 0.0, ncx = 0.0, bd = 0.0, tf = 0.0;
    for (int e = threadIdx.x; e < n * n; e += BNT) {
        const int i = e % n, j = e / n;
        const double sr = (double)wr[i] + wr[j], si = (double)wi[i] + wi[j];
        sep = fmin(sep, sqrt(sr * sr + si * si));
        if (i < j) {
            const double dr = (double)wr[i] - wr[j], di = (double)wi[i] - wi[j];
            gap = fmin(gap, sqrt(dr * dr + di * di));
        }
        const double t = T[e];
        tf += t * t;
    }
    for (int i = threadIdx.x; i < n; i += BNT) {
        if (wi[i] != 0.f) ncx += 1.0;
        mx = fmax(mx, sqrt((double)wr[i] * wr[i] + (double)wi[i] * wi[i]));
        const double d = T[(size_t)i * n + i];
        bd += d * d;
        if (i + 1 < n && T[(size_t)i * n + i + 1] != 0.f) {
            const double b = T[(size_t)(i + 1) * n + i], c = T[(size_t)i * n + i + 1];
            bd += b * b + c * c;
        }
    }
    sep = wg_min(sep, red);
    gap = wg_min(gap, red);
    mx = wg_max(mx, red);
    ncx = wg_sum(ncx, red);
    bd = wg_sum(bd, red);
    tf = wg_sum(tf, red);
    if (threadIdx.x == 0) {
        auto lg = [](double x) { return log10(fmax(x, 1e-300)); };
        const double s = fmax(sep, 1e-300);
        const double tfn = sqrt(tf);
        const double hen = tfn > 0.0 ? sqrt(fmax(tf - bd, 0.0)) / tfn : 0.0;
        const double rg = n > 1 ? lg(gap / fmax(mx, 1e-300)) : 0.0;
        f[0] = f[1] = (float)log2((double)n);
        f[2] = f[3] = (float)lg(q.nA / sqrt((double)n));
        f[4] = (float)lg(q.nC / (double)n);
        f[5] = (float)lg(s);
        f[6] = (float)lg(2.0 * q.nA / s);
        f[7] = f[8] = (float)hen;
        f[9] = f[10] = (float)(ncx / n);
        f[11] = f[12] = (float)rg;
        f[13] = f[14] = (float)lg(q.orth);
        f[15] = 1.f;
    }
}

// Class of every equation from the network's probabilities: 0 bfloat16-input
// transforms, 1 binary32, 2 plain binary64 (the equation leaves the batch and
// is solved by the single-equation binary64 path).  In a batch a refinement
// that stalls costs only its share of batch-wide passes (about 0.5 ms per
// equation at 1024 equations), while a needless binary64 re-solve costs a
// whole single-equation solve (about 10 ms at these orders), so class 2 is
// taken only when p2 > 20 p1 (log-score offset -ln 20 = -3).
constexpr float kBatchClass2Offset = -3.0f;
__global__ void k_bchoose(BatchEq *eqs, const int *order, int batch, const float *prob) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= batch) return;
    BatchEq &q = eqs[order[slot]];
    const float *p = prob + (size_t)slot * 3;
    float sc[3];
    for (int k = 0; k < 3; ++k) sc[k] = logf(fmaxf(p[k], 1e-30f));
    sc[2] += kBatchClass2Offset;
    int c = 0;
    if (sc[1] > sc[c]) c = 1;
    if (sc[2] > sc[c]) c = 2;
    q.cls = c;
    q.narrow = c == 0 ? 1 : 0;
    if (c == 2) {
        q.active = 0;
        q.status = SYLV_ST_NOT_CONVERGED;
    }
}

// selector inside the front of the batch: features, standardisation, one
// forward pass over the batch, class per equation
static void enqueue_selector(hipStream_t s, const BatchPlan &P) {
    hipLaunchKernelGGL(k_bfeatures, dim3(P.batch), dim3(BNT), 0, s, P.deq, P.dord, P.feat);
    mlp_standardize(s, P.batch, P.feat, P.sel + SYLV_MLP_NPARAM, P.sel + SYLV_MLP_NPARAM + SYLV_NFEAT, P.zfeat);
    sylv_mlp_forward(P.batch, P.zfeat, P.sel, P.prob, s);
    hipLaunchKernelGGL(k_bchoose, dim3((P.batch + 255) / 256), dim3(256), 0, s, P.deq, P.dord, P.batch, P.prob);
}

// A transform product of the batch in binary32 arithmetic.  Without the
// selector every equation takes the precision option's operand format
// (P.bf16); with the selector (P.autosel) the product runs twice, binary32
// operands for the equations of class 1 (amode bit 64) and bfloat16 ones for
// class 0 (bit 32): each launch skips the other equations at once.
template <typename TA, typename TB, typename TC>
static void tgemm(hipStream_t s, const BatchPlan &P, int fa, int ta, int fb, int tb, int fc, double alpha,
                  int amode, float beta) {
    if (!P.autosel) {
        gemm_batched<TA, TB, TC, float>(s, P.deq, P.dord, P.batch, P.nmax, fa, ta, fb, tb, fc, alpha, amode, beta,
                                        P.bf16);
        return;
    }
    gemm_batched<TA, TB, TC, float>(s, P.deq, P.dord, P.batch, P.nmax, fa, ta, fb, tb, fc, alpha, amode | 64, beta,
                                    0);
    gemm_batched<TA, TB, TC, float>(s, P.deq, P.dord, P.batch, P.nmax, fa, ta, fb, tb, fc, alpha, amode | 32, beta,
                                    1);
}

// second product of the forward transform, W = Y V: in full for general
// equations; for symmetric ones Y U = U^T R U is symmetric, so only its
// tiles on or above the diagonal are formed (into the free R buffer) and W
// is read off their mirror with the column reversal of V = U P
static void second_forward_product(hipStream_t s, const BatchPlan &P) {
    tgemm<float, float, float>(s, P, BF_Y, 0, BF_V, 0, BF_W, 1.0, 4, 0.f);
    tgemm<float, float, float>(s, P, BF_Y, 0, BF_U, 0, BF_R, 1.0, 8 | 16, 0.f);
    hipLaunchKernelGGL(k_bsym_fwd, dim3(P.batch), dim3(BNT), 0, s, P.deq, P.dord);
}

// stages 1-4 and the first iterate
static void enqueue_front(hipStream_t s, const BatchPlan &P) {
    const int batch = P.batch;
    hipLaunchKernelGGL(k_bprep, dim3(batch), dim3(BNT), 0, s, P.deq, P.dord);
    {
        ProfScope ps(KID_BHESS, s);
        if (P.h1 > 0) hipLaunchKernelGGL((k_bhess_reg<32, 8>), dim3(P.h1), dim3(1024), 0, s, P.deq, P.dord, 0);
        if (P.h2 > P.h1)
            hipLaunchKernelGGL((k_bhess_reg<16, 8>), dim3(P.h2 - P.h1), dim3(256), 0, s, P.deq, P.dord, P.h1);
        if (batch > P.h2)
            hipLaunchKernelGGL((k_bhess_reg<16, 4>), dim3(batch - P.h2), dim3(256), 0, s, P.deq, P.dord, P.h2);
    }
    {
        ProfScope ps(KID_BSCHUR, s);
        for (int bi = 0; bi < P.nsb; ++bi)
            if (P.sb[bi + 1] > P.sb[bi])
                hipLaunchKernelGGL(k_bschur, dim3(P.sb[bi + 1] - P.sb[bi]), dim3(BSNT), P.smem[bi], s, P.deq,
                                   P.dord + P.sb[bi]);
    }
    hipLaunchKernelGGL(k_bpost, dim3(batch), dim3(BNT), 0, s, P.deq, P.dord);
    if (P.orth) hipLaunchKernelGGL(k_borth, dim3(batch), dim3(BNT), 0, s, P.deq, P.dord);
    // first iterate: W = U^T (2^-e C) V, Y' solves T Y' + Y' TB = W, X = 2^e U Y' V^T
    if (P.autosel) enqueue_selector(s, P);
    tgemm<float, double, float>(s, P, BF_U, 1, BF_C, 0, BF_Y, 1.0, 1, 0.f);
    second_forward_product(s, P);
    trsyl_batched(s, P.deq, P.dord, batch, P.nmax);
    tgemm<float, float, float>(s, P, BF_U, 0, BF_W, 0, BF_Y, 1.0, 0, 0.f);
    tgemm<float, float, double>(s, P, BF_Y, 0, BF_V, 1, BF_X, 1.0, 2 | 8, 0.f);
    hipLaunchKernelGGL(k_bmirror_x, dim3(sym_pairs(P.nmax), batch), dim3(256), 0, s, P.deq, P.dord);
}

// binary64 residual R = C - A X - X A^T (one product for symmetric
// equations), norms and the per-equation decision;
// *dcnt = number of equations that take another correction
static void enqueue_pass(hipStream_t s, const BatchPlan &P, bool) {
    const int batch = P.batch;
    hipLaunchKernelGGL(k_bcopy_c, dim3(batch), dim3(BNT), 0, s, P.deq, P.dord);
    gemm_batched<double, double, double, double>(s, P.deq, P.dord, batch, P.nmax, BF_A, 0, BF_X, 0, BF_R, -1.0, 0,
                                                 1.0);
    gemm_batched<double, double, double, double>(s, P.deq, P.dord, batch, P.nmax, BF_X, 0, BF_A, 1, BF_R, -1.0, 4,
                                                 1.0);
    hipLaunchKernelGGL(k_bsymres, dim3(sym_pairs(P.nmax), batch), dim3(256), 0, s, P.deq, P.dord);
    hipLaunchKernelGGL(k_bzero, dim3(1), dim3(64), 0, s, P.dcnt);
    hipLaunchKernelGGL(k_bnorm, dim3(batch), dim3(BNT), 0, s, P.deq, P.dord, P.tol, P.max_iter, P.dcnt);
}

// correction of the active equations: W = 2^-e U^T R V, tri-solve,
// X += 2^e U Y' V^T
static void enqueue_correction(hipStream_t s, const BatchPlan &P) {
    const int batch = P.batch;
    tgemm<float, double, float>(s, P, BF_U, 1, BF_R, 0, BF_Y, 1.0, 1, 0.f);
    second_forward_product(s, P);
    trsyl_batched(s, P.deq, P.dord, batch, P.nmax);
    tgemm<float, float, float>(s, P, BF_U, 0, BF_W, 0, BF_Y, 1.0, 0, 0.f);
    tgemm<float, float, double>(s, P, BF_Y, 0, BF_V, 1, BF_X, 1.0, 2 | 8, 1.f);
    hipLaunchKernelGGL(k_bmirror_x, dim3(sym_pairs(P.nmax), batch), dim3(256), 0, s, P.deq, P.dord);
}

// ------------------------------------------------------------- hipGraph
// The launch sequence of a batch shape is captured once on an internal
// stream and replayed, as two graphs: the front graph (stages, first
// iterate, then `passes` refinement passes, each a residual with the
// per-equation decision followed by a correction) and the tail graph
// (`passes` more passes).  Equations are gated on the device (inactive ones
// return at once), so the graphs need no host decisions; the host reads one
// counter after each graph -- the number of equations the last pass sent to
// another correction -- and replays the tail graph while it is nonzero.  The
// per-equation cap of max_iter corrections ends every equation, so the
// whole refinement runs from graphs.  A graph pair is keyed by the
// workspace, the sorted orders and the options it was captured with.
// SYLV_BATCH_GRAPH=0 in the environment selects eager launches.
struct BatchGraph {
    hipStream_t gs = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    BatchEq *deq = nullptr;
    int passes = 0, bf16 = 0, max_iter = 0, orth = 0, autosel = 0;
    double tol = 0.0;
    std::vector<int> sizes;
    int tune[6] = {0, 0, 0, 0, 0, 0};  // batched tunables the graphs were captured with
};
static BatchGraph g_bgraph[64];

static bool batch_graph_enabled() {
    const char *v = std::getenv("SYLV_BATCH_GRAPH");
    return !(v && v[0] == '0');
}

// Capture of graph `which` (0 front, 1 tail) on g.gs.
static hipError_t batch_graph_capture(BatchGraph &g, const BatchPlan &P, int passes, int which) {
    hipError_t e;
    if ((e = hipStreamBeginCapture(g.gs, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    if (which == 0) enqueue_front(g.gs, P);
    for (int k = 0; k < passes; ++k) {
        enqueue_pass(g.gs, P, true);
        enqueue_correction(g.gs, P);
    }
    if ((e = hipStreamEndCapture(g.gs, &g.graph[which])) != hipSuccess) return e;
    if ((e = hipGraphInstantiate(&g.exec[which], g.graph[which], nullptr, nullptr, 0)) != hipSuccess) {
        hipGraphDestroy(g.graph[which]);
        g.graph[which] = nullptr;
        g.exec[which] = nullptr;
    }
    return e;
}

// Replays graph `which` (0 front, 1 tail) for this batch on stream s and
// reads the pending-correction counter into *hcnt.
static int batch_graph_run(hipStream_t s, const BatchPlan &P, const std::vector<int> &order, const int *nn,
                           int passes, int which, int *dcnt, int *hcnt) {
    int dev = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess || dev < 0 || dev >= 64) return SYLV_ERR_NOGPU;
    BatchGraph &g = g_bgraph[dev];
    if (!g.gs) {
        if ((e = hipStreamCreateWithFlags(&g.gs, hipStreamNonBlocking)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
        if ((e = hipEventCreateWithFlags(&g.e0, hipEventDisableTiming)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
        if ((e = hipEventCreateWithFlags(&g.e1, hipEventDisableTiming)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
    }
    std::vector<int> sizes(P.batch);
    for (int i = 0; i < P.batch; ++i) sizes[i] = nn[order[i]];
    int tv[6];
    batch_tune_get(tv);
    const bool same = g.deq == P.deq && g.passes == passes && g.bf16 == P.bf16 && g.max_iter == P.max_iter &&
                      g.tol == P.tol && g.orth == P.orth && g.autosel == P.autosel && g.sizes == sizes &&
                      std::equal(tv, tv + 6, g.tune);
    if (!same) {
        for (int k = 0; k < 2; ++k)
            if (g.exec[k]) {
                hipGraphExecDestroy(g.exec[k]);
                hipGraphDestroy(g.graph[k]);
                g.exec[k] = nullptr;
                g.graph[k] = nullptr;
            }
        g.deq = P.deq;
        g.passes = passes;
        g.bf16 = P.bf16;
        g.max_iter = P.max_iter;
        g.tol = P.tol;
        g.orth = P.orth;
        g.autosel = P.autosel;
        g.sizes = std::move(sizes);
        std::copy(tv, tv + 6, g.tune);
    }
    if (!g.exec[which] && (e = batch_graph_capture(g, P, passes, which)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
    if ((e = hipEventRecord(g.e0, s)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
    if ((e = hipStreamWaitEvent(g.gs, g.e0, 0)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
    if ((e = hipGraphLaunch(g.exec[which], g.gs)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
    if ((e = hipEventRecord(g.e1, g.gs)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
    if ((e = hipStreamWaitEvent(s, g.e1, 0)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
    if ((e = hipMemcpyAsync(hcnt, dcnt, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return SYLV_ERR_HIP - (int)e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
    return 0;
}

// Host driver.  All equations must be Lyapunov with order <= 256.
int lyap_batched(hipStream_t s, int batch, const int *nn, const double *const *A, const int *lda,
                 const double *const *C, const int *ldc, double *const *X, const int *ldx,
                 const sylv_opts &o, sylv_info *infos, void *work, size_t work_bytes, char *hbuf) {
    std::vector<int> order(batch);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nn[a] > nn[b]; });
    int nmax = 0;
    size_t ws_f = 0, ws_d = 0;
    for (int i = 0; i < batch; ++i) {
        nmax = std::max(nmax, nn[i]);
        ws_f += 6 * (size_t)nn[i] * nn[i];
        ws_d += (size_t)nn[i] * nn[i];
    }
    // workspace layout: [descriptors][order][counter][binary64 R...][binary32 H, U, W, Y ...]
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o2 = (off + 255) & ~(size_t)255; off = o2 + bytes; return o2; };
    const size_t o_eq = take(sizeof(BatchEq) * batch);
    const size_t o_ord = take(sizeof(int) * batch);
    const size_t o_cnt = take(64);
    const size_t o_d = take(sizeof(double) * ws_d);
    const size_t o_f = take(sizeof(float) * ws_f);
    const size_t o_sel = take(sizeof(float) * (size_t)batch * (2 * SYLV_NFEAT + SYLV_NCLASS));
    if (work_bytes < off) return -1;
    char *base = (char *)work;
    std::vector<BatchEq> hq(batch);
    double *pd = (double *)(base + o_d);
    float *pf = (float *)(base + o_f);
    for (int i = 0; i < batch; ++i) {
        BatchEq &q = hq[i];
        std::memset(&q, 0, sizeof(q));
        const int n = nn[i];
        const size_t n2 = (size_t)n * n;
        q.n = n;
        q.ptr[BF_A] = (void *)A[i]; q.ld[BF_A] = lda[i];
        q.ptr[BF_C] = (void *)C[i]; q.ld[BF_C] = ldc[i];
        q.ptr[BF_X] = (void *)X[i]; q.ld[BF_X] = ldx[i];
        q.ptr[BF_R] = pd; q.ld[BF_R] = n; pd += n2;
        q.ptr[BF_H] = pf; q.ld[BF_H] = n; pf += n2;
        q.ptr[BF_U] = pf; q.ld[BF_U] = n; pf += n2;
        q.ptr[BF_W] = pf; q.ld[BF_W] = n; pf += n2;
        q.ptr[BF_Y] = pf; q.ld[BF_Y] = n; pf += n2;
        q.ptr[BF_V] = pf; q.ld[BF_V] = n; pf += n2;
        q.ptr[BF_TB] = pf; q.ld[BF_TB] = n; pf += n2;
        q.active = 1;
    }
    BatchEq *deq = (BatchEq *)(base + o_eq);
    int *dord = (int *)(base + o_ord);
    int *dcnt = (int *)(base + o_cnt);
    hipError_t e;
    if ((e = hipMemcpyAsync(deq, hq.data(), sizeof(BatchEq) * batch, hipMemcpyHostToDevice, s)) != hipSuccess)
        return SYLV_ERR_HIP - (int)e;
    if ((e = hipMemcpyAsync(dord, order.data(), sizeof(int) * batch, hipMemcpyHostToDevice, s)) != hipSuccess)
        return SYLV_ERR_HIP - (int)e;
    static bool attr = false;
    if (!attr) {
        if ((e = hipFuncSetAttribute((const void *)k_bschur, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(sizeof(float) * band_size(256)))) != hipSuccess)
            return SYLV_ERR_HIP - (int)e;
        attr = true;
    }
    BatchPlan P;
    P.deq = deq; P.dord = dord; P.dcnt = dcnt;
    P.batch = batch; P.nmax = nmax;
    // narrow operands of the transforms: 1 bfloat16, 2 binary16 (a binary16
    // overflow of the tri-solve output shows as NaN and escalates)
    P.bf16 = (o.low == SYLV_PREC_BF16) ? 1 : (o.low == SYLV_PREC_FP16) ? 2 : 0;
    P.tol = o.tol; P.max_iter = o.max_iter;
    P.orth = o.orth_check != 0 ? 1 : 0;
    // learned precision choice: the features need the orthogonality probe
    P.autosel = (o.low == SYLV_PREC_AUTO) ? 1 : 0;
    P.feat = (float *)(base + o_sel);
    P.zfeat = P.feat + (size_t)batch * SYLV_NFEAT;
    P.prob = P.zfeat + (size_t)batch * SYLV_NFEAT;
    P.sel = nullptr;
    if (P.autosel) {
        P.orth = 1;
        int src = 0;
        P.sel = selector_device_blob(s, &src);
        if (!P.sel) return src ? src : SYLV_ERR_HIP;
    }
    const BatchTune tu = batch_tune();
    // Hessenberg size buckets (order is longest first): n > hess_hi,
    // hess_lo < n <= hess_hi, n <= hess_lo
    P.h1 = 0;
    while (P.h1 < batch && nn[order[P.h1]] > tu.hess_hi) ++P.h1;
    P.h2 = P.h1;
    while (P.h2 < batch && nn[order[P.h2]] > tu.hess_lo) ++P.h2;
    // band-QR LDS buckets: orders above band[0], (band[1], band[0]], ...
    int caps[4] = {256, 0, 0, 0}, ncap = 1;
    for (int k = 0; k < 3 && tu.band[k] > 0; ++k) caps[ncap++] = tu.band[k];
    int b0 = 0;
    for (int bi = 0; bi < ncap; ++bi) {
        const int lo = (bi + 1 < ncap) ? caps[bi + 1] : 0;
        int b1 = b0;
        while (b1 < batch && nn[order[b1]] > lo) ++b1;
        P.sb[bi] = b0;
        P.smem[bi] = (b1 > b0) ? sizeof(float) * (size_t)band_size(std::min(caps[bi], nn[order[b0]])) : 0;
        b0 = b1;
    }
    P.nsb = ncap;
    P.sb[ncap] = batch;
    double w = 0.0;
    for (int i = 0; i < batch; ++i) w += (14.0 / 3.0) * double(nn[i]) * nn[i] * nn[i];
    prof_add_work(KID_BHESS, w);

    int *hcnt = reinterpret_cast<int *>(hbuf);
    int rc = 0;
    if (batch_graph_enabled() && !prof_any_armed()) {
        // front graph, then tail graphs while equations remain (every pass
        // replayed from a captured graph)
        const int gpasses = tu.gpasses;
        rc = batch_graph_run(s, P, order, nn, gpasses, 0, dcnt, hcnt);
        if (rc) return rc;
        const int max_chunks = (o.max_iter + 1 + gpasses - 1) / gpasses + 1;
        for (int chunk = 1; *hcnt > 0 && chunk <= max_chunks; ++chunk) {
            rc = batch_graph_run(s, P, order, nn, gpasses, 1, dcnt, hcnt);
            if (rc) return rc;
        }
    } else {
        // eager launches (profiling armed, or graphs switched off)
        enqueue_front(s, P);
        for (int pass = 0; pass <= o.max_iter; ++pass) {
            enqueue_pass(s, P, false);
            if ((e = hipMemcpyAsync(hcnt, dcnt, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
                return SYLV_ERR_HIP - (int)e;
            if ((e = hipStreamSynchronize(s)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
            if (*hcnt == 0) break;
            enqueue_correction(s, P);
        }
    }
    if ((e = hipMemcpyAsync(hq.data(), deq, sizeof(BatchEq) * batch, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return SYLV_ERR_HIP - (int)e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
    double napply = 0.0;
    for (int i = 0; i < batch; ++i) napply += hq[i].napply;
    prof_add_work(KID_BSCHUR, 12.0 * napply);
    if (std::getenv("SYLV_TRACE")) {
        // per order bucket: cycles per QR step of the band-QR kernel, split
        // into the chase, the U row streams and the deflation scans
        const int edges[5] = {0, 64, 128, 180, 257};
        for (int b = 0; b < 4; ++b) {
            double cy[4] = {0, 0, 0, 0}, st = 0, sw = 0, cnt = 0;
            for (int i = 0; i < batch; ++i) {
                if (hq[i].n <= edges[b] || hq[i].n >= edges[b + 1]) continue;
                for (int k = 0; k < 4; ++k) cy[k] += (double)hq[i].cyc[k];
                st += hq[i].steps; sw += hq[i].sweeps; cnt += 1;
            }
            if (cnt == 0) continue;
            std::fprintf(stderr,
                         "[sylv] band QR n in (%d,%d): %.0f eqs, %.0f sweeps/eq, %.0f steps/eq, cycles/step "
                         "%.0f (chase %.0f, U %.0f, scan %.0f)\n",
                         edges[b], edges[b + 1], cnt, sw / cnt, st / cnt, cy[0] / st, cy[1] / st, cy[2] / st,
                         cy[3] / st);
        }
    }
    for (int i = 0; i < batch; ++i) {
        const BatchEq &q = hq[i];
        if (infos) {
            sylv_info &f = infos[i];
            std::memset(&f, 0, sizeof(f));
            f.rel_res = q.rel_res;
            f.orth_u = P.orth ? q.orth : 0.0;
            f.orth_v = f.orth_u;
            f.iterations = q.iterations;
            f.precision_used = o.low;
            f.chosen = -1;
            if (P.autosel) {
                f.chosen = q.cls;
                f.precision_used = q.cls == 0 ? SYLV_PREC_BF16 : q.cls == 1 ? SYLV_PREC_FP32 : SYLV_PREC_FP64;
            }
            f.status = q.status;
            f.fell_back = 0;
        }
    }
    return 0;
}

int batch_tune_set(int hess_hi, int hess_lo, const int *band, int gpasses) {
    if (hess_hi < 1 || hess_hi > 128) return -1;
    if (hess_lo < 1 || hess_lo > 64 || hess_lo > hess_hi) return -2;
    int prev = 256;
    bool ended = false;
    for (int k = 0; k < 3; ++k) {
        if (band[k] < 0 || (band[k] > 0 && (ended || band[k] >= prev))) return -3;
        if (band[k] == 0) ended = true;
        else prev = band[k];
    }
    if (gpasses < 1 || gpasses > 8) return -4;
    std::lock_guard<std::mutex> lk(g_btune_mu);
    g_btune.hess_hi = hess_hi;
    g_btune.hess_lo = hess_lo;
    for (int k = 0; k < 3; ++k) g_btune.band[k] = band[k];
    g_btune.gpasses = gpasses;
    return 0;
}

void batch_tune_get(int *vals) {
    const BatchTune t = batch_tune();
    vals[0] = t.hess_hi;
    vals[1] = t.hess_lo;
    vals[2] = t.band[0];
    vals[3] = t.band[1];
    vals[4] = t.band[2];
    vals[5] = t.gpasses;
}

size_t lyap_batched_bytes(int batch, const int *nn) {
    size_t ws_f = 0, ws_d = 0;
    for (int i = 0; i < batch; ++i) {
        ws_f += 6 * (size_t)nn[i] * nn[i];
        ws_d += (size_t)nn[i] * nn[i];
    }
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o2 = (off + 255) & ~(size_t)255; off = o2 + bytes; return o2; };
    take(sizeof(BatchEq) * batch);
    take(sizeof(int) * batch);
    take(64);
    take(sizeof(double) * ws_d);
    take(sizeof(float) * ws_f);
    take(sizeof(float) * (size_t)batch * (2 * SYLV_NFEAT + SYLV_NCLASS));
    return off + 256;
}

}  // namespace sylv
