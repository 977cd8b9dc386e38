// Batched Lyapunov solver AX + XA^T = C (eq. (1.3), real case) for many
// small equations (order <= 256): binary32 Schur forms + binary64
// refinement, one workgroup per equation, every stage covering the whole
// batch in one launch.  Equations are processed in decreasing order of size
// (longest first).
//
// Per equation:
//   1. k_bprep    H = fl32(A) (dense, ld n), U = I (row-major), ||A||_F, ||C||_F
//   2. k_bhess    Householder reduction of H to Hessenberg form, U <- U P_c
//   3. k_bschur   Francis double-shift QR on the Hessenberg band held in LDS
//                 (3 subdiagonals: 33.7K floats at n = 256); the reflectors of
//                 a sweep are logged and applied to the rows of U once per
//                 sweep, each thread streaming one row through registers
//   4. transforms on MFMA (gemm_batched), tri-solve T Y + Y T^T = C~ with T in
//      LDS (k_btrsyl), back-transform accumulated in binary64
//   5. refinement passes: R = C - AX - XA^T (binary64 MFMA), k_bnorm decides
//      per equation (converged / stalled / cap / NaN) and the scale 2^-e of R
//      for the binary32 correction.
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"
#include "../../include/sylv.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

namespace sylv {

constexpr int BNT = 256;   // threads of the per-equation kernels
constexpr int BSNT = 320;  // threads of the Schur kernel (5 waves)

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
__global__ __launch_bounds__(BNT) void k_bprep(BatchEq *eqs, const int *order) {
    __shared__ double red[8];
    BatchEq &q = eqs[order[blockIdx.x]];
    const int n = q.n;
    const double *A = (const double *)q.ptr[BF_A];
    const double *C = (const double *)q.ptr[BF_C];
    float *H = (float *)q.ptr[BF_H];
    float *U = (float *)q.ptr[BF_U];
    const int lda = q.ld[BF_A], ldc = q.ld[BF_C];
    double sa = 0.0, sc = 0.0;
    for (int e = threadIdx.x; e < n * n; e += BNT) {
        const int i = e % n, j = e / n;
        const double a = A[(size_t)j * lda + i], c = C[(size_t)j * ldc + i];
        sa += a * a;
        sc += c * c;
        H[e] = (float)a;
        U[e] = (i == j) ? 1.f : 0.f;
    }
    sa = wg_sum(sa, red);
    sc = wg_sum(sc, red);
    if (threadIdx.x == 0) {
        q.nA = sqrt(sa);
        q.nC = sqrt(sc);
        q.active = 1;
        q.status = SYLV_ST_NOT_CONVERGED;
        q.iterations = 0;
        q.qr_fail = 0;
        q.flag = 0;
        q.scale = 1.0;
        q.rel_res = INFINITY;
        q.prev_rel = INFINITY;
        q.corr = 0.0;
        q.stall = 0;
    }
}

// ----------------------------------------------------------- 2. Hessenberg
__global__ __launch_bounds__(BNT) void k_bhess(BatchEq *eqs, const int *order) {
    __shared__ float v[256];
    __shared__ float red[8];
    __shared__ float sh[3];
    BatchEq &q = eqs[order[blockIdx.x]];
    const int n = q.n;
    float *H = (float *)q.ptr[BF_H];
    float *U = (float *)q.ptr[BF_U];
    const int tid = threadIdx.x;
    for (int c = 0; c + 2 < n; ++c) {
        const int len = n - c - 1;  // rows c+1..n-1
        float mx = 0.f;
        for (int i = tid; i < len; i += BNT) {
            const float x = H[(size_t)c * n + c + 1 + i];
            v[i] = x;
            if (i > 0) mx = fmaxf(mx, fabsf(x));
        }
        mx = wg_max(mx, red);
        float ss = 0.f;
        if (mx > 0.f)
            for (int i = 1 + tid; i < len; i += BNT) {
                const float t = v[i] / mx;
                ss += t * t;
            }
        ss = wg_sum(ss, red);
        if (tid == 0) {
            const float alpha = v[0];
            if (mx == 0.f) { sh[0] = 0.f; sh[1] = alpha; sh[2] = 0.f; }
            else {
                const float nrm = hypotf(alpha, mx * sqrtf(ss));
                const float b = (alpha >= 0.f) ? -nrm : nrm;
                sh[0] = (b - alpha) / b;
                sh[1] = b;
                sh[2] = 1.f / (alpha - b);
            }
        }
        __syncthreads();
        const float tau = sh[0], beta = sh[1], scl = sh[2];
        for (int i = tid; i < len; i += BNT) {
            v[i] = (i == 0) ? 1.f : v[i] * scl;
            H[(size_t)c * n + c + 1 + i] = (i == 0) ? beta : 0.f;
        }
        __syncthreads();
        if (tau != 0.f) {
            // left: columns c+1..n-1, rows c+1..n-1 (one thread per column)
            for (int j = c + 1 + tid; j < n; j += BNT) {
                float *col = H + (size_t)j * n + c + 1;
                float w = 0.f;
                for (int i = 0; i < len; ++i) w += v[i] * col[i];
                w *= tau;
                for (int i = 0; i < len; ++i) col[i] -= w * v[i];
            }
            __syncthreads();
            // right: rows 0..n-1, columns c+1..n-1 (one thread per row); U too
            for (int i = tid; i < n; i += BNT) {
                float w = 0.f;
                for (int k = 0; k < len; ++k) w += H[(size_t)(c + 1 + k) * n + i] * v[k];
                w *= tau;
                for (int k = 0; k < len; ++k) H[(size_t)(c + 1 + k) * n + i] -= w * v[k];
                float *urow = U + (size_t)i * n + c + 1;
                float u = 0.f;
                for (int k = 0; k < len; ++k) u += urow[k] * v[k];
                u *= tau;
                for (int k = 0; k < len; ++k) urow[k] -= u * v[k];
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ 3. band-LDS Schur
// Column j of the band holds rows 0..min(j+3, n-1) (the Hessenberg part plus
// the two extra subdiagonals a bulge occupies).
SYLV_DEVINL int band_off(int i, int j, int n) {
    if (n < 4) return j * n + i;
    const int jt = n - 4;
    const int cs = (j <= jt) ? (j * (j + 7)) / 2 : (jt * (jt + 7)) / 2 + (j - jt) * n;
    return cs + i;
}
inline int band_size(int n) {
    if (n < 4) return n * n;
    const int jt = n - 4;
    return (jt * (jt + 7)) / 2 + 4 * n;
}
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
    int ihi = n - 1, its = 0, total = 0, fail = 0, nsteps = 0;
    double napply = 0.0;
    const int itmax = 30 * (n > 10 ? n : 10);
    while (ihi >= 0) {
        if (tid == 0) sint = 0;
        __syncthreads();
        for (int k = 1 + tid; k <= ihi; k += BSNT) {
            float hk = fabsf(HB(k, k - 1));
            float tst = fabsf(HB(k - 1, k - 1)) + fabsf(HB(k, k));
            if (tst == 0.f) {
                if (k >= 2) tst += fabsf(HB(k - 1, k - 2));
                if (k + 1 <= ihi) tst += fabsf(HB(k + 1, k));
            }
            if (hk <= fmaxf(smlnum, ulp * tst)) atomicMax(&sint, k);
        }
        __syncthreads();
        const int l = sint;
        __syncthreads();
        if (l > 0 && tid == 0) HB(l, l - 1) = 0.f;
        __syncthreads();
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
                    float *ur = U + (size_t)i * n;
                    float t1 = ur[k], t2 = ur[k + 1];
                    ur[k] = cs * t1 + sn * t2;
                    ur[k + 1] = cs * t2 - sn * t1;
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
        float h11 = HB(ihi - 1, ihi - 1), h12 = HB(ihi - 1, ihi);
        float h21 = HB(ihi, ihi - 1), h22 = HB(ihi, ihi);
        if (its == 10 || its == 20) {
            float sx = fabsf(HB(ihi, ihi - 1)) + fabsf(HB(ihi - 1, ihi - 2));
            h11 = 0.75f * sx + HB(ihi, ihi);
            h12 = -0.4375f * sx;
            h21 = sx;
            h22 = h11;
        }
        const float tr = h11 + h22, det = h11 * h22 - h12 * h21;
        float x, y, z;
        {
            float a00 = HB(l, l), a01 = HB(l, l + 1), a10 = HB(l + 1, l);
            float a11 = HB(l + 1, l + 1), a21 = HB(l + 2, l + 1);
            float sc = fabsf(a00) + fabsf(a10) + fabsf(a01) + fabsf(a11) + fabsf(a21) + fabsf(tr) + sqrtf(fabsf(det));
            if (sc == 0.f) sc = 1.f;
            const float rs = frcp(sc);
            float b00 = a00 * rs, b01 = a01 * rs, b10 = a10 * rs, b11 = a11 * rs, b21 = a21 * rs;
            float trs = tr * rs, dets = det * rs * rs;
            x = b00 * b00 + b01 * b10 - trs * b00 + dets;
            y = b10 * (b00 + b11 - trs);
            z = b10 * b21;
        }
        __syncthreads();
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
            if (wv < 2) {
                // left: columns {k-1} u [k+len, n), rows k, k+1, k2
                const int nL = lc0 + (n - (k + len));
                for (int qq = tid; qq < nL; qq += 128) {
                    if (lc0 && qq == 0) {
                        HB(k2, k - 1) = 0.f;
                        HB(k + 1, k - 1) = 0.f;
                        HB(k, k - 1) = beta;
                    } else {
                        const int j = k + len + qq - lc0;
                        float a0 = HB(k, j), a1 = HB(k + 1, j), a2 = HB(k2, j);
                        brefl(v1, v2, tau, a0, a1, a2);
                        HB(k2, j) = a2; HB(k, j) = a0; HB(k + 1, j) = a1;
                    }
                }
            } else if (wv < 4) {
                // right: rows [0, k) u {k+3}, columns k, k+1, k2
                const int extra = (len == 3 && k + 3 <= ihi) ? 1 : 0;
                const int nR = k + extra;
                for (int qq = tid - 128; qq < nR; qq += 128) {
                    const int i = (qq < k) ? qq : k + 3;
                    float a0 = HB(i, k), a1 = HB(i, k + 1), a2 = HB(i, k2);
                    brefl(v1, v2, tau, a0, a1, a2);
                    HB(i, k2) = a2; HB(i, k) = a0; HB(i, k + 1) = a1;
                }
            } else if (lane == 0) {
                // overlap block rows/cols k, k+1, k2: left then right
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
        }
        // apply the sweep's reflectors to the rows of U (row-major), each
        // thread streaming one row through a three-entry register window
        for (int i = tid; i < n; i += BSNT) {
            float *ur = U + (size_t)i * n;
            float z0 = ur[l], z1 = ur[l + 1], z2 = ur[l + 2];
            for (int k = l; k <= ihi - 1; ++k) {
                brefl(lv1[k], lv2[k], ltau[k], z0, z1, z2);
                ur[k] = z0;
                z0 = z1;
                z1 = z2;
                z2 = (k + 3 <= ihi) ? ur[k + 3] : 0.f;
            }
            ur[ihi] = z0;
        }
        __syncthreads();
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
    }
    if (tid == 0 && fail) {
        q.qr_fail = 1;
        q.status = SYLV_ST_QR_FAILED;
        q.active = 0;
    }
}
#undef HB

// ------------------------------------------ 4. Lyapunov tri-solve (T in LDS)
// T Y + Y T^T = W, T upper quasi-triangular (order n <= 256) stored packed
// in LDS (column j: rows 0..j+1), Y overwrites W in global memory.  Block
// pair (ib, jb) depends on the pairs below it (through T) and to its right
// (through T^T): wavefront over ibb + jbb with ibb counted from the bottom
// and jbb from the right.
__host__ __device__ __forceinline__ int up_off(int i, int j) { return (j * (j + 3)) / 2 + i; }

template <typename T>
SYLV_DEVINL int pair_solve_b(bool P, bool Q, T a00, T a01, T a10, T a11, T b00, T b01, T b10, T b11,
                             T r[4], T smin) {
    T m[4][4];
    const T zp = P ? T(1) : T(0), zq = Q ? T(1) : T(0), zpq = zp * zq;
    m[0][0] = a00 + b00; m[0][1] = a01 * zp; m[0][2] = b10 * zq; m[0][3] = T(0);
    m[1][0] = a10 * zp; m[1][1] = P ? a11 + b00 : T(1); m[1][2] = T(0); m[1][3] = b10 * zpq;
    m[2][0] = b01 * zq; m[2][1] = T(0); m[2][2] = Q ? a00 + b11 : T(1); m[2][3] = a01 * zpq;
    m[3][0] = T(0); m[3][1] = b01 * zpq; m[3][2] = a10 * zpq; m[3][3] = (P && Q) ? a11 + b11 : T(1);
    int flag = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int pr = c;
        T pv = fabs(m[c][c]);
#pragma unroll
        for (int rr = c + 1; rr < 4; ++rr) {
            T v = fabs(m[rr][c]);
            if (v > pv) { pv = v; pr = rr; }
        }
#pragma unroll
        for (int rr = c + 1; rr < 4; ++rr) {
            const bool sw = (pr == rr);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                T x = m[c][k], y = m[rr][k];
                m[c][k] = sw ? y : x;
                m[rr][k] = sw ? x : y;
            }
            T x = r[c], y = r[rr];
            r[c] = sw ? y : x;
            r[rr] = sw ? x : y;
        }
        T piv = m[c][c];
        if (fabs(piv) < smin) { piv = (piv >= T(0)) ? smin : -smin; m[c][c] = piv; flag = 1; }
        const T inv = T(1) / piv;
#pragma unroll
        for (int rr = c + 1; rr < 4; ++rr) {
            const T f = m[rr][c] * inv;
#pragma unroll
            for (int k = c + 1; k < 4; ++k) m[rr][k] -= f * m[c][k];
            r[rr] -= f * r[c];
        }
    }
#pragma unroll
    for (int c = 3; c >= 0; --c) {
        T acc = r[c];
#pragma unroll
        for (int k = c + 1; k < 4; ++k) acc -= m[c][k] * r[k];
        r[c] = acc / m[c][c];
    }
    return flag;
}

__global__ __launch_bounds__(BNT) void k_btrsyl(BatchEq *eqs, const int *order) {
    extern __shared__ unsigned char smem_raw[];
    float *Tp = reinterpret_cast<float *>(smem_raw);
    __shared__ int bstart[257];
    __shared__ int nbs;
    __shared__ float tmax_s;
    __shared__ float red[8];
    BatchEq &q = eqs[order[blockIdx.x]];
    if (!q.active) return;
    const int n = q.n;
    const float *Tg = (const float *)q.ptr[BF_H];
    float *Y = (float *)q.ptr[BF_W];
    const int tid = threadIdx.x;
    float mx = 0.f;
    for (int j = 0; j < n; ++j) {
        const int rows = (j + 2 < n) ? j + 2 : n;
        for (int i = tid; i < rows; i += BNT) {
            const float t = Tg[(size_t)j * n + i];
            Tp[up_off(i, j)] = t;
            mx = fmaxf(mx, fabsf(t));
        }
    }
    mx = wg_max(mx, red);
    if (tid == 0) {
        int nb = 0, i = 0;
        while (i < n) {
            bstart[nb++] = i;
            i += (i + 1 < n && Tp[up_off(i + 1, i)] != 0.f) ? 2 : 1;
        }
        bstart[nb] = n;
        nbs = nb;
        tmax_s = mx;
    }
    __syncthreads();
    const int P = nbs;
    const float smin = fmaxf(num<float>::ulp * tmax_s, num<float>::safmin);
    int myflag = 0;
#define TT(i, j) Tp[up_off((i), (j))]
#define YY(i, j) Y[(size_t)(j) * n + (i)]
    for (int e = 0; e <= 2 * P - 2; ++e) {
        const int lo = e - (P - 1) > 0 ? e - (P - 1) : 0;
        const int hi = e < P - 1 ? e : P - 1;
        const int nunits = hi - lo + 1;
        const int tpu = nunits <= 4 ? 64 : nunits <= 8 ? 32 : nunits <= 16 ? 16 : nunits <= 32 ? 8
                        : nunits <= 64 ? 4 : nunits <= 128 ? 2 : 1;
        const int u = tid / tpu, sub = tid % tpu;
        float part[4] = {0.f, 0.f, 0.f, 0.f};
        int ri = 0, pi = 0, cj = 0, qj = 0;
        const bool active = u < nunits;
        if (active) {
            const int ibb = lo + u, jbb = e - ibb;
            const int ib = P - 1 - ibb, jb = P - 1 - jbb;
            ri = bstart[ib]; pi = bstart[ib + 1] - ri;
            cj = bstart[jb]; qj = bstart[jb + 1] - cj;
            const int r2 = (pi == 2) ? ri + 1 : ri;
            const int c2 = (qj == 2) ? cj + 1 : cj;
            // sum over rows below: T(ri.., r') Y(r', cj..)
#pragma unroll 2
            for (int rp = ri + pi + sub; rp < n; rp += tpu) {
                const float a0 = TT(ri, rp), a1 = TT(r2, rp);
                const float y0 = YY(rp, cj), y1 = YY(rp, c2);
                part[0] += a0 * y0; part[1] += a1 * y0;
                part[2] += a0 * y1; part[3] += a1 * y1;
            }
            // sum over columns to the right: Y(ri.., c') T(cj.., c')
#pragma unroll 2
            for (int cp = cj + qj + sub; cp < n; cp += tpu) {
                const float b0 = TT(cj, cp), b1 = TT(c2, cp);
                const float y0 = YY(ri, cp), y1 = YY(r2, cp);
                part[0] += y0 * b0; part[1] += y1 * b0;
                part[2] += y0 * b1; part[3] += y1 * b1;
            }
        }
        for (int o = 1; o < tpu; o <<= 1) {
#pragma unroll
            for (int z = 0; z < 4; ++z) part[z] += __shfl_xor(part[z], o);
        }
        if (active && sub == 0) {
            const bool P2 = (pi == 2), Q2 = (qj == 2);
            const float a00 = TT(ri, ri);
            const float a01 = P2 ? TT(ri, ri + 1) : 0.f;
            const float a10 = P2 ? TT(ri + 1, ri) : 0.f;
            const float a11 = P2 ? TT(ri + 1, ri + 1) : 0.f;
            // right coefficient T^T restricted to block jb
            const float b00 = TT(cj, cj);
            const float b01 = Q2 ? TT(cj + 1, cj) : 0.f;
            const float b10 = Q2 ? TT(cj, cj + 1) : 0.f;
            const float b11 = Q2 ? TT(cj + 1, cj + 1) : 0.f;
            float r[4];
            r[0] = YY(ri, cj) - part[0];
            r[1] = P2 ? YY(ri + 1, cj) - part[1] : 0.f;
            r[2] = Q2 ? YY(ri, cj + 1) - part[2] : 0.f;
            r[3] = (P2 && Q2) ? YY(ri + 1, cj + 1) - part[3] : 0.f;
            myflag |= pair_solve_b<float>(P2, Q2, a00, a01, a10, a11, b00, b01, b10, b11, r, smin);
            YY(ri, cj) = r[0];
            if (P2) YY(ri + 1, cj) = r[1];
            if (Q2) YY(ri, cj + 1) = r[2];
            if (P2 && Q2) YY(ri + 1, cj + 1) = r[3];
        }
        __syncthreads();
    }
#undef TT
#undef YY
    if (myflag) atomicOr(&q.flag, 1);
}

// --------------------------------------- 5. residual norms and loop control
__global__ __launch_bounds__(BNT) void k_bcopy_c(BatchEq *eqs, const int *order) {
    BatchEq &q = eqs[order[blockIdx.x]];
    if (!q.active) return;
    const int n = q.n;
    const double *C = (const double *)q.ptr[BF_C];
    double *R = (double *)q.ptr[BF_R];
    const int ldc = q.ld[BF_C];
    for (int e = threadIdx.x; e < n * n; e += BNT) R[e] = C[(size_t)(e / n) * ldc + e % n];
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
        const double rel = sqrt(sr) / (q.nC + sqrt(sx) * 2.0 * q.nA);
        q.rel_res = rel;
        int done = 0;
        if (!(rel == rel) || !isfinite(rel) || !(mr == mr)) { q.status = SYLV_ST_NAN; done = 1; }
        else if (rel <= tol) { q.status = q.flag ? SYLV_ST_PERTURBED : SYLV_OK; done = 1; }
        else if (q.iterations >= max_iter) { q.status = SYLV_ST_NOT_CONVERGED; done = 1; }
        else {
            if (rel > 0.5 * q.prev_rel) {
                if (++q.stall >= 2) { q.status = SYLV_ST_NOT_CONVERGED; done = 1; }
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
        ws_f += 4 * (size_t)nn[i] * nn[i];
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
    // stages 1-3
    hipLaunchKernelGGL(k_bprep, dim3(batch), dim3(BNT), 0, s, deq, dord);
    {
        double w = 0.0;
        for (int i = 0; i < batch; ++i) w += (14.0 / 3.0) * double(nn[i]) * nn[i] * nn[i];
        prof_add_work(KID_BHESS, w);
        ProfScope ps(KID_BHESS, s);
        hipLaunchKernelGGL(k_bhess, dim3(batch), dim3(BNT), 0, s, deq, dord);
    }
    {
        const size_t sm = sizeof(float) * (size_t)band_size(nmax);
        static bool attr = false;
        if (!attr) {
            if ((e = hipFuncSetAttribute((const void *)k_bschur, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)(sizeof(float) * band_size(256)))) != hipSuccess)
                return SYLV_ERR_HIP - (int)e;
            attr = true;
        }
        ProfScope ps(KID_BSCHUR, s);
        hipLaunchKernelGGL(k_bschur, dim3(batch), dim3(BSNT), sm, s, deq, dord);
    }
    const size_t smt = sizeof(float) * (size_t)(up_off(0, nmax - 1) + nmax);
    {
        static bool attr = false;
        if (!attr) {
            if ((e = hipFuncSetAttribute((const void *)k_btrsyl, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)(sizeof(float) * (up_off(0, 255) + 256)))) != hipSuccess)
                return SYLV_ERR_HIP - (int)e;
            attr = true;
        }
    }
    auto trsolve = [&]() {
        ProfScope ps(KID_BTRSYL, s);
        hipLaunchKernelGGL(k_btrsyl, dim3(batch), dim3(BNT), smt, s, deq, dord);
    };
    // first iterate: W = U^T C U (U stored row-major = U^T column-major),
    // Y solves T Y + Y T^T = W, X = U Y U^T
    gemm_batched<float, double, float, float>(s, deq, dord, batch, nmax, BF_U, 0, BF_C, 0, BF_Y, 1.f, 0, 0.f);
    gemm_batched<float, float, float, float>(s, deq, dord, batch, nmax, BF_Y, 0, BF_U, 1, BF_W, 1.f, 0, 0.f);
    trsolve();
    gemm_batched<float, float, float, float>(s, deq, dord, batch, nmax, BF_U, 1, BF_W, 0, BF_Y, 1.f, 0, 0.f);
    gemm_batched<float, float, double, float>(s, deq, dord, batch, nmax, BF_Y, 0, BF_U, 0, BF_X, 1.f, 0, 0.f);
    int *hcnt = reinterpret_cast<int *>(hbuf);
    for (int pass = 0; pass <= o.max_iter; ++pass) {
        // R = C - A X - X A^T (binary64)
        hipLaunchKernelGGL(k_bcopy_c, dim3(batch), dim3(BNT), 0, s, deq, dord);
        gemm_batched<double, double, double, double>(s, deq, dord, batch, nmax, BF_A, 0, BF_X, 0, BF_R, -1.0, 0, 1.0);
        gemm_batched<double, double, double, double>(s, deq, dord, batch, nmax, BF_X, 0, BF_A, 1, BF_R, -1.0, 0, 1.0);
        if ((e = hipMemsetAsync(dcnt, 0, sizeof(int), s)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
        hipLaunchKernelGGL(k_bnorm, dim3(batch), dim3(BNT), 0, s, deq, dord, o.tol, o.max_iter, dcnt);
        if ((e = hipMemcpyAsync(hcnt, dcnt, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return SYLV_ERR_HIP - (int)e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
        if (*hcnt == 0) break;
        // correction: W = 2^-e U^T R U ; tri-solve ; X += 2^e U Y U^T
        gemm_batched<float, double, float, float>(s, deq, dord, batch, nmax, BF_U, 0, BF_R, 0, BF_Y, 1.f, 1, 0.f);
        gemm_batched<float, float, float, float>(s, deq, dord, batch, nmax, BF_Y, 0, BF_U, 1, BF_W, 1.f, 0, 0.f);
        trsolve();
        gemm_batched<float, float, float, float>(s, deq, dord, batch, nmax, BF_U, 1, BF_W, 0, BF_Y, 1.f, 0, 0.f);
        gemm_batched<float, float, double, float>(s, deq, dord, batch, nmax, BF_Y, 0, BF_U, 0, BF_X, 1.f, 2, 1.f);
    }
    if ((e = hipMemcpyAsync(hq.data(), deq, sizeof(BatchEq) * batch, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return SYLV_ERR_HIP - (int)e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
    double napply = 0.0;
    for (int i = 0; i < batch; ++i) napply += hq[i].napply;
    prof_add_work(KID_BSCHUR, 12.0 * napply);
    for (int i = 0; i < batch; ++i) {
        const BatchEq &q = hq[i];
        if (infos) {
            sylv_info &f = infos[i];
            std::memset(&f, 0, sizeof(f));
            f.rel_res = q.rel_res;
            f.iterations = q.iterations;
            f.precision_used = SYLV_PREC_FP32;
            f.status = q.status;
            f.fell_back = 0;
        }
    }
    return 0;
}

size_t lyap_batched_bytes(int batch, const int *nn) {
    size_t ws_f = 0, ws_d = 0;
    for (int i = 0; i < batch; ++i) {
        ws_f += 4 * (size_t)nn[i] * nn[i];
        ws_d += (size_t)nn[i] * nn[i];
    }
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o2 = (off + 255) & ~(size_t)255; off = o2 + bytes; return o2; };
    take(sizeof(BatchEq) * batch);
    take(sizeof(int) * batch);
    take(64);
    take(sizeof(double) * ws_d);
    take(sizeof(float) * ws_f);
    return off + 256;
}

}  // namespace sylv
