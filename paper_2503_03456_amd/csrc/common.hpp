// Shared device/host helpers for the gfx950 Sylvester solver.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <cmath>
#include <cfloat>

#define SYLV_DEVINL __device__ __forceinline__

// Column-major element access.
#define CM(a, i, j, ld) ((a)[(size_t)(j) * (size_t)(ld) + (size_t)(i)])

namespace sylv {

template <typename T> struct num;
// big: a power of two well below the magnitude whose reciprocal is subnormal.
template <> struct num<float> {
    static constexpr float ulp = 5.9604644775390625e-08f;  // 2^-24, unit roundoff of binary32
    static constexpr float safmin = 1.17549435e-38f;
    static constexpr float big = 0x1p100f;
};
template <> struct num<double> {
    static constexpr double ulp = 1.1102230246251565e-16;  // 2^-53
    static constexpr double safmin = 2.2250738585072014e-308;
    static constexpr double big = 0x1p1000;
};

// Error checking on the host: returns the negative ABI code from the caller.
#define HIP_TRY(expr)                                         \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return SYLV_ERR_HIP - (int)_e;  \
    } while (0)

// Fast reciprocal / square root for reflector generation: the hardware
// approximations (1 ulp in binary32) and, for binary64, v_rcp_f64 refined by
// two Newton steps.  A relative error of a few ulps in tau or v keeps the
// reflector orthogonal to working precision.
SYLV_DEVINL float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
SYLV_DEVINL double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}
SYLV_DEVINL float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
SYLV_DEVINL double fsqrt(double x) { return sqrt(x); }

// Householder reflector for a vector of length 2 or 3 (z ignored when
// len == 2): P = I - tau v v^T, v = (1, v1, v2), P x = beta e1.  Returns
// tau = 0 when x(1:) is zero (P = I).  Everything but beta is formed from the
// vector scaled by 1/mm, mm its largest magnitude clamped to [safmin, big]:
// a collapsed bulge can leave entries below the normal range, where the
// reciprocal of the magnitude itself would overflow, and near the top of the
// range that reciprocal would be subnormal.
template <typename T>
SYLV_DEVINL void reflector3(int len, T x, T y, T z, T &v1, T &v2, T &tau, T &beta) {
    if (len == 2) z = T(0);
    T tail = fmax(fabs(y), fabs(z));
    if (tail == T(0)) {
        v1 = T(0); v2 = T(0); tau = T(0); beta = x;
        return;
    }
    const T mm = fmin(fmax(fmax(fabs(x), tail), num<T>::safmin), num<T>::big);
    const T rm = frcp(mm);
    const T xs = x * rm, ys = y * rm, zs = z * rm;
    const T ns = fsqrt(xs * xs + ys * ys + zs * zs);
    const T bs = (x >= T(0)) ? -ns : ns;
    tau = (bs - xs) * frcp(bs);
    const T sc = frcp(xs - bs);
    v1 = ys * sc;
    v2 = zs * sc;
    beta = bs * mm;
}

// DPP lane move (CTRL a gfx9 DPP control: row_shr:k = 0x110 + k, row_bcast:15
// = 0x142, row_bcast:31 = 0x143); lanes without a source read 0
template <int CTRL>
SYLV_DEVINL float dpp_move(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
SYLV_DEVINL double dpp_move(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}

// 16x16x4 MFMA in the precision T (binary32 or binary64 accumulate).  With
// the operands fed swapped (op(B)^T in the A slot, op(A)^T in the B slot),
// lane l ends up holding C(l & 15, orow(l, r)) in accumulator r, i.e. each
// lane's accumulators run down a column of C.
template <typename T> struct mfma16;
template <> struct mfma16<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static SYLV_DEVINL v4 op(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static SYLV_DEVINL int orow(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct mfma16<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static SYLV_DEVINL v4 op(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static SYLV_DEVINL int orow(int l, int r) { return (l >> 4) + 4 * r; }
};

// Symmetric Lyapunov helpers on one pair of 32 x 32 tiles (ti <= tj) of an
// n x n binary64 matrix R, in place, 256 threads.  Both tiles are staged in
// LDS so that every global access runs down columns (coalesced):
//   res = true:  R(i, j) <- C(i, j) + w, w = R(i, j) + R(j, i)  (R = -A X on entry)
//   res = false: R(i, j) <- (R(i, j) + R(j, i)) / 2
// w is the same sum for (i, j) and (j, i), so the result of res = false is
// exactly symmetric.  sa, sb: 32 x 33 doubles of LDS each.
SYLV_DEVINL int sym_pair_count(int n) {
    const int nt = (n + 31) / 32;
    return nt * (nt + 1) / 2;
}
SYLV_DEVINL void sym_pair_index(int k, int &ti, int &tj) {
    // k = tj (tj + 1) / 2 + ti, 0 <= ti <= tj
    int j = (int)((sqrt(8.0 * k + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > k) --j;
    while ((j + 1) * (j + 2) / 2 <= k) ++j;
    tj = j;
    ti = k - j * (j + 1) / 2;
}
SYLV_DEVINL void sym_tile_pair(bool res, int n, const double *C, int ldc, double *R, int ldr, int ti, int tj,
                               double (*sa)[33], double (*sb)[33]) {
    const int r0 = 32 * ti, c0 = 32 * tj;
    for (int e = threadIdx.x; e < 1024; e += 256) {
        const int ii = e & 31, jj = e >> 5;
        // sa[jj][ii] = R(r0 + ii, c0 + jj), sb[jj][ii] = R(c0 + ii, r0 + jj)
        sa[jj][ii] = (r0 + ii < n && c0 + jj < n) ? R[(size_t)(c0 + jj) * ldr + r0 + ii] : 0.0;
        sb[jj][ii] = (c0 + ii < n && r0 + jj < n) ? R[(size_t)(r0 + jj) * ldr + c0 + ii] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256) {
        const int ii = e & 31, jj = e >> 5;
        if (r0 + ii < n && c0 + jj < n) {
            const double w = sa[jj][ii] + sb[ii][jj];   // R(i, j) + R(j, i)
            R[(size_t)(c0 + jj) * ldr + r0 + ii] = res ? C[(size_t)(c0 + jj) * ldc + r0 + ii] + w : 0.5 * w;
        }
        if (ti != tj && c0 + ii < n && r0 + jj < n) {
            const double w = sa[ii][jj] + sb[jj][ii];   // R(j', i') + R(i', j'), same sum
            R[(size_t)(r0 + jj) * ldr + c0 + ii] = res ? C[(size_t)(r0 + jj) * ldc + c0 + ii] + w : 0.5 * w;
        }
    }
}

// First column (x, y, z) of (H - s1 I)(H - s2 I) e1 for the leading 3x2
// corner a00 a01 / a10 a11 / . a21 of an unreduced Hessenberg block, up to a
// positive scale.  The shifts are a real pair (cplx = 0: s1 = p, s2 = q) or
// a complex pair p +- i q (cplx = 1).  Formed from the differences a00 - s
// rather than from trace and determinant: near a cluster of equal
// eigenvalues those differences are exact while the expanded polynomial
// cancels to rounding noise and the QR iteration stagnates.
template <typename T>
SYLV_DEVINL void shift_column(T a00, T a01, T a10, T a11, T a21, T p, T q, bool cplx, T &x, T &y, T &z) {
    if (cplx) {
        const T d0 = a00 - p;
        T sc = fabs(d0) + fabs(q) + fabs(a10);
        if (sc == T(0)) sc = T(1);
        const T h = a10 / sc;
        x = h * a01 + d0 * (d0 / sc) + q * (q / sc);
        y = h * (d0 + (a11 - p));
        z = h * a21;
    } else {
        const T d1 = a00 - p, d2 = a00 - q;
        T sc = fabs(d2) + fabs(a10);
        if (sc == T(0)) sc = T(1);
        const T h = a10 / sc;
        x = h * a01 + d1 * (d2 / sc);
        y = h * (d1 + (a11 - q));
        z = h * a21;
    }
}

// Eigenvalues of [[h11, h12], [h21, h22]] as a shift pair for shift_column.
template <typename T>
SYLV_DEVINL void shift_pair(T h11, T h12, T h21, T h22, T &p, T &q, bool &cplx) {
    const T hp = T(0.5) * (h11 - h22), bc = h12 * h21, disc = hp * hp + bc;
    if (disc >= T(0)) {
        const T r = sqrt(disc);
        const T w = hp + ((hp >= T(0)) ? r : -r);
        p = h22 + w;
        q = (w != T(0)) ? h22 - bc / w : h22;
        cplx = false;
    } else {
        p = h22 + hp;
        q = sqrt(-disc);
        cplx = true;
    }
}

}  // namespace sylv

// ABI error codes (mirrors include/sylv.h)
#ifndef SYLV_ERR_HIP
#define SYLV_ERR_HIP (-100)
#define SYLV_ERR_ALLOC (-200)
#define SYLV_ERR_NOGPU (-300)
#endif
