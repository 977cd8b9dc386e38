// QR algorithm kernels for the real Schur form (the low- or high-precision
// Schur factorisations the paper's Sec. 2.1 assumes, computed by the QR
// algorithm of Golub & Van Loan, Sec. 7.5).
//
// Building blocks, all single-workgroup and LDS-resident:
//   * francis_lds: implicit double-shift QR sweeps on a small dense upper
//     Hessenberg matrix held in LDS, accumulating the orthogonal factor;
//     deflation on negligible subdiagonal entries, exceptional shifts every
//     10 sweeps without a deflation, real-eigenvalue 2x2 blocks split by one
//     rotation.  One barrier per bulge step: the 3x3 overlap block of a
//     step is owned by one thread, so left and right updates never race.
//   * francis_wave: the same sweeps for windows of order <= 64 on one
//     wavefront, without barriers.
//   * k_aed: aggressive early deflation on the trailing window of the active
//     block (Braman, Byers & Mathias 2002, part II): Schur form of the window,
//     spike test from the bottom, restoration of Hessenberg form of the
//     undeflated part; its eigenvalues become the next sweep's shifts.  With
//     a zero spike it is simply the full Schur form of the window.
//   * k_chase: one window phase of a small-bulge multishift sweep (part I of
//     the same reference): a chain of bulges spaced three rows apart moves
//     `adv` rows down inside an LDS window while the window's orthogonal
//     factor is accumulated in LDS.  A step is a left phase and a right
//     phase; in the right phase one lane per bulge also forms the bulge's
//     next reflector.  The updates outside the window follow in one MFMA
//     launch (k_win_update).
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

#include <algorithm>
#include <mutex>

namespace sylv {

// ------------------------------------------------------------------ helpers

// Split the 2x2 block at (k, k) of the LDS matrix H (n x n) if its
// eigenvalues are real: rotate so the block becomes upper triangular.
// Updates rows k,k+1 (cols k..n-1), cols k,k+1 (rows 0..k+1) and cols k,k+1
// of Z (nz rows).  Must be called by all threads (contains barriers).
template <typename T, int NT>
SYLV_DEVINL void std2x2_lds(int n, T *H, int ldh, T *Z, int ldz, int nz, int k) {
    const int tid = threadIdx.x;
    T a = CM(H, k, k, ldh), b = CM(H, k, k + 1, ldh);
    T c = CM(H, k + 1, k, ldh), d = CM(H, k + 1, k + 1, ldh);
    __syncthreads();
    if (c == T(0)) return;
    T p = T(0.5) * (a - d);
    T disc = p * p + b * c;
    if (disc < T(0)) return;  // complex pair: keep the block
    // eigenvalue lam with |lam - d| = |p| + sqrt(disc); eigenvector (lam - d, c)
    T e1 = p + copysign(sqrt(disc), p);
    T nv = hypot(e1, c);
    T cs = e1 / nv, sn = c / nv;
    // rows k, k+1 of H: [r_k; r_k1] <- G^T [r_k; r_k1],  G = [[cs,-sn],[sn,cs]]
    for (int j = k + tid; j < n; j += NT) {
        T t1 = CM(H, k, j, ldh), t2 = CM(H, k + 1, j, ldh);
        CM(H, k, j, ldh) = cs * t1 + sn * t2;
        CM(H, k + 1, j, ldh) = cs * t2 - sn * t1;
    }
    __syncthreads();
    for (int i = tid; i <= k + 1; i += NT) {
        T t1 = CM(H, i, k, ldh), t2 = CM(H, i, k + 1, ldh);
        CM(H, i, k, ldh) = cs * t1 + sn * t2;
        CM(H, i, k + 1, ldh) = cs * t2 - sn * t1;
    }
    for (int i = tid; i < nz; i += NT) {
        T t1 = CM(Z, i, k, ldz), t2 = CM(Z, i, k + 1, ldz);
        CM(Z, i, k, ldz) = cs * t1 + sn * t2;
        CM(Z, i, k + 1, ldz) = cs * t2 - sn * t1;
    }
    __syncthreads();
    if (tid == 0) CM(H, k + 1, k, ldh) = T(0);
    __syncthreads();
}

// Apply the reflector (1, v1, v2) with tau to a 3-vector.  A length-2
// reflector has v2 = 0 and leaves a2 unchanged, so callers load a2 from a
// clamped (valid) index and store it before a0/a1: no branches around LDS
// accesses, which lets the loads of one item issue together.
template <typename T>
SYLV_DEVINL void refl_apply(int, T v1, T v2, T tau, T &a0, T &a1, T &a2) {
    T s = (a0 + v1 * a1 + v2 * a2) * tau;
    a0 -= s;
    a1 -= s * v1;
    a2 -= s * v2;
}

// Francis double-shift QR on an n x n upper Hessenberg H in LDS (full Schur
// form of H), Z (nz x n, LDS or global) <- Z * Q.  Returns 0 or 1
// (iteration cap).  All threads must call it.  sint: one int of LDS scratch.
template <typename T, int NT>
SYLV_DEVINL int francis_lds(int n, T *H, int ldh, T *Z, int ldz, int nz, int *sint,
                            int *nsweep = nullptr, int *nstep = nullptr) {
    const int tid = threadIdx.x;
    const T ulp = num<T>::ulp, smlnum = num<T>::safmin * T(n) / num<T>::ulp;
    int ihi = n - 1, its = 0, total = 0;
    const int itmax = 30 * (n > 10 ? n : 10);
    while (ihi >= 0) {
        if (tid == 0) *sint = 0;
        __syncthreads();
        for (int k = 1 + tid; k <= ihi; k += NT) {
            T hk = fabs(CM(H, k, k - 1, ldh));
            T tst = fabs(CM(H, k - 1, k - 1, ldh)) + fabs(CM(H, k, k, ldh));
            if (tst == T(0)) {
                if (k >= 2) tst += fabs(CM(H, k - 1, k - 2, ldh));
                if (k + 1 <= ihi) tst += fabs(CM(H, k + 1, k, ldh));
            }
            if (hk <= fmax(smlnum, ulp * tst)) atomicMax(sint, k);
        }
        __syncthreads();
        const int l = *sint;
        __syncthreads();
        if (l > 0 && tid == 0) CM(H, l, l - 1, ldh) = T(0);
        __syncthreads();
        if (l == ihi) { ihi -= 1; its = 0; continue; }
        if (l == ihi - 1) {
            std2x2_lds<T, NT>(n, H, ldh, Z, ldz, nz, l);
            ihi -= 2; its = 0;
            continue;
        }
        if (++total > itmax) return 1;
        ++its;
        if (nsweep) { ++*nsweep; *nstep += ihi - l; }
        T h11 = CM(H, ihi - 1, ihi - 1, ldh), h12 = CM(H, ihi - 1, ihi, ldh);
        T h21 = CM(H, ihi, ihi - 1, ldh), h22 = CM(H, ihi, ihi, ldh);
        // exceptional shifts every 10 sweeps without a deflation, built from
        // the bottom of the active block and, every 20, from its top (breaks
        // the cycles a stagnating block can fall into)
        if (its % 10 == 0) {
            const bool top = (its % 20 == 0);
            const T s = top ? fabs(CM(H, l + 1, l, ldh)) + fabs(CM(H, l + 2, l + 1, ldh))
                            : fabs(CM(H, ihi, ihi - 1, ldh)) + fabs(CM(H, ihi - 1, ihi - 2, ldh));
            h11 = T(0.75) * s + (top ? CM(H, l, l, ldh) : CM(H, ihi, ihi, ldh));
            h12 = T(-0.4375) * s;
            h21 = s;
            h22 = h11;
        }
        T x, y, z;
        {
            T sp, sq;
            bool cplx;
            shift_pair(h11, h12, h21, h22, sp, sq, cplx);
            shift_column(CM(H, l, l, ldh), CM(H, l, l + 1, ldh), CM(H, l + 1, l, ldh), CM(H, l + 1, l + 1, ldh),
                         CM(H, l + 2, l + 1, ldh), sp, sq, cplx, x, y, z);
        }
        __syncthreads();
        // The column a step reduces (k-1) is read by every thread at the top
        // of that step, so its final values (beta, 0, 0) are written one step
        // later, when no thread reads it.
        int pcol = -1, pk2 = 0;
        T pbeta = T(0);
        for (int k = l; k <= ihi - 1; ++k) {
            const int len = (k <= ihi - 2) ? 3 : 2;
            if (k > l) {
                x = CM(H, k, k - 1, ldh);
                y = CM(H, k + 1, k - 1, ldh);
                z = CM(H, (len == 3) ? k + 2 : k + 1, k - 1, ldh);
            }
            T v1, v2, tau, beta;
            reflector3(len, x, y, z, v1, v2, tau, beta);
            // Work split by wave so that no wave runs two code paths
            // (WL = (NW-1)/3 waves per role):
            //   waves [0, WL): left application on columns [k+len, n) (and the
            //           deferred column of the previous step)
            //   waves [WL, 2WL): right application on rows [0, k) u {k+3}
            //   waves [2WL, NW-1): the accumulated factor Z (rows 0..nz-1)
            //   wave NW-1, lane 0: the overlap block rows/cols k..k+len-1
            constexpr int NWV = NT / 64;
            constexpr int WL = (NWV - 1) / 3, TL = 64 * WL;
            static_assert(NWV >= 4, "francis_lds needs at least 4 waves");
            const int wv = tid >> 6, lane = tid & 63;
            const int k2 = (len == 3) ? k + 2 : k + 1;  // clamped third index
            if (wv < WL) {
                if (tid == 0 && pcol >= 0) {
                    CM(H, pk2, pcol, ldh) = T(0);
                    CM(H, pcol + 2, pcol, ldh) = T(0);
                    CM(H, pcol + 1, pcol, ldh) = pbeta;
                }
                const int nL = n - (k + len);
                for (int q = tid; q < nL; q += TL) {
                    const int j = k + len + q;
                    T a0 = CM(H, k, j, ldh), a1 = CM(H, k + 1, j, ldh), a2 = CM(H, k2, j, ldh);
                    refl_apply(len, v1, v2, tau, a0, a1, a2);
                    CM(H, k2, j, ldh) = a2; CM(H, k, j, ldh) = a0; CM(H, k + 1, j, ldh) = a1;
                }
            } else if (wv < 2 * WL) {
                const int extra = (len == 3 && k + 3 <= ihi) ? 1 : 0;
                const int nR = k + extra;
                for (int q = tid - TL; q < nR; q += TL) {
                    const int i = (q < k) ? q : k + 3;
                    T a0 = CM(H, i, k, ldh), a1 = CM(H, i, k + 1, ldh), a2 = CM(H, i, k2, ldh);
                    refl_apply(len, v1, v2, tau, a0, a1, a2);
                    CM(H, i, k2, ldh) = a2; CM(H, i, k, ldh) = a0; CM(H, i, k + 1, ldh) = a1;
                }
            } else if (wv < NWV - 1) {
                for (int i = tid - 2 * TL; i < nz; i += NT - 64 - 2 * TL) {
                    T a0 = CM(Z, i, k, ldz), a1 = CM(Z, i, k + 1, ldz), a2 = CM(Z, i, k2, ldz);
                    refl_apply(len, v1, v2, tau, a0, a1, a2);
                    CM(Z, i, k2, ldz) = a2; CM(Z, i, k, ldz) = a0; CM(Z, i, k + 1, ldz) = a1;
                }
            } else if (lane == 0) {
                // overlap block in registers: left then right on rows/cols
                // k, k+1, k2 (k2 = k+1 duplicates for a length-2 step: the
                // duplicate is stored first so the genuine value wins)
                const int ix[3] = {k, k + 1, k2};
                T b[3][3];
#pragma unroll
                for (int jj = 0; jj < 3; ++jj)
#pragma unroll
                    for (int ii = 0; ii < 3; ++ii) b[ii][jj] = CM(H, ix[ii], ix[jj], ldh);
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) refl_apply(len, v1, v2, tau, b[0][jj], b[1][jj], b[2][jj]);
#pragma unroll
                for (int ii = 0; ii < 3; ++ii) refl_apply(len, v1, v2, tau, b[ii][0], b[ii][1], b[ii][2]);
#pragma unroll
                for (int jj = 2; jj >= 0; --jj)
#pragma unroll
                    for (int ii = 2; ii >= 0; --ii) CM(H, ix[ii], ix[jj], ldh) = b[ii][jj];
            }
            __syncthreads();
            pcol = (k > l) ? k - 1 : -1;
            pbeta = beta;
            pk2 = k2;
        }
        if (pcol >= 0 && tid == 0) {
            CM(H, pk2, pcol, ldh) = T(0);
            CM(H, pcol + 2, pcol, ldh) = T(0);
            CM(H, pcol + 1, pcol, ldh) = pbeta;
        }
        __syncthreads();
    }
    // exact zeros below the first subdiagonal
    for (int e = tid; e < n * n; e += NT) {
        int i = e % n, j = e / n;
        if (i > j + 1) CM(H, i, j, ldh) = T(0);
    }
    __syncthreads();
    return 0;
}

// -------------------------------------------------------- francis_wave
// The same double-shift QR sweeps for a window of order n <= 64, run by one
// wavefront: lane i owns row / column i.  Every lane forms the same
// reflector; the left update (columns of rows k..k+2), the right update
// (rows of columns k..k+2) and the Z update of a bulge step follow each other
// in program order, and the LDS operations of one wavefront complete in
// order, so a step needs no barrier.  The deflation scan is a ballot.
// Returns 0, or 1 when the iteration cap ran out.
// Orders the LDS accesses of one wavefront around this point (a compiler
// fence at wavefront scope; the hardware keeps a wave's LDS operations in order).
SYLV_DEVINL void wave_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// v of lane src (uniform) broadcast to the wavefront, through scalar registers
SYLV_DEVINL float wave_bcast(float v, int src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}
SYLV_DEVINL double wave_bcast(double v, int src) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), src);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}

template <typename T>
SYLV_DEVINL int francis_wave(int n, T *H, int ldh, T *Z, int ldz, int nz, int *nsweep, int *nstep) {
    const int lane = threadIdx.x & 63;
    const T ulp = num<T>::ulp, smlnum = num<T>::safmin * T(n) / num<T>::ulp;
    int ihi = n - 1, its = 0, total = 0;
    const int itmax = 30 * (n > 10 ? n : 10);
    while (ihi >= 0) {
        bool neg = false;
        if (lane >= 1 && lane <= ihi) {
            const int k = lane;
            const T hk = fabs(CM(H, k, k - 1, ldh));
            T tst = fabs(CM(H, k - 1, k - 1, ldh)) + fabs(CM(H, k, k, ldh));
            if (tst == T(0)) {
                if (k >= 2) tst += fabs(CM(H, k - 1, k - 2, ldh));
                if (k + 1 <= ihi) tst += fabs(CM(H, k + 1, k, ldh));
            }
            neg = hk <= fmax(smlnum, ulp * tst);
        }
        const unsigned long long mask = __ballot(neg);
        const int l = mask ? 63 - __clzll(mask) : 0;   // largest negligible index
        wave_order();
        if (l > 0 && lane == 0) CM(H, l, l - 1, ldh) = T(0);
        wave_order();
        if (l == ihi) { ihi -= 1; its = 0; continue; }
        if (l == ihi - 1) {
            // 2x2 block: split by one rotation when its eigenvalues are real
            const int k = l;
            const T a = CM(H, k, k, ldh), b = CM(H, k, k + 1, ldh);
            const T c = CM(H, k + 1, k, ldh), d = CM(H, k + 1, k + 1, ldh);
            const T pp = T(0.5) * (a - d), disc = pp * pp + b * c;
            wave_order();
            if (c != T(0) && disc >= T(0)) {
                const T e1 = pp + copysign(sqrt(disc), pp);
                const T nv = hypot(e1, c);
                const T cs = e1 / nv, sn = c / nv;
                if (lane >= k && lane < n) {
                    const int j = lane;
                    const T t1 = CM(H, k, j, ldh), t2 = CM(H, k + 1, j, ldh);
                    CM(H, k, j, ldh) = cs * t1 + sn * t2;
                    CM(H, k + 1, j, ldh) = cs * t2 - sn * t1;
                }
                wave_order();
                if (lane <= k + 1) {
                    const int i = lane;
                    const T t1 = CM(H, i, k, ldh), t2 = CM(H, i, k + 1, ldh);
                    CM(H, i, k, ldh) = cs * t1 + sn * t2;
                    CM(H, i, k + 1, ldh) = cs * t2 - sn * t1;
                }
                if (lane < nz) {
                    const int i = lane;
                    const T t1 = CM(Z, i, k, ldz), t2 = CM(Z, i, k + 1, ldz);
                    CM(Z, i, k, ldz) = cs * t1 + sn * t2;
                    CM(Z, i, k + 1, ldz) = cs * t2 - sn * t1;
                }
                wave_order();
                if (lane == 0) CM(H, k + 1, k, ldh) = T(0);
                wave_order();
            }
            ihi -= 2; its = 0;
            continue;
        }
        if (++total > itmax) return 1;
        ++its;
        if (nsweep && lane == 0) { ++*nsweep; *nstep += ihi - l; }
        T h11 = CM(H, ihi - 1, ihi - 1, ldh), h12 = CM(H, ihi - 1, ihi, ldh);
        T h21 = CM(H, ihi, ihi - 1, ldh), h22 = CM(H, ihi, ihi, ldh);
        if (its % 10 == 0) {
            // exceptional shifts as in the barrier version above
            const bool top = (its % 20 == 0);
            const T sx = top ? fabs(CM(H, l + 1, l, ldh)) + fabs(CM(H, l + 2, l + 1, ldh))
                             : fabs(CM(H, ihi, ihi - 1, ldh)) + fabs(CM(H, ihi - 1, ihi - 2, ldh));
            h11 = T(0.75) * sx + (top ? CM(H, l, l, ldh) : CM(H, ihi, ihi, ldh));
            h12 = T(-0.4375) * sx;
            h21 = sx;
            h22 = h11;
        }
        T x, y, z;
        {
            T sp, sq;
            bool cplx;
            shift_pair(h11, h12, h21, h22, sp, sq, cplx);
            shift_column(CM(H, l, l, ldh), CM(H, l, l + 1, ldh), CM(H, l + 1, l, ldh), CM(H, l + 1, l + 1, ldh),
                         CM(H, l + 2, l + 1, ldh), sp, sq, cplx, x, y, z);
        }
        for (int k = l; k <= ihi - 1; ++k) {
            const int len = (k <= ihi - 2) ? 3 : 2;
            const int k2 = (len == 3) ? k + 2 : k + 1;   // clamped third index
            // (x, y, z) for k > l: rows k..k2 of column k-1, broadcast from
            // the lanes that formed them in the previous right update
            T v1, v2, tau, beta;
            reflector3(len, x, y, z, v1, v2, tau, beta);
            wave_order();
            // left: rows k..k2, columns k..n-1; column k-1 becomes (beta, 0, 0)
            if (k > l && lane == k - 1) {
                CM(H, k2, lane, ldh) = T(0);
                CM(H, k + 1, lane, ldh) = T(0);
                CM(H, k, lane, ldh) = beta;
            } else if (lane >= k && lane < n) {
                const int j = lane;
                T a0 = CM(H, k, j, ldh), a1 = CM(H, k + 1, j, ldh), a2 = CM(H, k2, j, ldh);
                refl_apply(len, v1, v2, tau, a0, a1, a2);
                CM(H, k2, j, ldh) = a2; CM(H, k, j, ldh) = a0; CM(H, k + 1, j, ldh) = a1;
            }
            wave_order();
            // right: columns k..k2, rows 0..min(k+3, ihi)
            const int rmax = (k + 3 < ihi) ? k + 3 : ihi;
            // H rows 0..rmax and Z rows 0..nz-1: both rows' loads first (rows
            // clamped into range, stores only for real rows), then the updates
            const bool hrow = lane <= rmax, zrow = lane < nz;
            const int ih = hrow ? lane : 0, iz = zrow ? lane : 0;
            T a0 = CM(H, ih, k, ldh), a1 = CM(H, ih, k + 1, ldh), a2 = CM(H, ih, k2, ldh);
            T b0 = CM(Z, iz, k, ldz), b1 = CM(Z, iz, k + 1, ldz), b2 = CM(Z, iz, k2, ldz);
            refl_apply(len, v1, v2, tau, a0, a1, a2);
            refl_apply(len, v1, v2, tau, b0, b1, b2);
            if (hrow) { CM(H, ih, k2, ldh) = a2; CM(H, ih, k, ldh) = a0; CM(H, ih, k + 1, ldh) = a1; }
            if (zrow) { CM(Z, iz, k2, ldz) = b2; CM(Z, iz, k, ldz) = b0; CM(Z, iz, k + 1, ldz) = b1; }
            const T col_k = hrow ? a0 : T(0);   // this lane's new H(lane, k)
            if (k + 1 <= ihi - 1) {
                // next step's column: rows k+1 .. k+1+len'-1 of column k (lanes <= rmax)
                const int kn2 = (k + 1 <= ihi - 2) ? k + 3 : k + 2;
                x = wave_bcast(col_k, k + 1);
                y = wave_bcast(col_k, k + 2);
                z = wave_bcast(col_k, kn2);
            }
            wave_order();
        }
    }
    // exact zeros below the first subdiagonal
    for (int e = lane; e < n * n; e += 64) {
        const int i = e % n, j = e / n;
        if (i > j + 1) CM(H, i, j, ldh) = T(0);
    }
    wave_order();
    return 0;
}

// Householder vector of x (len entries, LDS, stride 1) by wavefront 0:
// P x = beta e1, P = I - tau v v^T, v[0] = 1, written to v (may alias x).
// Max and scaled sum of squares are wavefront reductions.  Lanes 0..63 call
// it; lane 0 stores tau and beta.
template <typename T>
SYLV_DEVINL void house_wave(int len, T *x, T *v, T *tau_out, T *beta_out) {
    const int lane = threadIdx.x & 63;
    const T alpha = x[0];
    T mx = T(0);
    for (int i = 1 + lane; i < len; i += 64) mx = fmax(mx, fabs(x[i]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    T tau = T(0), beta = alpha, sc = T(0);
    if (mx > T(0)) {
        T ss = T(0);
        for (int i = 1 + lane; i < len; i += 64) { const T q = x[i] / mx; ss += q * q; }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
        const T xn = mx * sqrt(ss), nrm = hypot(alpha, xn);
        const T b = (alpha >= T(0)) ? -nrm : nrm;
        tau = (b - alpha) / b;
        sc = T(1) / (alpha - b);
        beta = b;
    }
    for (int i = 1 + lane; i < len; i += 64) v[i] = x[i] * sc;
    if (lane == 0) { v[0] = T(1); *tau_out = tau; *beta_out = beta; }
}

// ---------------------------------------------------------------- k_aed
// out[0] = status (0 ok, 1 QR cap), out[1] = nd (deflated count), out[2] =
// ns (undeflated count); wr/wi (length nw) receive the eigenvalues of the
// undeflated part in diagonal order.  Zw (global, nw x nw, ld nw) receives
// the window's orthogonal factor.  spike_on = 0 means the window is the
// whole active block (no spike): full Schur form, everything deflates.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_aed(int nw, T *H, int ldh, int kwtop, int spike_on,
                                           T *Zw, int *out, T *wr, T *wi) {
    extern __shared__ unsigned char smem_raw[];
    // odd leading dimension: row-wise accesses across consecutive columns hit
    // distinct LDS banks
    const int L = nw | 1;
    T *Tw = reinterpret_cast<T *>(smem_raw);
    T *Zl = Tw + L * nw;
    T *sp = Zl + L * nw;  // spike, length nw
    int *sint = reinterpret_cast<int *>(sp + nw);
    const int tid = threadIdx.x;
    for (int e = tid; e < nw * nw; e += NT) {
        int i = e % nw, j = e / nw;
        Tw[j * L + i] = CM(H, kwtop + i, kwtop + j, ldh);
        Zl[j * L + i] = (i == j) ? T(1) : T(0);
    }
    __syncthreads();
    int nsw = 0, nst = 0;
    const long long c0 = clock64();
    int st;
    if (nw <= 64) {
        // one wavefront, no barriers; the others wait for its status
        if (tid < 64) {
            st = francis_wave<T>(nw, Tw, L, Zl, L, nw, &nsw, &nst);
            if (tid == 0) sint[1] = st;
        }
        __syncthreads();
        st = sint[1];
    } else {
        st = francis_lds<T, NT>(nw, Tw, L, Zl, L, nw, sint + 1, &nsw, &nst);
    }
    const long long c1 = clock64();
    if (tid == 0) { out[3] = nsw; out[4] = nst; out[5] = (int)((c1 - c0) >> 10); }
    if (st) {
        if (tid == 0) { out[0] = 1; out[1] = 0; out[2] = 0; }
        return;  // window left untouched in global memory
    }
    const T s = spike_on ? CM(H, kwtop, kwtop - 1, ldh) : T(0);
    for (int j = tid; j < nw; j += NT) sp[j] = s * Zl[j * L];
    __syncthreads();
    // deflation test from the bottom (no reordering)
    const T ulp = num<T>::ulp, smlnum = num<T>::safmin * T(nw) / num<T>::ulp;
    int ns = nw;
    while (ns > 0) {
        bool two = (ns >= 2) && (Tw[(ns - 2) * L + (ns - 1)] != T(0));
        if (!two) {
            T foo = fabs(Tw[(ns - 1) * L + (ns - 1)]);
            if (foo == T(0)) foo = fabs(s);
            if (fabs(sp[ns - 1]) <= fmax(smlnum, ulp * foo)) ns -= 1;
            else break;
        } else {
            T foo = fabs(Tw[(ns - 1) * L + (ns - 1)]) +
                    sqrt(fabs(Tw[(ns - 2) * L + (ns - 1)])) * sqrt(fabs(Tw[(ns - 1) * L + (ns - 2)]));
            if (foo == T(0)) foo = fabs(s);
            if (fmax(fabs(sp[ns - 1]), fabs(sp[ns - 2])) <= fmax(smlnum, ulp * foo)) ns -= 2;
            else break;
        }
    }
    // eigenvalues of the undeflated part (shift candidates)
    if (tid == 0) {
        int i = 0;
        while (i < ns) {
            if (i + 1 < ns && Tw[i * L + i + 1] != T(0)) {
                T a = Tw[i * L + i], b = Tw[(i + 1) * L + i];
                T c = Tw[i * L + i + 1], d = Tw[(i + 1) * L + i + 1];
                T p = T(0.5) * (a - d), disc = p * p + b * c, mid = T(0.5) * (a + d);
                if (disc >= T(0)) {
                    T r = sqrt(disc);
                    wr[i] = mid + r; wr[i + 1] = mid - r; wi[i] = wi[i + 1] = T(0);
                } else {
                    T r = sqrt(-disc);
                    wr[i] = wr[i + 1] = mid; wi[i] = r; wi[i + 1] = -r;
                }
                i += 2;
            } else {
                wr[i] = Tw[i * L + i]; wi[i] = T(0);
                i += 1;
            }
        }
    }
    for (int j = ns + tid; j < nw; j += NT) sp[j] = T(0);
    __syncthreads();
    T newsub = (ns >= 1) ? sp[0] : T(0);
    if (ns > 1 && s != T(0)) {
        // reflect the spike onto its first entry: P sp = beta e1, P = I - tau v v^T
        // (v stored in sp with v[0] = 1)
        __shared__ T sh_tau, sh_beta;
        if (tid < 64) house_wave<T>(ns, sp, sp, &sh_tau, &sh_beta);
        __syncthreads();
        const T tau = sh_tau;
        newsub = sh_beta;
        if (tau != T(0)) {
            // left: rows 0..ns-1, all columns
            for (int j = tid; j < nw; j += NT) {
                T acc = T(0);
                for (int i = 0; i < ns; ++i) acc += sp[i] * Tw[j * L + i];
                acc *= tau;
                for (int i = 0; i < ns; ++i) Tw[j * L + i] -= acc * sp[i];
            }
            __syncthreads();
            // right: columns 0..ns-1, rows 0..ns-1 (rows below are zero there)
            for (int i = tid; i < ns; i += NT) {
                T acc = T(0);
                for (int j = 0; j < ns; ++j) acc += Tw[j * L + i] * sp[j];
                acc *= tau;
                for (int j = 0; j < ns; ++j) Tw[j * L + i] -= acc * sp[j];
            }
            for (int i = tid; i < nw; i += NT) {
                T acc = T(0);
                for (int j = 0; j < ns; ++j) acc += Zl[j * L + i] * sp[j];
                acc *= tau;
                for (int j = 0; j < ns; ++j) Zl[j * L + i] -= acc * sp[j];
            }
            __syncthreads();
        }
        // Householder reduction of Tw(0:ns, 0:ns) back to Hessenberg form;
        // the left reflectors also act on columns ns..nw-1.  Per column: the
        // reflector on wavefront 0; then the left update of the columns to
        // the right and the update of Z side by side, then the right update
        // of rows 0..ns-1; each dot product split over an aligned group of
        // RG lanes (strided over the vector) and summed by shuffles.
        constexpr int RG = 8, NG = NT / RG;
        T *v = sp;  // reuse
        const int grp = tid / RG, sub = tid % RG;
        for (int c = 0; c + 2 < ns; ++c) {
            const int len = ns - c - 1;  // rows c+1..ns-1
            if (tid < 64) house_wave<T>(len, Tw + c * L + c + 1, v, &sh_tau, &sh_beta);
            __syncthreads();
            const T tau = sh_tau;
            // column c becomes (beta, 0, ..., 0) below its diagonal (no update
            // of this column reads it)
            for (int i = tid; i < len; i += NT) Tw[c * L + c + 1 + i] = (i == 0) ? sh_beta : T(0);
            if (tau != T(0)) {
                const int ncol = nw - c - 1;
                for (int gi = grp; gi < ncol + nw; gi += NG) {
                    const bool lft = gi < ncol;
                    // left: column j = c+1+gi, entries Tw(c+1+i, j); Z: row zi, entries Zl(zi, c+1+i)
                    T *base = lft ? Tw + (size_t)(c + 1 + gi) * L + c + 1 : Zl + (size_t)(c + 1) * L + (gi - ncol);
                    const int step = lft ? 1 : L;
                    T acc = T(0);
                    for (int i = sub; i < len; i += RG) acc += v[i] * base[i * step];
#pragma unroll
                    for (int o = 1; o < RG; o <<= 1) acc += __shfl_xor(acc, o);
                    acc *= tau;
                    for (int i = sub; i < len; i += RG) base[i * step] -= acc * v[i];
                }
                __syncthreads();
                for (int gi = grp; gi < ns; gi += NG) {
                    // right: row gi, entries Tw(gi, c+1+j)
                    T *base = Tw + (size_t)(c + 1) * L + gi;
                    T acc = T(0);
                    for (int j = sub; j < len; j += RG) acc += base[(size_t)j * L] * v[j];
#pragma unroll
                    for (int o = 1; o < RG; o <<= 1) acc += __shfl_xor(acc, o);
                    acc *= tau;
                    for (int j = sub; j < len; j += RG) base[(size_t)j * L] -= acc * v[j];
                }
            }
            __syncthreads();
        }
    }
    // write back: window, spike column, Zw
    for (int e = tid; e < nw * nw; e += NT) {
        int i = e % nw, j = e / nw;
        CM(H, kwtop + i, kwtop + j, ldh) = Tw[j * L + i];
        Zw[e] = Zl[j * L + i];
    }
    if (spike_on) {
        for (int i = tid; i < nw; i += NT) CM(H, kwtop + i, kwtop - 1, ldh) = (i == 0) ? newsub : T(0);
    }
    if (tid == 0) { out[0] = 0; out[1] = nw - ns; out[2] = ns; }
}

template <typename T>
size_t aed_smem(int nw) {
    return sizeof(T) * ((size_t)2 * (nw | 1) * nw + nw) + 8 * sizeof(int);
}

// Raises a kernel's dynamic-LDS limit to at least sm bytes (once per size).
static int lds_limit(const void *kfn, size_t sm, size_t &attr_set, std::mutex &mu) {
    std::lock_guard<std::mutex> lk(mu);
    if (sm > attr_set) {
        if (hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm) != hipSuccess) {
            (void)hipGetLastError();
            return -1;
        }
        attr_set = sm;
    }
    return 0;
}

// waves: 4 (256 threads: one wave per role, windows <= 64 in one pass) or 7
// (448 threads: two waves per role)
template <typename T>
int aed_launch(hipStream_t s, int nw, T *H, int ldh, int kwtop, int spike_on, T *Zw, int *out,
               T *wr, T *wi, int waves) {
    size_t sm = aed_smem<T>(nw);
    if (sm > 160 * 1024) return -1;
    static std::mutex mu;
    static size_t attr4 = 0, attr7 = 0;
    ProfScope ps(KID_AED, s);
    if (waves == 4) {
        auto kfn = k_aed<T, 256>;
        if (lds_limit((const void *)kfn, sm, attr4, mu)) return -1;
        hipLaunchKernelGGL(kfn, dim3(1), dim3(256), sm, s, nw, H, ldh, kwtop, spike_on, Zw, out, wr, wi);
    } else {
        auto kfn = k_aed<T, 448>;
        if (lds_limit((const void *)kfn, sm, attr7, mu)) return -1;
        hipLaunchKernelGGL(kfn, dim3(1), dim3(448), sm, s, nw, H, ldh, kwtop, spike_on, Zw, out, wr, wi);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int aed_launch<float>(hipStream_t, int, float *, int, int, int, float *, int *, float *, float *, int);
template int aed_launch<double>(hipStream_t, int, double *, int, int, int, double *, int *, double *, double *,
                                int);
template size_t aed_smem<float>(int);
template size_t aed_smem<double>(int);

// ------------------------------------------------------------- k_chase
// One phase of a multishift sweep over the active block [ktop, kbot].
// Bulge b (0-based, b = 0 introduced first) of a chain sits at position
// p = t - 3b at the chain's time t (its reflector acts on rows/cols
// ktop+p .. ktop+p+2; p = 0 is the introduction, p = N-2 the 2x2 exit step,
// N = kbot-ktop+1).  The phase runs times t0 .. t0+adv-1 inside the window
// [ws, ws+W) of H, which is loaded to LDS; Uw (W x W, LDS) accumulates the
// window's orthogonal factor and is written to global memory for the
// off-window GEMM updates.  A sweep's bulges may form several chains, each
// introduced one window width after the one below it (two QR steps whose
// shift sets multiply to the sweep's shift polynomial): their windows are
// disjoint, and workgroup g chases chain window g of the launch.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_chase(T *H, int ldh, int ktop, int kbot, ChaseSet<T> set, int adv) {
    const ChaseWin<T> cw = set.w[blockIdx.x];
    const int ws = cw.ws, W = cw.W, t0 = cw.t0, nbulge = cw.nbulge;
    const T *trd = cw.trd;
    T *Uw_out = cw.Uw;
    extern __shared__ unsigned char smem_raw[];
    const int L = W | 1;  // odd leading dimension: conflict-free row-wise access
    T *Hw = reinterpret_cast<T *>(smem_raw);
    T *Uw = Hw + L * W;
    // per bulge and time parity: v1, v2, tau, beta and q (or -1), len, ulo, uhi
    T *refl = Uw + L * W;
    int *rinfo = reinterpret_cast<int *>(refl + 8 * nbulge);
    int *ulo = rinfo + 8 * nbulge;  // per column of Uw: nonzero row range
    int *uhi = ulo + W;
    const int tid = threadIdx.x;
    const int N = kbot - ktop + 1;
    for (int e = tid; e < W * W; e += NT) {
        int i = e % W, j = e / W;
        Hw[j * L + i] = CM(H, ws + i, ws + j, ldh);
        Uw[j * L + i] = (i == j) ? T(1) : T(0);
    }
    for (int j = tid; j < W; j += NT) { ulo[j] = j; uhi[j] = j; }
    __syncthreads();
    const int kb = kbot - ws;  // local index of kbot
    const int tpb = NT / nbulge;             // phase A: threads per bulge
    const int myb = tid / tpb, slot = tid % tpb;
    // phase B: lane b of wavefront 0 leads bulge b (nbulge <= 64); the other
    // wavefronts split the bulges' remaining rows, tpr threads per bulge
    const int tpr = (NT - 64) / nbulge;
    const int rb = (tid - 64) / tpr, rslot = (tid - 64) % tpr;
    // Reflector of bulge b from its column (x, y, z) into parity buf, with
    // the row range of Uw its columns can touch (interval hull of the three
    // columns' ranges; columns of distinct bulges are disjoint).
    auto commit = [&](int b, int buf, int q, int len, T x, T y, T z) {
        T v1, v2, tau, beta;
        reflector3(len, x, y, z, v1, v2, tau, beta);
        T *rf = refl + 4 * (buf * nbulge + b);
        rf[0] = v1; rf[1] = v2; rf[2] = tau; rf[3] = beta;
        int lo = ulo[q], hi = uhi[q];
        for (int c = 1; c < len; ++c) { lo = min(lo, ulo[q + c]); hi = max(hi, uhi[q + c]); }
        for (int c = 0; c < len; ++c) { ulo[q + c] = lo; uhi[q + c] = hi; }
        int *ri = rinfo + 4 * (buf * nbulge + b);
        ri[0] = q; ri[1] = len; ri[2] = lo; ri[3] = hi;
    };
    // Reflector of bulge b at time t read from the window: at the start of
    // the phase, and for a bulge introduced mid-phase (its first column
    // depends on the previous bulge's last updates).
    auto form = [&](int b, int t, int buf) {
        const int p = t - 3 * b;
        if (p < 0 || p > N - 2) { rinfo[4 * (buf * nbulge + b)] = -1; return; }
        const int q = ktop + p - ws;  // local row of the reflector
        const int len = (p <= N - 3) ? 3 : 2;
        T x, y, z;
        if (p == 0) {
            shift_column(Hw[q * L + q], Hw[(q + 1) * L + q], Hw[q * L + q + 1], Hw[(q + 1) * L + q + 1],
                         Hw[(q + 1) * L + q + 2], trd[3 * b], trd[3 * b + 1], trd[3 * b + 2] != T(0), x, y, z);
        } else {
            x = Hw[(q - 1) * L + q];
            y = Hw[(q - 1) * L + q + 1];
            z = Hw[(q - 1) * L + ((len == 3) ? q + 2 : q + 1)];
        }
        commit(b, buf, q, len, x, y, z);
    };
    for (int b = tid; b < nbulge; b += NT) form(b, t0, t0 & 1);
    __syncthreads();
    for (int t = t0; t < t0 + adv; ++t) {
        const int buf = t & 1;
        if (t > t0 && t >= 0 && t % 3 == 0 && t / 3 < nbulge) {
            if (tid == 0) form(t / 3, t, buf);
            __syncthreads();
        }
        // Each active bulge gets a fixed group of tpb threads; a thread works
        // only on its own bulge, so there is no sequential loop over bulges.
        // phase A: left applications, rows q..q+len-1, columns q-1 (p>0: set
        // beta, zeros) and q..W-1.  Distinct bulges touch distinct rows.
        if (myb < nbulge) {
            const int *ri = rinfo + 4 * (buf * nbulge + myb);
            const int q = ri[0];
            if (q >= 0) {
                const int len = ri[1];
                const T *rf = refl + 4 * (buf * nbulge + myb);
                const T v1 = rf[0], v2 = rf[1], tau = rf[2];
                const bool intro = (t - 3 * myb == 0);
                const int c0 = intro ? q : q - 1;
                const int q2 = (len == 3) ? q + 2 : q + 1;  // clamped third row
#pragma unroll 2
                for (int j = c0 + slot; j < W; j += tpb) {
                    if (!intro && j == q - 1) {
                        Hw[j * L + q2] = T(0);
                        Hw[j * L + q + 1] = T(0);
                        Hw[j * L + q] = rf[3];
                        continue;
                    }
                    T a0 = Hw[j * L + q], a1 = Hw[j * L + q + 1], a2 = Hw[j * L + q2];
                    refl_apply(len, v1, v2, tau, a0, a1, a2);
                    Hw[j * L + q2] = a2; Hw[j * L + q] = a0; Hw[j * L + q + 1] = a1;
                }
            }
        }
        __syncthreads();
        // phase B: right applications on columns q..q+len-1 (rows 0..min(q+3, kb))
        // and on Uw (rows ulo..uhi only).  Distinct bulges touch distinct
        // columns.  The rows q+1..q+3 hold the bulge's next column (column q
        // after this step): the bulge's lead lane in wavefront 0 updates them
        // itself and forms the next step's reflector from them, so there is
        // no separate reflector phase (no other bulge touches column q in this
        // step), and the leads run side by side in one wavefront.
        if (tid < 64) {
            const int b = tid;
            if (b < nbulge) {
                const int *ri = rinfo + 4 * (buf * nbulge + b);
                const int q = ri[0];
                int *rn = rinfo + 4 * ((buf ^ 1) * nbulge + b);
                if (q >= 0) {
                    const int len = ri[1];
                    const T *rf = refl + 4 * (buf * nbulge + b);
                    const T v1 = rf[0], v2 = rf[1], tau = rf[2];
                    int rmax = q + 3 < kb ? q + 3 : kb;
                    if (rmax > W - 1) rmax = W - 1;
                    const int q2 = (len == 3) ? q + 2 : q + 1;
                    // rows q+1..rmax (1..3 of them): all loads first (a
                    // missing third row repeats the last one, stored once),
                    // then the updates, then the stores
                    const int nrow = rmax - q;
                    T r0[3], r1[3], r2[3];
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        const int i = q + 1 + (u < nrow ? u : nrow - 1);
                        r0[u] = Hw[q * L + i]; r1[u] = Hw[(q + 1) * L + i]; r2[u] = Hw[q2 * L + i];
                    }
#pragma unroll
                    for (int u = 0; u < 3; ++u) refl_apply(len, v1, v2, tau, r0[u], r1[u], r2[u]);
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        if (u < nrow) {
                            const int i = q + 1 + u;
                            Hw[q2 * L + i] = r2[u]; Hw[q * L + i] = r0[u]; Hw[(q + 1) * L + i] = r1[u];
                        }
                    }
                    const T nx = r0[0], ny = nrow >= 2 ? r0[1] : T(0), nz = nrow >= 3 ? r0[2] : T(0);
                    const int pn = t + 1 - 3 * b;
                    if (t + 1 < t0 + adv && pn <= N - 2)
                        commit(b, buf ^ 1, q + 1, (pn <= N - 3) ? 3 : 2, nx, ny, nz);
                    else
                        rn[0] = -1;
                } else {
                    rn[0] = -1;
                }
            }
        } else if (rb < nbulge) {
            const int *ri = rinfo + 4 * (buf * nbulge + rb);
            const int q = ri[0];
            if (q >= 0) {
                const int len = ri[1];
                const int lo = ri[2], hi = ri[3];
                const T *rf = refl + 4 * (buf * nbulge + rb);
                const T v1 = rf[0], v2 = rf[1], tau = rf[2];
                int rmax = q + 3 < kb ? q + 3 : kb;
                if (rmax > W - 1) rmax = W - 1;
                const int nr = q + 1;  // rows 0..q here; q+1..rmax go to the lead lane
                const int nu = hi - lo + 1;
                const int q2 = (len == 3) ? q + 2 : q + 1;  // clamped third column
#pragma unroll 2
                for (int e = rslot; e < nr + nu; e += tpr) {
                    T *M = (e < nr) ? Hw : Uw;
                    int i = (e < nr) ? e : lo + (e - nr);
                    T a0 = M[q * L + i], a1 = M[(q + 1) * L + i], a2 = M[q2 * L + i];
                    refl_apply(len, v1, v2, tau, a0, a1, a2);
                    M[q2 * L + i] = a2; M[q * L + i] = a0; M[(q + 1) * L + i] = a1;
                }
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < W * W; e += NT) {
        int i = e % W, j = e / W;
        CM(H, ws + i, ws + j, ldh) = Hw[j * L + i];
        Uw_out[e] = Uw[j * L + i];
    }
}

template <typename T>
size_t chase_smem(int W, int nbulge) {
    return sizeof(T) * ((size_t)2 * (W | 1) * W + 8 * nbulge) + sizeof(int) * (8 * nbulge + 2 * W);
}

template <typename T>
int chase_launch(hipStream_t s, T *H, int ldh, int ktop, int kbot, const ChaseSet<T> &set, int nwin, int adv,
                 int waves) {
    if (nwin < 1 || nwin > kChaseMaxWin) return -1;
    size_t sm = 0;
    for (int g = 0; g < nwin; ++g) {
        const int nbulge = set.w[g].nbulge;
        if (nbulge < 1 || nbulge > 64 || (64 * waves - 64) / nbulge < 1) return -1;  // one lead lane per bulge
        sm = std::max(sm, chase_smem<T>(set.w[g].W, nbulge));
    }
    if (sm > 160 * 1024) return -1;
    static std::mutex mu;
    static size_t attr8 = 0, attr16 = 0;
    auto k8 = k_chase<T, 512>;
    auto k16 = k_chase<T, 1024>;
    if (lds_limit(waves == 8 ? (const void *)k8 : (const void *)k16, sm, waves == 8 ? attr8 : attr16, mu))
        return -1;
    if (prof_armed(KID_CHASE)) {
        // algorithmic flops of this phase: every application of a bulge's
        // reflector to one row or column (length 3: 12 flops, length 2: 8),
        // left (window columns right of the bulge), right (window rows up to
        // the bulge) and on the window's orthogonal factor
        const int N = kbot - ktop + 1;
        double fl = 0.0;
        for (int g = 0; g < nwin; ++g) {
            const ChaseWin<T> &cw = set.w[g];
            const int kb = kbot - cw.ws, W = cw.W;
            for (int t = cw.t0; t < cw.t0 + adv; ++t)
                for (int b = 0; b < cw.nbulge; ++b) {
                    int p = t - 3 * b;
                    if (p < 0 || p > N - 2) continue;
                    int q = ktop + p - cw.ws, len = (p <= N - 3) ? 3 : 2;
                    int rmax = q + 3 < kb ? q + 3 : kb;
                    if (rmax > W - 1) rmax = W - 1;
                    fl += (len == 3 ? 12.0 : 8.0) * ((W - q) + (rmax + 1) + W);
                }
        }
        prof_add_work(KID_CHASE, fl);
    }
    {
        ProfScope ps(KID_CHASE, s);
        if (waves == 8)
            hipLaunchKernelGGL(k8, dim3(nwin), dim3(512), sm, s, H, ldh, ktop, kbot, set, adv);
        else
            hipLaunchKernelGGL(k16, dim3(nwin), dim3(1024), sm, s, H, ldh, ktop, kbot, set, adv);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int chase_launch<float>(hipStream_t, float *, int, int, int, const ChaseSet<float> &, int, int, int);
template int chase_launch<double>(hipStream_t, double *, int, int, int, const ChaseSet<double> &, int, int, int);
template size_t chase_smem<float>(int, int);
template size_t chase_smem<double>(int, int);

// ------------------------------------------------------- small utilities

// Largest k in [klo+1, kbot] with a negligible subdiagonal H(k, k-1) (which is
// then set to exact zero), or klo if none.  Written to *out.
template <typename T>
__global__ __launch_bounds__(256) void k_find_ktop(T *H, int ldh, int klo, int kbot, int *out) {
    __shared__ int best;
    if (threadIdx.x == 0) best = klo;
    __syncthreads();
    const T ulp = num<T>::ulp, smlnum = num<T>::safmin * T(kbot + 1) / num<T>::ulp;
    for (int k = klo + 1 + threadIdx.x; k <= kbot; k += blockDim.x) {
        T hk = fabs(CM(H, k, k - 1, ldh));
        T tst = fabs(CM(H, k - 1, k - 1, ldh)) + fabs(CM(H, k, k, ldh));
        if (tst == T(0)) {
            if (k - 2 >= klo) tst += fabs(CM(H, k - 1, k - 2, ldh));
            if (k + 1 <= kbot) tst += fabs(CM(H, k + 1, k, ldh));
        }
        if (hk <= fmax(smlnum, ulp * tst)) atomicMax(&best, k);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (best > klo) CM(H, best, best - 1, ldh) = T(0);
        *out = best;
    }
}
template <typename T>
void find_ktop(hipStream_t s, T *H, int ldh, int klo, int kbot, int *out) {
    ProfScope ps(KID_FIND_KTOP, s);
    hipLaunchKernelGGL((k_find_ktop<T>), dim3(1), dim3(256), 0, s, H, ldh, klo, kbot, out);
}
template void find_ktop<float>(hipStream_t, float *, int, int, int, int *);
template void find_ktop<double>(hipStream_t, double *, int, int, int, int *);

// Trailing entries for exceptional shifts, written to out (host-mapped or
// device memory): out[2q] = H(i0+q, i0+q), out[2q+1] = H(i0+q, i0+q-1) for
// q < m, out[2m] = H(i0-1, i0-2).  Requires i0 >= 2.
template <typename T>
__global__ __launch_bounds__(256) void k_gather_sub(const T *H, int ldh, int i0, int m, T *out) {
    for (int q = threadIdx.x; q <= m; q += blockDim.x) {
        if (q < m) {
            out[2 * q] = CM(H, i0 + q, i0 + q, ldh);
            out[2 * q + 1] = CM(H, i0 + q, i0 + q - 1, ldh);
        } else {
            out[2 * m] = CM(H, i0 - 1, i0 - 2, ldh);
        }
    }
}
template <typename T>
void gather_sub(hipStream_t s, const T *H, int ldh, int i0, int m, T *out) {
    hipLaunchKernelGGL((k_gather_sub<T>), dim3(1), dim3(256), 0, s, H, ldh, i0, m, out);
}
template void gather_sub<float>(hipStream_t, const float *, int, int, int, float *);
template void gather_sub<double>(hipStream_t, const double *, int, int, int, double *);

// Split a converged 2x2 block at (k, k) of the full n x n H (global) if its
// eigenvalues are real; rotate rows k,k+1 / cols k,k+1 of H and U.
template <typename T>
__global__ __launch_bounds__(256) void k_std2x2(int n, T *H, int ldh, T *U, int ldu, int k) {
    T a = CM(H, k, k, ldh), b = CM(H, k, k + 1, ldh);
    T c = CM(H, k + 1, k, ldh), d = CM(H, k + 1, k + 1, ldh);
    if (c == T(0)) return;
    T p = T(0.5) * (a - d), disc = p * p + b * c;
    if (disc < T(0)) return;
    T e1 = p + copysign(sqrt(disc), p);
    T nv = hypot(e1, c);
    T cs = e1 / nv, sn = c / nv;
    __syncthreads();
    for (int j = k + threadIdx.x; j < n; j += blockDim.x) {
        T t1 = CM(H, k, j, ldh), t2 = CM(H, k + 1, j, ldh);
        CM(H, k, j, ldh) = cs * t1 + sn * t2;
        CM(H, k + 1, j, ldh) = cs * t2 - sn * t1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= k + 1; i += blockDim.x) {
        T t1 = CM(H, i, k, ldh), t2 = CM(H, i, k + 1, ldh);
        CM(H, i, k, ldh) = cs * t1 + sn * t2;
        CM(H, i, k + 1, ldh) = cs * t2 - sn * t1;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        T t1 = CM(U, i, k, ldu), t2 = CM(U, i, k + 1, ldu);
        CM(U, i, k, ldu) = cs * t1 + sn * t2;
        CM(U, i, k + 1, ldu) = cs * t2 - sn * t1;
    }
    __syncthreads();
    if (threadIdx.x == 0) CM(H, k + 1, k, ldh) = T(0);
}
template <typename T>
void std2x2(hipStream_t s, int n, T *H, int ldh, T *U, int ldu, int k) {
    hipLaunchKernelGGL((k_std2x2<T>), dim3(1), dim3(256), 0, s, n, H, ldh, U, ldu, k);
}
template void std2x2<float>(hipStream_t, int, float *, int, float *, int, int);
template void std2x2<double>(hipStream_t, int, double *, int, double *, int, int);

// Zero every entry below the first subdiagonal (n x n).
template <typename T>
__global__ void k_clean_lower(int n, T *H, int ldh) {
    size_t total = (size_t)n * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(e % n), j = (int)(e / n);
        if (i > j + 1) H[(size_t)j * ldh + i] = T(0);
    }
}
template <typename T>
void clean_lower(hipStream_t s, int n, T *H, int ldh) {
    if (n <= 0) return;
    size_t g = ((size_t)n * n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL((k_clean_lower<T>), dim3((int)g), dim3(256), 0, s, n, H, ldh);
}
template void clean_lower<float>(hipStream_t, int, float *, int);
template void clean_lower<double>(hipStream_t, int, double *, int);

}  // namespace sylv
