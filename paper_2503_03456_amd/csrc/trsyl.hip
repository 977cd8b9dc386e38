// Quasi-triangular Sylvester equation TA Y + Y TB = C (the substitution step
// of the Bartels-Stewart algorithm, paper Sec. 2.2.1), TA m x m and TB n x n
// upper quasi-triangular, C overwritten by Y.
//
// GPU formulation: Y is cut into tiles of at most 64 x 64 whose boundaries
// never split a 2x2 diagonal block.  Tile (I, J) depends on the tiles below
// it in its block column (through TA) and on the tiles left of it in its
// block row (through TB), so all tiles on one anti-diagonal (counted from
// the bottom-left corner) are independent: one launch per anti-diagonal,
// one workgroup per tile.  The updated right-hand side
//        C_IJ - TA(I, below) Y(below, J) - Y(I, left) TB(left, J)
// is formed on MFMA: right-looking for a single equation (after each
// anti-diagonal, k_trsyl_update subtracts its contributions from every later
// tile on the whole chip), left-looking inside the tile's own workgroup for
// the batched form.  Each tile's workgroup then solves the small
// quasi-triangular tile equation in LDS by a wavefront over its 1x1/2x2
// diagonal-block pairs: every pair is a p*q <= 4 linear system, embedded in
// a fixed 4x4 system and solved by Gaussian elimination with partial
// pivoting; a pivot below s_min = u * max(max|TA|, max|TB|) is replaced by
// +-s_min and a flag is raised (the usual triangular-Sylvester convention).
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace sylv {

template <typename T> struct mfma16t;
template <> struct mfma16t<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static SYLV_DEVINL v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static SYLV_DEVINL int orow(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct mfma16t<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static SYLV_DEVINL v4 op(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static SYLV_DEVINL int orow(int l, int r) { return (l >> 4) + 4 * r; }
};

// Sums of x over aligned groups of g lanes (g a power of two <= 64, uniform):
// the last lane of each group ends with its group's sum (other lanes hold
// partial sums).  Doubling row shifts within rows of 16, then the row
// broadcasts for groups of 32 and 64.
template <typename T>
SYLV_DEVINL void group_sum4(T (&x)[4], int g) {
    if (g > 1) {
#pragma unroll
        for (int z = 0; z < 4; ++z) x[z] += dpp_move<0x111>(x[z]);
    }
    if (g > 2) {
#pragma unroll
        for (int z = 0; z < 4; ++z) x[z] += dpp_move<0x112>(x[z]);
    }
    if (g > 4) {
#pragma unroll
        for (int z = 0; z < 4; ++z) x[z] += dpp_move<0x114>(x[z]);
    }
    if (g > 8) {
#pragma unroll
        for (int z = 0; z < 4; ++z) x[z] += dpp_move<0x118>(x[z]);
    }
    if (g > 16) {
#pragma unroll
        for (int z = 0; z < 4; ++z) x[z] += dpp_move<0x142>(x[z]);
    }
    if (g > 32) {
#pragma unroll
        for (int z = 0; z < 4; ++z) x[z] += dpp_move<0x143>(x[z]);
    }
}

constexpr int TS = 64;       // tile capacity
constexpr int TBASE = 63;    // nominal boundary spacing (adjusted by +1 at 2x2 blocks)
constexpr int TLD = TS + 1;  // LDS leading dimension of tiles
constexpr int TBK = 32;      // K slab of the in-tile MFMA update
// threads of a single-equation tile workgroup: 512 with the staged inverses
// (binary32), 256 with the in-place eliminations (measured best of 256/512/1024)
constexpr int TRSYL_NT_PRE = 512, TRSYL_NT = 256;

// Boundary k of a quasi-triangular matrix of order n cut every TBASE rows.
template <typename T>
SYLV_DEVINL int tile_bound(const T *Tm, int ld, int n, int k) {
    int b = k * TBASE;
    if (b <= 0) return 0;
    if (b >= n) return n;
    if (CM(Tm, b, b - 1, ld) != T(0)) b += 1;
    return b;
}

// Block-pair system of the tri-solve: TA_ii Y + Y TB_jj = R with TA_ii, TB_jj
// of order 1 or 2.  The unknowns are embedded in a fixed 4-vector
// (y00, y10, y01, y11) -- an order-1 block leaves its entries as identity
// rows -- so every lane runs the same straight-line code with static
// register indices: Gaussian elimination with partial pivoting, a pivot
// below smin replaced by +-smin (flag set).  Each pivot's reciprocal is
// formed once (hardware reciprocal, Newton-refined in binary64) and serves
// both the elimination and the back substitution.
template <typename T>
SYLV_DEVINL int pair_solve(bool P, bool Q, T a00, T a01, T a10, T a11, T b00, T b01, T b10, T b11,
                           T r[4], T smin) {
    T m[4][4];
    const T zp = P ? T(1) : T(0), zq = Q ? T(1) : T(0), zpq = zp * zq;
    m[0][0] = a00 + b00;       m[0][1] = a01 * zp;        m[0][2] = b10 * zq;        m[0][3] = T(0);
    m[1][0] = a10 * zp;        m[1][1] = P ? a11 + b00 : T(1); m[1][2] = T(0);      m[1][3] = b10 * zpq;
    m[2][0] = b01 * zq;        m[2][1] = T(0);            m[2][2] = Q ? a00 + b11 : T(1); m[2][3] = a01 * zpq;
    m[3][0] = T(0);            m[3][1] = b01 * zpq;       m[3][2] = a10 * zpq;       m[3][3] = (P && Q) ? a11 + b11 : T(1);
    if (!P) r[1] = T(0);
    if (!Q) r[2] = T(0);
    if (!(P && Q)) r[3] = T(0);
    int flag = 0;
    T inv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        // pivot: largest |m[r][c]|, r >= c; swap it into row c with selects
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
        if (fabs(piv) < smin) {
            piv = (piv >= T(0)) ? smin : -smin;
            m[c][c] = piv;
            flag = 1;
        }
        inv[c] = frcp(piv);
#pragma unroll
        for (int rr = c + 1; rr < 4; ++rr) {
            const T f = m[rr][c] * inv[c];
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
        r[c] = acc * inv[c];
    }
    return flag;
}

// Inverse of the embedded 4 x 4 block-pair matrix of pair_solve (same
// pivoting and s_min rule): Minv[k][l], rows and columns in the unknown order
// (y00, y10, y01, y11).  The embedding keeps real and dummy unknowns
// uncoupled, so the real rows of Minv vanish in the dummy columns.
template <typename T>
SYLV_DEVINL int pair_inverse(bool P, bool Q, T a00, T a01, T a10, T a11, T b00, T b01, T b10, T b11,
                             T Minv[4][4], T smin) {
    T m[4][4], r[4][4];
    const T zp = P ? T(1) : T(0), zq = Q ? T(1) : T(0), zpq = zp * zq;
    m[0][0] = a00 + b00;       m[0][1] = a01 * zp;        m[0][2] = b10 * zq;        m[0][3] = T(0);
    m[1][0] = a10 * zp;        m[1][1] = P ? a11 + b00 : T(1); m[1][2] = T(0);      m[1][3] = b10 * zpq;
    m[2][0] = b01 * zq;        m[2][1] = T(0);            m[2][2] = Q ? a00 + b11 : T(1); m[2][3] = a01 * zpq;
    m[3][0] = T(0);            m[3][1] = b01 * zpq;       m[3][2] = a10 * zpq;       m[3][3] = (P && Q) ? a11 + b11 : T(1);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) r[i][k] = (i == k) ? T(1) : T(0);
    int flag = 0;
    T inv[4];
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
                T u = r[c][k], v = r[rr][k];
                r[c][k] = sw ? v : u;
                r[rr][k] = sw ? u : v;
            }
        }
        T piv = m[c][c];
        if (fabs(piv) < smin) {
            piv = (piv >= T(0)) ? smin : -smin;
            m[c][c] = piv;
            flag = 1;
        }
        inv[c] = T(1) / piv;
#pragma unroll
        for (int rr = c + 1; rr < 4; ++rr) {
            const T f = m[rr][c] * inv[c];
#pragma unroll
            for (int k = c + 1; k < 4; ++k) m[rr][k] -= f * m[c][k];
#pragma unroll
            for (int k = 0; k < 4; ++k) r[rr][k] -= f * r[c][k];
        }
    }
#pragma unroll
    for (int col = 0; col < 4; ++col)
#pragma unroll
        for (int c = 3; c >= 0; --c) {
            T acc = r[c][col];
#pragma unroll
            for (int k = c + 1; k < 4; ++k) acc -= m[c][k] * Minv[k][col];
            Minv[c][col] = acc * inv[c];
        }
    return flag;
}

// acc += A B on MFMA for one output tile (p x q <= TS x TS): A is p x K
// (leading dimension lda_), B is K x q (ldb_).  The four wavefronts take a
// 2 x 2 grid of 32 x 32 output blocks; stA / stB are the LDS slabs.  All
// 256 threads call it.
template <typename T>
SYLV_DEVINL void tile_gemm(typename mfma16t<T>::v4 (&acc)[2][2], const T *Ap, int lda_, const T *Bp, int ldb_,
                           int K, int p, int q, T (*stA)[TS + 16], T (*stB)[TS + 16]) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int wm = w & 1, wn = w >> 1;
    // A slab: tile rows 0..p-1 x k0..k0+TBK-1 ; B slab: k0.. x tile cols 0..q-1.
    // Each thread holds 8 elements of each slab; the next slab is loaded
    // into registers while the current one feeds the MFMAs.
    // Loads at clamped addresses (p, q, K >= 1 here), masked by a 0/1
    // factor (the operands are finite): no branch per load, so the 16 loads
    // of a slab are in flight together.
    T ra[8], rb[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) {
            const int i = l, k = w + 4 * rr;
            const int ic = i < p ? i : p - 1, kc = k0 + k < K ? k0 + k : K - 1;
            ra[rr] = Ap[(size_t)kc * lda_ + ic] * T((i < p && k0 + k < K) ? 1 : 0);
            const int kk = t & 31, j = (t >> 5) + 8 * rr;
            const int jc = j < q ? j : q - 1, kkc = k0 + kk < K ? k0 + kk : K - 1;
            rb[rr] = Bp[(size_t)jc * ldb_ + kkc] * T((j < q && k0 + kk < K) ? 1 : 0);
        }
    };
    const int nk = (K + TBK - 1) / TBK;
    if (nk > 0) load(0);
    for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) {
            stA[w + 4 * rr][l] = ra[rr];
            stB[t & 31][(t >> 5) + 8 * rr] = rb[rr];
        }
        __syncthreads();
        if (kt + 1 < nk) load((kt + 1) * TBK);
#pragma unroll
        for (int kk = 0; kk < TBK / 4; ++kk) {
            const int kr = 4 * kk + (l >> 4);
            T fa[2], fb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) fa[a] = stA[kr][32 * wm + 16 * a + (l & 15)];
#pragma unroll
            for (int b = 0; b < 2; ++b) fb[b] = stB[kr][32 * wn + 16 * b + (l & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = mfma16t<T>::op(fb[b], fa[a], acc[a][b]);
        }
        __syncthreads();
    }
}

// One tile (I, J) of Y: off-diagonal updates (lazy: all of them here, the
// left-looking form; otherwise the right-looking updates of
// k_trsyl_update have already been applied to C), then the in-LDS solve.
// mirror (symmetric Lyapunov, m = n, TB = P TA^T P): the column tiles are
// the mirror images of the row tiles, c_J = n - r_{nt-J}, so that the
// solution Y' = Y P of a symmetric Y (persymmetric: Y'(i, j) =
// Y'(n-1-j, n-1-i)) maps tile (I, J) onto tile (nt-1-J, nt-1-I) of the same
// anti-diagonal; wmirror also stores that mirror tile.
// NT: threads of the workgroup (256 with the left-looking MFMA updates of
// the batched form; the single-equation form runs the same count: 1024
// threads, which spread each block pair's sums over more lanes, left the
// binary32 tile time unchanged and slowed the binary64 one).
// PRE: Pinv holds, for every element (i, j) of Y (at 4 ((size_t) j m + i)),
// the row of the inverse block-pair matrix for its unknown (k_trsyl_prep);
// the tile stages its part in LDS and each block pair's solve becomes a
// 4 x 4 matrix-vector product.
template <typename T, int NT = 256, bool PRE = false>
SYLV_DEVINL void trsyl_tile(int m, int n, const T *__restrict__ TA, int ldta, const T *__restrict__ TB,
                            int ldtb, T *C, int ldc, int I, int J, double maxab, int *flag, int mirror = 0,
                            int wmirror = 0, bool lazy = true, const T *__restrict__ Pinv = nullptr) {
    __shared__ T sA[TS * TLD];   // TA diagonal tile, later reused
    __shared__ T sB[TS * TLD];   // TB diagonal tile
    __shared__ T sC[TS * TLD];   // rhs -> Y tile
    typedef T t4 __attribute__((ext_vector_type(4)));
    __shared__ t4 sI[PRE ? TS * TS : 1];   // PRE: inverse rows, element (i, j) at j * TS + i
    __shared__ T stA[TBK][TS + 16];
    __shared__ T stB[TBK][TS + 16];
    __shared__ int rstart[TS + 1], cstart[TS + 1];
    __shared__ int nrb_s, ncb_s;
    typedef typename mfma16t<T>::v4 v4;

    const int r0 = tile_bound(TA, ldta, m, I), r1 = tile_bound(TA, ldta, m, I + 1);
    int c0, c1;
    if (mirror) {
        const int nt = (m + TBASE - 1) / TBASE;
        c0 = n - tile_bound(TA, ldta, m, nt - J);
        c1 = n - tile_bound(TA, ldta, m, nt - 1 - J);
    } else {
        c0 = tile_bound(TB, ldtb, n, J);
        c1 = tile_bound(TB, ldtb, n, J + 1);
    }
    const int p = r1 - r0, q = c1 - c0;
    if (p <= 0 || q <= 0) return;  // empty tile (uniform over the workgroup)
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int wm = w & 1, wn = w >> 1;

    // ---- 1. off-diagonal updates on MFMA (left-looking form): acc =
    //         TA(r0:r1, r1:m) Y(r1:m, c0:c1) + Y(r0:r1, 0:c0) TB(0:c0, c0:c1)
    if constexpr (NT == 256) {
        v4 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = v4{0, 0, 0, 0};
        if (lazy) {
            tile_gemm<T>(acc, TA + (size_t)r1 * ldta + r0, ldta, C + (size_t)c0 * ldc + r1, ldc, m - r1, p, q, stA,
                         stB);
            tile_gemm<T>(acc, C + r0, ldc, TB + (size_t)c0 * ldtb, ldtb, c0, p, q, stA, stB);
        }
        // rhs tile: sC(i, j) = C(r0+i, c0+j) - acc
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int i = 32 * wm + 16 * a + (l & 15);
                    int j = 32 * wn + 16 * b + mfma16t<T>::orow(l, r);
                    const int ic = i < p ? i : p - 1, jc = j < q ? j : q - 1;
                    const T cv = C[(size_t)(c0 + jc) * ldc + r0 + ic];
                    sC[j * TLD + i] = (cv - acc[a][b][r]) * T((i < p && j < q) ? 1 : 0);
                }
    } else {
        // the right-hand side is complete in C (right-looking updates)
        for (int e = t; e < TS * TS; e += NT) {
            const int i = e % TS, j = e / TS;
            const int ic = i < p ? i : p - 1, jc = j < q ? j : q - 1;
            sC[j * TLD + i] = C[(size_t)(c0 + jc) * ldc + r0 + ic] * T((i < p && j < q) ? 1 : 0);
        }
    }
    if constexpr (PRE) {
        // the tile's inverse rows: 16-byte loads, consecutive threads down a column
#pragma unroll 4
        for (int e = t; e < TS * TS; e += NT) {
            const int i = e % TS, j = e / TS;
            const int ic = i < p ? i : p - 1, jc = j < q ? j : q - 1;
            sI[j * TS + i] = *reinterpret_cast<const t4 *>(Pinv + 4 * ((size_t)(c0 + jc) * m + r0 + ic));
        }
    }
#pragma unroll 8
    for (int e = t; e < TS * TS; e += NT) {
        const int i = e % TS, j = e / TS;
        const T av = CM(TA, r0 + (i < p ? i : p - 1), r0 + (j < p ? j : p - 1), ldta);
        const T bv = CM(TB, c0 + (i < q ? i : q - 1), c0 + (j < q ? j : q - 1), ldtb);
        sA[j * TLD + i] = av * T((i < p && j < p) ? 1 : 0);
        sB[j * TLD + i] = bv * T((i < q && j < q) ? 1 : 0);
    }
    __syncthreads();
    // block structure of the diagonal tiles (start rows of 1x1/2x2 blocks)
    if (t == 0) {
        int nb = 0, i = 0;
        while (i < p) { rstart[nb++] = i; i += (i + 1 < p && sA[i * TLD + i + 1] != T(0)) ? 2 : 1; }
        rstart[nb] = p;
        nrb_s = nb;
        nb = 0; i = 0;
        while (i < q) { cstart[nb++] = i; i += (i + 1 < q && sB[i * TLD + i + 1] != T(0)) ? 2 : 1; }
        cstart[nb] = q;
        ncb_s = nb;
    }
    __syncthreads();
    const int P = nrb_s, Q = ncb_s;
    const T smin = (T)fmax((double)num<T>::ulp * maxab, (double)num<T>::safmin);
    int myflag = 0;
    // ---- 2. wavefront over block pairs: unit (ib, jb), ib counted from the
    // bottom; anti-diagonal e = ib + jb.  A unit's sums over the solved rows
    // below and columns to the left are split over tpu adjacent lanes (the
    // largest power of two with tpu * units <= NT, at most 64).
    for (int e = 0; e <= P + Q - 2; ++e) {
        const int jlo = e - (P - 1) > 0 ? e - (P - 1) : 0;
        const int jhi = e < Q - 1 ? e : Q - 1;
        const int nunits = jhi - jlo + 1;
        // lanes per unit: the largest power of two <= 64 with tpu * nunits <= NT
        // (at most 64 units: a tile has at most 64 block rows and columns)
        int tpu = 64, lg = 6;
        while (tpu > 1 && tpu * nunits > NT) { tpu >>= 1; --lg; }
        const int u = t >> lg, sub = t & (tpu - 1);
        T part[4] = {T(0), T(0), T(0), T(0)};
        int ri = 0, pi = 0, cj = 0, qj = 0;
        const bool active = u < nunits;
        if (active) {
            const int jb = jlo + u, ibb = e - jb;  // ibb from the bottom
            const int ib = P - 1 - ibb;
            ri = rstart[ib]; pi = rstart[ib + 1] - ri;
            cj = cstart[jb]; qj = cstart[jb + 1] - cj;
            // rows below the block: r' in [ri+pi, p) ; cols left: c' in [0, cj).
            // One loop for every block shape (an order-1 block masks its
            // second row or column), so units of different shapes sharing
            // a wavefront do not split it.
            // Both sums in one loop, k < nr the rows below (u = TA(ri.., r'),
            // w = Y(r', cj..)), then the columns to the left (u = Y(ri.., c'),
            // w = TB(c', cj..)): part += (u0 w0, u1 w0, u0 w1, u1 w1).  The
            // second row / column of an order-1 block is read at the first
            // one's index and masked, so the loads carry no condition.
            const T zp = (pi == 2) ? T(1) : T(0), zq = (qj == 2) ? T(1) : T(0);
            const int ri1 = ri + (pi == 2 ? 1 : 0), cj1 = cj + (qj == 2 ? 1 : 0);
            const int nr = p - ri - pi, ntot = nr + cj;
#pragma unroll 16
            for (int k = sub; k < ntot; k += tpu) {
                const bool rows = k < nr;
                const int x = rows ? ri + pi + k : k - nr;
                const T *Ub = rows ? sA : sC;
                const T *Wb = rows ? sC : sB;
                const T u0 = Ub[x * TLD + ri], u1 = Ub[x * TLD + ri1] * zp;
                const T w0 = Wb[cj * TLD + x], w1 = Wb[cj1 * TLD + x] * zq;
                part[0] += u0 * w0; part[1] += u1 * w0;
                part[2] += u0 * w1; part[3] += u1 * w1;
            }
        }
        const bool solver = active && sub == tpu - 1;
        // the solver's right-hand side and inverse rows (written by no other
        // unit) are loaded while the group sums run
        T rhs[4];
        t4 m0, m1, m2, m3;
        if (PRE) {
            const int ri1 = ri + (pi == 2 ? 1 : 0), cj1 = cj + (qj == 2 ? 1 : 0);
            const T zp = (pi == 2) ? T(1) : T(0), zq = (qj == 2) ? T(1) : T(0);
            rhs[0] = sC[cj * TLD + ri];
            rhs[1] = sC[cj * TLD + ri1] * zp;
            rhs[2] = sC[cj1 * TLD + ri] * zq;
            rhs[3] = sC[cj1 * TLD + ri1] * (zp * zq);
            m0 = sI[cj * TS + ri];
            m1 = sI[cj * TS + ri1];
            m2 = sI[cj1 * TS + ri];
            m3 = sI[cj1 * TS + ri1];
        }
        // the unit's sums land in its last lane, which solves the pair
        group_sum4<T>(part, tpu);
        if (PRE && solver) {
            // y = Minv r with the staged rows of the pair's unknowns
            const bool P2 = (pi == 2), Q2 = (qj == 2);
            T r[4];
#pragma unroll
            for (int z = 0; z < 4; ++z) r[z] = rhs[z] - part[z];
            sC[cj * TLD + ri] = m0[0] * r[0] + m0[1] * r[1] + m0[2] * r[2] + m0[3] * r[3];
            if (P2) sC[cj * TLD + ri + 1] = m1[0] * r[0] + m1[1] * r[1] + m1[2] * r[2] + m1[3] * r[3];
            if (Q2) sC[(cj + 1) * TLD + ri] = m2[0] * r[0] + m2[1] * r[1] + m2[2] * r[2] + m2[3] * r[3];
            if (P2 && Q2)
                sC[(cj + 1) * TLD + ri + 1] = m3[0] * r[0] + m3[1] * r[1] + m3[2] * r[2] + m3[3] * r[3];
        } else if (solver) {
            // every block pair through the 4 x 4 embedding (order-1 blocks
            // as identity rows): one code path for all shapes
            const bool P2 = (pi == 2), Q2 = (qj == 2);
            const T a00 = sA[ri * TLD + ri];
            const T a01 = P2 ? sA[(ri + 1) * TLD + ri] : T(0);
            const T a10 = P2 ? sA[ri * TLD + ri + 1] : T(0);
            const T a11 = P2 ? sA[(ri + 1) * TLD + ri + 1] : T(0);
            const T b00 = sB[cj * TLD + cj];
            const T b01 = Q2 ? sB[(cj + 1) * TLD + cj] : T(0);
            const T b10 = Q2 ? sB[cj * TLD + cj + 1] : T(0);
            const T b11 = Q2 ? sB[(cj + 1) * TLD + cj + 1] : T(0);
            // rhs entries (y00, y10, y01, y11) minus the accumulated sums
            T r[4];
            r[0] = sC[cj * TLD + ri] - part[0];
            r[1] = P2 ? sC[cj * TLD + ri + 1] - part[1] : T(0);
            r[2] = Q2 ? sC[(cj + 1) * TLD + ri] - part[2] : T(0);
            r[3] = (P2 && Q2) ? sC[(cj + 1) * TLD + ri + 1] - part[3] : T(0);
            myflag |= pair_solve<T>(P2, Q2, a00, a01, a10, a11, b00, b01, b10, b11, r, smin);
            sC[cj * TLD + ri] = r[0];
            if (P2) sC[cj * TLD + ri + 1] = r[1];
            if (Q2) sC[(cj + 1) * TLD + ri] = r[2];
            if (P2 && Q2) sC[(cj + 1) * TLD + ri + 1] = r[3];
        }
        __syncthreads();
    }
    for (int e = t; e < p * q; e += NT) {
        int i = e % p, j = e / p;
        C[(size_t)(c0 + j) * ldc + r0 + i] = sC[j * TLD + i];
    }
    if (wmirror)  // Y'(n-1-j, n-1-i) = Y'(i, j), consecutive threads down a column
        for (int e = t; e < p * q; e += NT) {
            int j = e % q, i = e / q;
            C[(size_t)(n - 1 - (r0 + i)) * ldc + (n - 1 - (c0 + j))] = sC[j * TLD + i];
        }
    if (myflag) atomicOr(flag, 1);
}

// mirror: symmetric Lyapunov (see trsyl_tile); the grid then covers only
// the tiles with 2J <= d
template <typename T, bool PRE, int NT>
__global__ __launch_bounds__(NT) void k_trsyl_diag(int m, int n, const T *__restrict__ TA, int ldta,
                                                   const T *__restrict__ TB, int ldtb, T *C, int ldc,
                                                   int d, int nI, int jmin, const double *maxab,
                                                   int *flag, int mirror, const T *__restrict__ Pinv,
                                                   const int *pflag) {
    const int J = jmin + blockIdx.x;
    const int I = nI - 1 - (d - J);
    trsyl_tile<T, NT, PRE>(m, n, TA, ldta, TB, ldtb, C, ldc, I, J, *maxab, flag, mirror,
                                 mirror && 2 * J < d, false, Pinv);
    // the pivots perturbed when the inverses were formed count for every solve
    if (PRE && d == 0 && threadIdx.x == 0 && *pflag) atomicOr(flag, 1);
}

// Inverse rows of every block pair (one workgroup per tile, the tile's own
// block partition as trsyl_tile scans it): for the pair at (ri, cj) of tile
// (I, J), row k of its inverse embedded matrix goes to the element of
// unknown k, Pinv[4 ((size_t) j m + i) + l].  *pflag = 1 when a pivot below
// s_min was replaced.
template <typename T>
__global__ __launch_bounds__(256) void k_trsyl_prep(int m, int n, const T *__restrict__ TA, int ldta,
                                                    const T *__restrict__ TB, int ldtb, const double *maxab,
                                                    int *pflag, T *Pinv, int mirror) {
    __shared__ int rstart[TS + 1], cstart[TS + 1];
    __shared__ int nrb_s, ncb_s;
    const int I = blockIdx.y, J = blockIdx.x;
    const int r0 = tile_bound(TA, ldta, m, I), r1 = tile_bound(TA, ldta, m, I + 1);
    int c0, c1;
    if (mirror) {
        const int nt = (m + TBASE - 1) / TBASE;
        c0 = n - tile_bound(TA, ldta, m, nt - J);
        c1 = n - tile_bound(TA, ldta, m, nt - 1 - J);
    } else {
        c0 = tile_bound(TB, ldtb, n, J);
        c1 = tile_bound(TB, ldtb, n, J + 1);
    }
    const int p = r1 - r0, q = c1 - c0;
    if (p <= 0 || q <= 0) return;
    if (threadIdx.x == 0) {
        int nb = 0, i = 0;
        while (i < p) { rstart[nb++] = i; i += (i + 1 < p && CM(TA, r0 + i + 1, r0 + i, ldta) != T(0)) ? 2 : 1; }
        rstart[nb] = p;
        nrb_s = nb;
        nb = 0; i = 0;
        while (i < q) { cstart[nb++] = i; i += (i + 1 < q && CM(TB, c0 + i + 1, c0 + i, ldtb) != T(0)) ? 2 : 1; }
        cstart[nb] = q;
        ncb_s = nb;
    }
    __syncthreads();
    const int P = nrb_s, Q = ncb_s;
    const T smin = (T)fmax((double)num<T>::ulp * *maxab, (double)num<T>::safmin);
    int myflag = 0;
    for (int u = threadIdx.x; u < P * Q; u += 256) {
        const int ib = u % P, jb = u / P;
        const int ri = r0 + rstart[ib], pi = rstart[ib + 1] - rstart[ib];
        const int cj = c0 + cstart[jb], qj = cstart[jb + 1] - cstart[jb];
        const bool P2 = pi == 2, Q2 = qj == 2;
        const T a00 = CM(TA, ri, ri, ldta);
        const T a01 = P2 ? CM(TA, ri, ri + 1, ldta) : T(0);
        const T a10 = P2 ? CM(TA, ri + 1, ri, ldta) : T(0);
        const T a11 = P2 ? CM(TA, ri + 1, ri + 1, ldta) : T(0);
        const T b00 = CM(TB, cj, cj, ldtb);
        const T b01 = Q2 ? CM(TB, cj, cj + 1, ldtb) : T(0);
        const T b10 = Q2 ? CM(TB, cj + 1, cj, ldtb) : T(0);
        const T b11 = Q2 ? CM(TB, cj + 1, cj + 1, ldtb) : T(0);
        T Mi[4][4];
        myflag |= pair_inverse<T>(P2, Q2, a00, a01, a10, a11, b00, b01, b10, b11, Mi, smin);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool valid = (k == 0) || (k == 1 && P2) || (k == 2 && Q2) || (k == 3 && P2 && Q2);
            if (valid) {
                T *dst = Pinv + 4 * ((size_t)(cj + (k >> 1)) * m + ri + (k & 1));
#pragma unroll
                for (int l = 0; l < 4; ++l) dst[l] = Mi[k][l];
            }
        }
    }
    if (myflag) atomicOr(pflag, 1);
}

// Right-looking updates after anti-diagonal d is solved: every tile (I, J)
// of a later anti-diagonal loses the contributions of the solved tile of its
// block column, (K, J) with K = nI-1-d+J (through TA(I, K)), and of the
// solved tile of its block row, (I, L) with L = d-(nI-1-I) (through TB(L, J)):
//   C_IJ -= TA(I, K) Y(K, J) + Y(I, L) TB(L, J).
// Every pair (destination, source) is met exactly once over the sweep, so
// C_IJ holds the full right-hand side when its own anti-diagonal comes up.
// One workgroup per tile (grid nJ x nI); tiles without a source exit at
// once.  mirror: tiles with 2J > their anti-diagonal are never solved
// directly (their mirror images are written instead) and need no update.
template <typename T>
__global__ __launch_bounds__(256) void k_trsyl_update(int m, int n, const T *__restrict__ TA, int ldta,
                                                     const T *__restrict__ TB, int ldtb, T *C, int ldc, int d,
                                                     int nI, int nJ, int mirror) {
    __shared__ T stA[TBK][TS + 16];
    __shared__ T stB[TBK][TS + 16];
    typedef typename mfma16t<T>::v4 v4;
    const int J = blockIdx.x, I = blockIdx.y;
    const int dIJ = nI - 1 - I + J;
    if (dIJ <= d) return;
    if (mirror && 2 * J > dIJ) return;
    const int K = nI - 1 - d + J, L = d - (nI - 1 - I);
    const bool hasK = K < nI, hasL = L >= 0;   // K > I and L < J hold since dIJ > d
    if (!hasK && !hasL) return;
    auto rb_ = [&](int k) { return tile_bound(TA, ldta, m, k); };
    auto cb_ = [&](int k) {
        return mirror ? n - tile_bound(TA, ldta, m, nI - k) : tile_bound(TB, ldtb, n, k);
    };
    const int r0 = rb_(I), r1 = rb_(I + 1), c0 = cb_(J), c1 = cb_(J + 1);
    const int p = r1 - r0, q = c1 - c0;
    if (p <= 0 || q <= 0) return;
    v4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = v4{0, 0, 0, 0};
    if (hasK) {
        const int k0 = rb_(K), k1 = rb_(K + 1);
        tile_gemm<T>(acc, TA + (size_t)k0 * ldta + r0, ldta, C + (size_t)c0 * ldc + k0, ldc, k1 - k0, p, q, stA, stB);
    }
    if (hasL) {
        const int l0 = cb_(L), l1 = cb_(L + 1);
        tile_gemm<T>(acc, C + (size_t)l0 * ldc + r0, ldc, TB + (size_t)c0 * ldtb + l0, ldtb, l1 - l0, p, q, stA, stB);
    }
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int wm = w & 1, wn = w >> 1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 32 * wm + 16 * a + (l & 15);
                const int j = 32 * wn + 16 * b + mfma16t<T>::orow(l, r);
                if (i < p && j < q) C[(size_t)(c0 + j) * ldc + r0 + i] -= acc[a][b][r];
            }
}

// Batched form: tiles of anti-diagonal d of every active equation
// (grid.x = tile within the anti-diagonal, grid.y = equation slot).
// TA = T (field H), TB = the upper quasi-triangular right coefficient
// (field TB), Y overwrites field W.
__global__ __launch_bounds__(256) void k_btrsyl_diag(BatchEq *eqs, const int *order, int d) {
    BatchEq &q = eqs[order[blockIdx.y]];
    if (!q.active) return;
    const int n = q.n;
    const int nI = (n + TBASE - 1) / TBASE;
    if (d > 2 * nI - 2) return;
    const int jmin = d - (nI - 1) > 0 ? d - (nI - 1) : 0;
    const int jmax = d < nI - 1 ? d : nI - 1;
    const int J = jmin + (int)blockIdx.x;
    if (J > jmax) return;
    // symmetric equations: one tile of each mirror pair (2J < d) also
    // stores its mirror; the self-mirror tile (2J = d) is solved whole
    if (q.sym && 2 * J > d) return;
    const int I = nI - 1 - (d - J);
    trsyl_tile<float>(n, n, (const float *)q.ptr[BF_H], q.ld[BF_H], (const float *)q.ptr[BF_TB],
                      q.ld[BF_TB], (float *)q.ptr[BF_W], q.ld[BF_W], I, J, q.tmax, &q.flag, q.sym,
                      q.sym && 2 * J < d);
}

void trsyl_batched(hipStream_t s, BatchEq *eqs, const int *order, int batch, int nmax) {
    if (batch <= 0 || nmax <= 0) return;
    const int nI = (nmax + TBASE - 1) / TBASE;
    for (int d = 0; d <= 2 * nI - 2; ++d) {
        const int tiles = (d < nI ? d + 1 : 2 * nI - 1 - d);
        ProfScope ps(KID_BTRSYL, s);
        hipLaunchKernelGGL(k_btrsyl_diag, dim3(tiles, batch), dim3(256), 0, s, eqs, order, d);
    }
}

template <typename T>
void trsyl_prep(hipStream_t s, int m, int n, const T *TA, int ldta, const T *TB, int ldtb, const double *maxab,
                int *pflag, T *Pinv, int mirror) {
    if (m <= 0 || n <= 0) return;
    if (m != n) mirror = 0;
    const int nI = (m + TBASE - 1) / TBASE, nJ = (n + TBASE - 1) / TBASE;
    hipMemsetAsync(pflag, 0, sizeof(int), s);
    hipLaunchKernelGGL((k_trsyl_prep<T>), dim3(nJ, nI), dim3(256), 0, s, m, n, TA, ldta, TB, ldtb, maxab, pflag,
                       Pinv, mirror);
}
template void trsyl_prep<float>(hipStream_t, int, int, const float *, int, const float *, int, const double *,
                                int *, float *, int);

template <typename T>
void trsyl(hipStream_t s, int m, int n, const T *TA, int ldta, const T *TB, int ldtb, T *C, int ldc,
           const double *maxab, int *flag, int mirror, const T *Pinv, const int *pflag) {
    if (m <= 0 || n <= 0) return;
    if (m != n) mirror = 0;
    const int nI = (m + TBASE - 1) / TBASE, nJ = (n + TBASE - 1) / TBASE;
    for (int d = 0; d <= nI + nJ - 2; ++d) {
        int jmin = d - (nI - 1) > 0 ? d - (nI - 1) : 0;
        int jmax = d < nJ - 1 ? d : nJ - 1;
        if (mirror && jmax > d / 2) jmax = d / 2;
        ProfScope ps(KID_TRSYL, s);
        bool pre = false;
        if constexpr (sizeof(T) == 4) {   // the staged inverse rows fit LDS in binary32 only
            if (Pinv && pflag) {
                hipLaunchKernelGGL((k_trsyl_diag<T, true, TRSYL_NT_PRE>), dim3(jmax - jmin + 1), dim3(TRSYL_NT_PRE),
                                   0, s, m, n, TA, ldta, TB, ldtb, C, ldc, d, nI, jmin, maxab, flag, mirror, Pinv,
                                   pflag);
                pre = true;
            }
        }
        if (!pre)
            hipLaunchKernelGGL((k_trsyl_diag<T, false, TRSYL_NT>), dim3(jmax - jmin + 1), dim3(TRSYL_NT), 0, s, m, n, TA,
                               ldta, TB, ldtb, C, ldc, d, nI, jmin, maxab, flag, mirror, Pinv, pflag);
        if (d < nI + nJ - 2)
            hipLaunchKernelGGL((k_trsyl_update<T>), dim3(nJ, nI), dim3(256), 0, s, m, n, TA, ldta, TB, ldtb, C,
                               ldc, d, nI, nJ, mirror);
    }
}
template void trsyl<float>(hipStream_t, int, int, const float *, int, const float *, int, float *, int,
                           const double *, int *, int, const float *, const int *);
template void trsyl<double>(hipStream_t, int, int, const double *, int, const double *, int, double *,
                            int, const double *, int *, int, const double *, const int *);

}  // namespace sylv
