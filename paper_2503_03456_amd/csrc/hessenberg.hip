// Blocked Householder reduction to upper Hessenberg form, H = U0^T A U0
// (the first phase of the QR algorithm, Golub & Van Loan Sec. 7.4.3, in the
// blocked form where a panel of nb reflectors Q = I - V T V^T is applied to
// the trailing matrix as A <- Q^T (A - Y V^T), Y = A V T).
//
// Per panel column (one pair of launches):
//   k_hess_col  (one workgroup): finish y and T of the previous column,
//               bring the current column up to date with the panel's earlier
//               reflectors (right: -Y V(col,:)^T; left: -V T^T V^T a), and
//               generate its Householder vector.  For n <= 4096 the
//               register-resident k_hess_col_r does the same with the column
//               held in registers and latency-oriented loads and reductions.
//   k_hess_gemv (many workgroups): y_raw = A(:, col+1:n) v over row blocks x
//               column slices; partial sums are combined in a fixed order by
//               the next k_hess_col (deterministic).
// After the panel: trailing update with MFMA GEMMs.  U0 is formed at the end
// by applying the stored block reflectors backwards to the identity.
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace sylv {

constexpr int HNT = 1024;
constexpr int HKS = 16;   // most contraction slices of a split panel product (k_hess_tsum holds 16)

template <typename T>
SYLV_DEVINL T block_sum(T v, T *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    T s = T(0);
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// Reduce cnt (<= 32) per-thread accumulators over the workgroup in one pass:
// wave shuffles, one LDS round, fixed summation order.  out[j] for j < cnt.
template <typename T>
SYLV_DEVINL void multi_sum(int cnt, T acc[32], T *red /* 16 x 32 */, T *out) {
    const int tid = threadIdx.x, w = tid >> 6;
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        if (j < cnt) {
            T v = acc[j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            acc[j] = v;
        }
    }
    if ((tid & 63) == 0) {
#pragma unroll
        for (int j = 0; j < 32; ++j)
            if (j < cnt) red[w * 32 + j] = acc[j];
    }
    __syncthreads();
    if (tid < cnt) {
        T sum = T(0);
        for (int q = 0; q < HNT / 64; ++q) sum += red[q * 32 + tid];
        out[tid] = sum;
    }
    __syncthreads();
}

// State: A (n x n, lda), V (n x n, ldv = n) reflector vectors (column c holds
// the vector of column c's reflector, 1 at row c+1, zeros above), Tp (nb x nb,
// ld nb) the panel's T, Y (n x nb, ld n), Ypart (S x n) partials of y_raw for
// column `col-1`, tau (n).
template <typename T>
__global__ __launch_bounds__(HNT) void k_hess_col(int n, T *A, int lda, T *V, T *Tp, int nb, T *Y,
                                                 const T *Ypart, int S, T *tau, int k0, int i,
                                                 int finalize_only) {
    __shared__ T red[HNT / 64];
    __shared__ T red2[(HNT / 64) * 32];
    __shared__ T wv[64];
    __shared__ T cv[64];
    __shared__ T sh[4];
    const int tid = threadIdx.x;
    const int ldv = n;
    if (i > 0) {
        // finish column i-1: w = V(:,k0:k0+i-1)^T v_{i-1}; T(0:i-1, i-1); y_{i-1}
        const int cp = k0 + i - 1;
        const T tp = tau[cp];
        {
            T acc[32];
#pragma unroll
            for (int j = 0; j < 32; ++j) acc[j] = T(0);
            for (int r = cp + 1 + tid; r < n; r += HNT) {
                const T vc = CM(V, r, cp, ldv);
#pragma unroll
                for (int j = 0; j < 32; ++j)
                    if (j < i - 1) acc[j] += CM(V, r, k0 + j, ldv) * vc;
            }
            multi_sum(i - 1, acc, red2, wv);
        }
        if (tid < i - 1) {
            // T(0:i-1, i-1) = -tau T(0:i-1,0:i-1) w   (T upper triangular)
            T acc = T(0);
#pragma unroll 8
            for (int j = tid; j < i - 1; ++j) acc += Tp[j * nb + tid] * wv[j];
            cv[tid] = -tp * acc;
        }
        __syncthreads();
        if (tid < i - 1) Tp[(i - 1) * nb + tid] = cv[tid];
        if (tid == 0) Tp[(i - 1) * nb + (i - 1)] = tp;
        // the loops below have run-time trip counts; unrolling lets their
        // independent loads overlap (the summation order is unchanged)
        for (int r = tid; r < n; r += HNT) {
            T yr = T(0);
#pragma unroll 8
            for (int s = 0; s < S; ++s) yr += Ypart[(size_t)s * n + r];
            T acc = T(0);
#pragma unroll 8
            for (int j = 0; j < i - 1; ++j) acc += CM(Y, r, j, n) * wv[j];
            CM(Y, r, i - 1, n) = tp * (yr - acc);
        }
        __syncthreads();
    }
    if (finalize_only) return;
    const int col = k0 + i;
    // right update of the current column by the panel's earlier reflectors:
    // a(r) -= sum_j Y(r, j) V(col, k0+j)
    for (int j = tid; j < i; j += HNT) cv[j] = CM(V, col, k0 + j, ldv);
    __syncthreads();
    for (int r = tid; r < n; r += HNT) {
        T acc = T(0);
#pragma unroll 8
        for (int j = 0; j < i; ++j) acc += CM(Y, r, j, n) * cv[j];
        CM(A, r, col, lda) -= acc;
    }
    __syncthreads();
    // left update on rows k0+1..n-1: a -= V T^T (V^T a)
    if (i > 0) {
        {
            T acc[32];
#pragma unroll
            for (int j = 0; j < 32; ++j) acc[j] = T(0);
            for (int r = k0 + 1 + tid; r < n; r += HNT) {
                const T ar = CM(A, r, col, lda);
#pragma unroll
                for (int j = 0; j < 32; ++j)
                    if (j < i) acc[j] += CM(V, r, k0 + j, ldv) * ar;
            }
            multi_sum(i, acc, red2, wv);
        }
        if (tid < i) {
            // c = T^T b: c(j) = sum_{j' <= j} T(j', j) b(j')
            T acc = T(0);
#pragma unroll 8
            for (int jp = 0; jp <= tid; ++jp) acc += Tp[tid * nb + jp] * wv[jp];
            cv[tid] = acc;
        }
        __syncthreads();
        for (int r = k0 + 1 + tid; r < n; r += HNT) {
            T acc = T(0);
#pragma unroll 8
            for (int j = 0; j < i; ++j) acc += CM(V, r, k0 + j, ldv) * cv[j];
            CM(A, r, col, lda) -= acc;
        }
        __syncthreads();
    }
    // Householder vector for a(col+1:n): zeros below col+1
    const int len = n - col - 1;
    T mx = T(0);
    for (int r = col + 2 + tid; r < n; r += HNT) mx = fmax(mx, fabs(CM(A, r, col, lda)));
    // block max
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    mx = T(0);
    for (int w = 0; w < HNT / 64; ++w) mx = fmax(mx, red[w]);
    T ss = T(0);
    if (mx > T(0))
        for (int r = col + 2 + tid; r < n; r += HNT) {
            T q = CM(A, r, col, lda) / mx;
            ss += q * q;
        }
    ss = block_sum(ss, red);
    if (tid == 0) {
        T alpha = CM(A, col + 1, col, lda);
        if (mx == T(0) || len < 2) {
            sh[0] = T(0); sh[1] = alpha; sh[2] = T(0);
        } else {
            T xn = mx * sqrt(ss);
            T nrm = hypot(alpha, xn);
            T b = (alpha >= T(0)) ? -nrm : nrm;
            sh[0] = (b - alpha) / b;
            sh[1] = b;
            sh[2] = T(1) / (alpha - b);
        }
    }
    __syncthreads();
    const T tc = sh[0], beta = sh[1], sc = sh[2];
    for (int r = tid; r < n; r += HNT) {
        T v;
        if (r <= col) v = T(0);
        else if (r == col + 1) v = T(1);
        else v = CM(A, r, col, lda) * sc;
        CM(V, r, col, ldv) = v;
    }
    __syncthreads();
    for (int r = col + 1 + tid; r < n; r += HNT) CM(A, r, col, lda) = (r == col + 1) ? beta : T(0);
    if (tid == 0) tau[col] = tc;
}

// ------------------------------------------------- register-resident variant
// The same per-column step for n <= NQ * HNT with the column held in
// registers (each thread owns rows tid + q HNT, q < NQ), arranged for
// latency: every loop issues its loads unconditionally (clamped indices,
// masked values) so they overlap, the two panel reductions run one
// wavefront per (column, row part) with a single shuffle tree each, y and the
// right update share one pass over Y, and the column is read from and written
// to global memory once.  Requires nb <= 32.

template <typename T>
SYLV_DEVINL T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// out[j] = sum_{r in [r0, n)} V(r, k0 + j) xs[r] for j < cnt (cnt <= 32),
// xs in LDS indexed by row.  Work unit = (column, part of the rows): with cnt
// columns over NWV wavefronts each column's rows split into P = NWV / cnt
// parts (P = 1 once cnt >= NWV); parts combine in a fixed order.
template <typename T>
SYLV_DEVINL void panel_dots(int n, int r0, const T *V, int ldv, int k0, int cnt, const T *xs, T *part,
                            T *out) {
    constexpr int NWV = HNT / 64;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int P = cnt >= NWV ? 1 : NWV / (cnt > 0 ? cnt : 1);
    if (cnt > 0) {
        const int rows = n - r0;
        const int chunk = ((rows + P - 1) / P + 63) & ~63;
        for (int u = w; u < cnt * P; u += NWV) {
            const int j = u / P, p = u - j * P;
            const int lo = r0 + p * chunk;
            const int hi = (lo + chunk < n) ? lo + chunk : n;
            const T *vc = V + (size_t)(k0 + j) * ldv;
            T acc = T(0);
#pragma unroll 8
            for (int r = lo + lane; r < hi; r += 64) acc += vc[r] * xs[r];
            acc = wave_sum(acc);
            if (lane == 0) part[j * NWV + p] = acc;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
        T sum = T(0);
        for (int p = 0; p < P; ++p) sum += part[threadIdx.x * NWV + p];
        out[threadIdx.x] = sum;
    }
    __syncthreads();
}

template <typename T, int NQ>
__global__ __launch_bounds__(HNT) void k_hess_col_r(int n, T *A, int lda, T *V, T *Tp, int nb, T *Y,
                                                   const T *Ypart, int S, T *tau, int k0, int i,
                                                   int finalize_only, const T *wT) {
    constexpr int NWV = HNT / 64;
    __shared__ T xs[NQ * HNT];
    __shared__ T tps[32 * 32];  // panel T, column c at tps[32 c]
    __shared__ T part[32 * NWV];
    __shared__ T wv[32], cm[32], cc[32], bv[32];
    __shared__ T red[NWV];
    __shared__ T sh[4];
    const int tid = threadIdx.x;
    const int ldv = n;
    const int col = k0 + i;
    const bool upd = !finalize_only;
    // stage: finished columns of T, the row V(col, k0:k0+i) (right update
    // coefficients, zero beyond), and for i > 0 the products
    // w = V(:, k0:k0+i-1)^T v_{i-1} that the previous column's GEMV launch
    // formed beside its product (wT)
    for (int e = tid; e < 32 * 32; e += HNT) {
        const int c = e >> 5, r = e & 31;
        tps[e] = (c < i - 1 && r < nb) ? Tp[c * nb + r] : T(0);
    }
    if (tid < 32) cm[tid] = (upd && tid < i) ? CM(V, col, k0 + tid, ldv) : T(0);
    if (tid < 32) wv[tid] = (tid < i - 1) ? wT[tid] : T(0);
    const int cp = k0 + i - 1;
    __syncthreads();
    T yfix = T(0);
    if (i > 0) {
        // T(0:i-1, i-1) = -tau T(0:i-1, 0:i-1) w
        const T tp = tau[cp];
        if (tid < 32) {
            T acc = T(0);
            for (int j = tid; j < i - 1; ++j) acc += tps[j * 32 + tid] * wv[j];
            const T v = (tid < i - 1) ? -tp * acc : (tid == i - 1 ? tp : T(0));
            if (tid < i) {
                tps[(i - 1) * 32 + tid] = v;
                Tp[(i - 1) * nb + tid] = v;
            }
            if (tid >= i - 1) wv[tid] = T(0);  // mask for the Y pass
        }
        __syncthreads();
        yfix = tp;
    }
    // one pass over Y: y_{i-1}(r) = tau (sum_s Ypart(s, r) - Y(r, 0:i-1) w) and
    // the right update a(r) -= Y(r, 0:i) V(col, k0:k0+i)^T
    T a[NQ];
    int rr[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        rr[q] = tid + q * HNT;
        a[q] = (upd && rr[q] < n) ? CM(A, rr[q], col, lda) : T(0);
    }
    if (i > 0) {
        T yr[NQ], s1[NQ], s2[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) { yr[q] = T(0); s1[q] = T(0); s2[q] = T(0); }
        for (int sb = 0; sb < S; sb += 8) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int sc = (sb + t < S) ? sb + t : S - 1;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int r = rr[q] < n ? rr[q] : n - 1;
                    const T v = Ypart[(size_t)sc * n + r];
                    yr[q] += (sb + t < S) ? v : T(0);
                }
            }
        }
        const int jm = i >= 2 ? i - 2 : 0;
        for (int jb = 0; jb < i - 1; jb += 8) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int j = jb + t;
                const int jc = j < jm ? j : jm;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int r = rr[q] < n ? rr[q] : n - 1;
                    T yv = CM(Y, r, jc, n);
                    yv = (j < i - 1) ? yv : T(0);
                    s1[q] += yv * wv[j & 31];
                    s2[q] += yv * cm[j & 31];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (rr[q] < n) {
                const T y = yfix * (yr[q] - s1[q]);
                CM(Y, rr[q], i - 1, n) = y;
                a[q] -= s2[q] + y * cm[i - 1];
            }
        }
    }
    if (finalize_only) return;
    // left update on rows k0+1..n-1: a -= V T^T (V^T a)
    if (i > 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (rr[q] < n) xs[rr[q]] = a[q];
        __syncthreads();
        panel_dots(n, k0 + 1, V, ldv, k0, i, xs, part, bv);
        if (tid < 32) {
            // c = T^T b: c(t) = sum_{j <= t} T(j, t) b(j)
            T acc = T(0);
            if (tid < i)
                for (int jp = 0; jp <= tid; ++jp) acc += tps[tid * 32 + jp] * bv[jp];
            cc[tid] = acc;
        }
        __syncthreads();
        T s3[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) s3[q] = T(0);
        const int jm = i - 1;
        for (int jb = 0; jb < i; jb += 8) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int j = jb + t;
                const int jc = j < jm ? j : jm;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int r = rr[q] < n ? rr[q] : n - 1;
                    T vv = CM(V, r, k0 + jc, ldv);
                    vv = (j < i) ? vv : T(0);
                    s3[q] += vv * cc[j & 31];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (rr[q] >= k0 + 1 && rr[q] < n) a[q] -= s3[q];
    }
    // Householder vector for a(col+1:n): zeros below col+1
    const int len = n - col - 1;
    T mx = T(0);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (rr[q] >= col + 2 && rr[q] < n) mx = fmax(mx, fabs(a[q]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if ((tid & 63) == 0) red[tid >> 6] = mx;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (rr[q] == col + 1) sh[3] = a[q];
    __syncthreads();
    mx = T(0);
    for (int w = 0; w < NWV; ++w) mx = fmax(mx, red[w]);
    T ss = T(0);
    if (mx > T(0)) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (rr[q] >= col + 2 && rr[q] < n) {
                const T z = a[q] / mx;
                ss += z * z;
            }
    }
    ss = block_sum(ss, red);
    if (tid == 0) {
        const T alpha = sh[3];
        if (mx == T(0) || len < 2) {
            sh[0] = T(0); sh[1] = alpha; sh[2] = T(0);
        } else {
            const T xn = mx * sqrt(ss);
            const T nrm = hypot(alpha, xn);
            const T b = (alpha >= T(0)) ? -nrm : nrm;
            sh[0] = (b - alpha) / b;
            sh[1] = b;
            sh[2] = T(1) / (alpha - b);
        }
    }
    __syncthreads();
    const T tc = sh[0], beta = sh[1], scl = sh[2];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int r = rr[q];
        if (r < n) {
            CM(V, r, col, ldv) = (r <= col) ? T(0) : (r == col + 1 ? T(1) : a[q] * scl);
            CM(A, r, col, lda) = (r <= col) ? a[q] : (r == col + 1 ? beta : T(0));
        }
    }
    if (tid == 0) tau[col] = tc;
}

// Ypart[s][r] = sum_{c in slice s} A(r, c) v(c), c in [col+1, n).  The
// workgroups of row block gridDim.x - 1 instead form the next column step's
// panel products wT[j] = sum_{r > col} V(r, k0 + j) v(r), j < col - k0 (one
// wavefront each), so that step starts from them.
template <typename T>
__global__ __launch_bounds__(256) void k_hess_gemv(int n, const T *A, int lda, const T *V, int col,
                                                  T *Ypart, int S, int k0, T *wT) {
    if ((int)blockIdx.x == (int)gridDim.x - 1) {
        const int j = blockIdx.y * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
        if (j >= col - k0) return;
        const T *vj = V + (size_t)(k0 + j) * n, *vc = V + (size_t)col * n;
        T acc = T(0);
#pragma unroll 8
        for (int r = col + 1 + lane; r < n; r += 64) acc += vj[r] * vc[r];
        acc = wave_sum(acc);
        if (lane == 0) wT[j] = acc;
        return;
    }
    __shared__ T vs[512];
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    const int c0 = col + 1, nc = n - c0;
    const int per = (nc + S - 1) / S;
    const int cb = c0 + s * per;
    int ce = cb + per;
    if (ce > n) ce = n;
    const int ldv = n;
    T acc = T(0);
    for (int base = cb; base < ce; base += 512) {
        int cnt = ce - base < 512 ? ce - base : 512;
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += 256) vs[q] = CM(V, base + q, col, ldv);
        __syncthreads();
        if (r < n)
#pragma unroll 8
            for (int q = 0; q < cnt; ++q) acc += CM(A, r, base + q, lda) * vs[q];
    }
    if (r < n) Ypart[(size_t)s * n + r] = acc;
}

// W2 = op(T) * sum_{z < nz} P_z for a panel: P_z (nbp x nt, ld nbp) are the
// split-K slices of V^T M, T (nbp x nbp, ld ldt) the panel's triangular
// factor, op(T) = T^T when trans.  One workgroup per 8 columns, one thread
// per entry: its nz slice values are loaded together and summed in slice
// order into LDS, then each thread forms its entry of op(T) S.
template <typename T>
__global__ __launch_bounds__(256) void k_hess_tsum(int nbp, int nt, int nz, const T *__restrict__ P,
                                                  const T *__restrict__ Tp, int ldt, int trans, T *__restrict__ W2) {
    __shared__ T S[8][33];
    __shared__ T Ts[32][33];
    const int tid = threadIdx.x, i = tid & 31, jj = tid >> 5, j = blockIdx.x * 8 + jj;
    for (int e = tid; e < 32 * 32; e += 256) {
        const int r = e & 31, l = e >> 5;
        T v = T(0);
        if (r < nbp && l < nbp) v = trans ? Tp[(size_t)r * ldt + l] : Tp[(size_t)l * ldt + r];
        Ts[r][l] = v;
    }
    const size_t slice = (size_t)nbp * nt;
    const bool in = i < nbp && j < nt;
    // clamped address, masked value: every load is issued unconditionally
    const T *p = P + (size_t)(j < nt ? j : nt - 1) * nbp + (i < nbp ? i : nbp - 1);
    T v[16];
#pragma unroll
    for (int z = 0; z < 16; ++z) v[z] = p[(z < nz ? z : nz - 1) * slice];
    T sum = T(0);
#pragma unroll
    for (int z = 0; z < 16; ++z)
        if (z < nz) sum += v[z];
    S[jj][i] = in ? sum : T(0);
    __syncthreads();
    if (in) {
        T acc = T(0);
        for (int l = 0; l < nbp; ++l) acc += Ts[i][l] * S[jj][l];
        W2[(size_t)j * nbp + i] = acc;
    }
}

// W2 (nbp x nt) = op(T) (V^T M): V the panel's reflectors (mr x nbp, ld ldv),
// M (mr x nt, ld ldm).  The contraction over mr runs split over the chip
// (the output has only nt / 64 tiles); with BF16 inputs the plain GEMMs.
template <typename T>
static void panel_vtm(hipStream_t s, int nbp, int nt, int mr, const T *Vp, int ldv, const T *M, int ldm,
                      const T *Tp, int ldt, int trans, T *W, T *W2, T *Pk, int bf16) {
    const int tiles = (nt + 63) / 64;
    if (!bf16 && nbp <= 32 && tiles < 128) {
        const int ks = std::min(HKS, std::max(1, 512 / tiles));
        const int nz = gemm_splitk<T>(s, 1, 0, nbp, nt, mr, Vp, ldv, M, ldm, Pk, ks);
        hipLaunchKernelGGL((k_hess_tsum<T>), dim3((nt + 7) / 8), dim3(256), 0, s, nbp, nt, nz, Pk, Tp, ldt, trans,
                           W2);
        return;
    }
    gemm<T, T, T, T>(s, 1, 0, nbp, nt, mr, T(1), Vp, ldv, M, ldm, T(0), W, nbp, T(1), bf16);
    gemm<T, T, T, T>(s, trans, 0, nbp, nt, nbp, T(1), Tp, ldt, W, nbp, T(0), W2, nbp);
}

template <typename T>
size_t hessenberg_work_elems(int n, int nb, int S) {
    int np = (n + nb - 1) / nb;
    return (size_t)n * n              // V
           + (size_t)np * nb * nb     // T per panel
           + (size_t)n * nb           // Y
           + (size_t)S * n            // Ypart
           + (size_t)n                // tau
           + (size_t)2 * nb * n       // W, W2 for the trailing update
           + (size_t)HKS * nb * n     // split-K partial products of V^T M
           + 64;                      // wT: the next column step's panel products
}
template size_t hessenberg_work_elems<float>(int, int, int);
template size_t hessenberg_work_elems<double>(int, int, int);

// One column step: the register-resident kernel while the column fits
// (n <= 4 HNT, nb <= 32), else the general one.
template <typename T>
static void hess_col(hipStream_t s, int n, T *A, int lda, T *V, T *Tp, int nb, T *Y, const T *Ypart, int S,
                     T *tau, int k0, int i, int fin, const T *wT) {
    if (nb <= 32 && n <= HNT)
        hipLaunchKernelGGL((k_hess_col_r<T, 1>), dim3(1), dim3(HNT), 0, s, n, A, lda, V, Tp, nb, Y, Ypart, S,
                           tau, k0, i, fin, wT);
    else if (nb <= 32 && n <= 2 * HNT)
        hipLaunchKernelGGL((k_hess_col_r<T, 2>), dim3(1), dim3(HNT), 0, s, n, A, lda, V, Tp, nb, Y, Ypart, S,
                           tau, k0, i, fin, wT);
    else if (nb <= 32 && n <= 4 * HNT)
        hipLaunchKernelGGL((k_hess_col_r<T, 4>), dim3(1), dim3(HNT), 0, s, n, A, lda, V, Tp, nb, Y, Ypart, S,
                           tau, k0, i, fin, wT);
    else
        hipLaunchKernelGGL((k_hess_col<T>), dim3(1), dim3(HNT), 0, s, n, A, lda, V, Tp, nb, Y, Ypart, S, tau,
                           k0, i, fin);
}

// A (n x n) -> H in place; U (n x n) receives U0.  work: hessenberg_work_elems.
template <typename T>
void hessenberg(hipStream_t s, int n, T *A, int lda, T *U, int ldu, T *work, int nb, int S, int bf16) {
    if (n <= 0) return;
    identity<T>(s, n, U, ldu);
    if (n <= 2) return;
    const int np = (n - 2 + nb - 1) / nb;  // panels covering columns 0..n-3
    T *V = work;
    T *Tall = V + (size_t)n * n;
    T *Y = Tall + (size_t)((n + nb - 1) / nb) * nb * nb;
    T *Ypart = Y + (size_t)n * nb;
    T *tau = Ypart + (size_t)S * n;
    T *W = tau + n;
    T *W2 = W + (size_t)nb * n;
    T *Pk = W2 + (size_t)nb * n;
    T *wT = Pk + (size_t)HKS * nb * n;
    hipMemsetAsync(V, 0, sizeof(T) * (size_t)n * n, s);
    hipMemsetAsync(Tall, 0, sizeof(T) * (size_t)((n + nb - 1) / nb) * nb * nb, s);
    const int rb = (n + 255) / 256;
    for (int p = 0; p < np; ++p) {
        const int k0 = p * nb;
        const int nbp = (n - 2 - k0) < nb ? (n - 2 - k0) : nb;
        T *Tp = Tall + (size_t)p * nb * nb;
        for (int i = 0; i < nbp; ++i) {
            {
                ProfScope ps(KID_HESS_COL, s);
                hess_col<T>(s, n, A, lda, V, Tp, nb, Y, Ypart, S, tau, k0, i, 0, wT);
            }
            {
                ProfScope ps(KID_HESS_GEMV, s);
                hipLaunchKernelGGL((k_hess_gemv<T>), dim3(rb + 1, S), dim3(256), 0, s, n, A, lda, V, k0 + i,
                                   Ypart, S, k0, wT);
            }
        }
        hess_col<T>(s, n, A, lda, V, Tp, nb, Y, Ypart, S, tau, k0, nbp, 1, wT);
        const int c1 = k0 + nbp;  // first trailing column
        const int nt = n - c1;
        if (nt > 0) {
            // right: A(:, c1:n) -= Y V(c1:n, k0:k0+nbp)^T
            gemm<T, T, T, T>(s, 0, 1, n, nt, nbp, T(-1), Y, n, V + (size_t)k0 * n + c1, n, T(1),
                             A + (size_t)c1 * lda, lda, T(1), bf16);
            // left: A(k0+1:n, c1:n) -= V T^T (V^T A(k0+1:n, c1:n))
            const int mr = n - k0 - 1;
            panel_vtm<T>(s, nbp, nt, mr, V + (size_t)k0 * n + k0 + 1, n, A + (size_t)c1 * lda + k0 + 1, lda,
                         Tp, nb, 1, W, W2, Pk, bf16);
            gemm<T, T, T, T>(s, 0, 0, mr, nt, nbp, T(-1), V + (size_t)k0 * n + k0 + 1, n, W2, nbp,
                             T(1), A + (size_t)c1 * lda + k0 + 1, lda, T(1), bf16);
        }
    }
    // U0 = Q_0 Q_1 ... : apply the block reflectors backwards to the identity
    for (int p = np - 1; p >= 0; --p) {
        const int k0 = p * nb;
        const int nbp = (n - 2 - k0) < nb ? (n - 2 - k0) : nb;
        T *Tp = Tall + (size_t)p * nb * nb;
        const int mr = n - k0 - 1;
        T *Us = U + (size_t)(k0 + 1) * ldu + k0 + 1;
        panel_vtm<T>(s, nbp, mr, mr, V + (size_t)k0 * n + k0 + 1, n, Us, ldu, Tp, nb, 0, W, W2, Pk, bf16);
        gemm<T, T, T, T>(s, 0, 0, mr, mr, nbp, T(-1), V + (size_t)k0 * n + k0 + 1, n, W2, nbp, T(1),
                         Us, ldu, T(1), bf16);
    }
}
template void hessenberg<float>(hipStream_t, int, float *, int, float *, int, float *, int, int, int);
template void hessenberg<double>(hipStream_t, int, double *, int, double *, int, double *, int, int, int);

}  // namespace sylv
