// Symmetric eigen-decomposition S = Q diag(d) Q^T for the symmetric-
// coefficient variant of Bartels-Stewart (Sec. 2.2.2: once A and B are
// diagonalised by orthogonal similarities the transformed equation is
// solved elementwise).
//
// Method: two-sided block Jacobi with a parallel (round-robin) ordering
// (Golub & Van Loan Sec. 8.5: the cyclic Jacobi rotation of Alg. 8.5.1,
// its parallel ordering and its block version).  The index set is cut into
// nb2 blocks of JB rows (nb2 even; a trailing block may be partly or wholly
// outside the matrix).  A sweep is nb2 - 1 rounds; in each round the blocks
// are matched into nb2/2 disjoint pairs and
//   k_jac_pairs  (one workgroup per pair) runs one cyclic Jacobi sweep over
//                the 2JB x 2JB pair block in LDS, keeping the accumulated
//                rotation J_g (2JB x 2JB);
//   k_jac_apply  applies every J_g at once, S <- J^T S J and Q <- Q J
//                (J = the direct sum of the J_g), tile by tile: tile (g, h)
//                of S becomes J_g^T S(I_g, I_h) J_h, written together with
//                its transpose so that S stays exactly symmetric.
// A rotation is taken only where |s_pq| > u ||S||_F / n (u = unit roundoff
// of T); the iteration stops after a sweep that took none, which leaves
// ||off(S)||_F <= u ||S||_F.
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

#include <cstring>

namespace sylv {

constexpr int JB = 16;        // rows per block
constexpr int JP = 2 * JB;    // order of a pair block
constexpr int JLD = JP + 1;   // padded LDS leading dimension
// Inner sweeps per pair block and round.  One suffices: the block meets its
// partner again in the next outer sweep, and exact inner diagonalisation
// neither saves outer sweeps nor improves accuracy (it only adds rotations).
constexpr int JIN = 1;

// Round-robin tournament of m + 1 players (m odd), round r in [0, m):
// match g pairs player 0 with 1 + r (g = 0) or 1 + (r + g) mod m with
// 1 + (r - g) mod m.  Over the m rounds every pair meets exactly once.
SYLV_DEVINL void rr_match(int r, int g, int m, int &x, int &y) {
    if (g == 0) {
        x = 0;
        y = 1 + r;
    } else {
        x = 1 + (r + g) % m;
        y = 1 + (r - g + m) % m;
    }
    if (x > y) { int t = x; x = y; y = t; }
}

// Rotation zeroing s_pq (Alg. 8.5.1): t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
// tau = (s_qq - s_pp) / (2 s_pq), c = 1/sqrt(1 + t^2), s = t c.
template <typename T>
SYLV_DEVINL void jac_rot(T app, T aqq, T apq, T &c, T &s, T &t) {
    // hardware reciprocal / square root (a few ulps): the rotation stays
    // orthogonal to working accuracy and the closed-form diagonal update
    // uses the same t
    const T tau = (aqq - app) * frcp(T(2) * apq);
    const T at = fabs(tau);
    T tt;
    if (at > T(1)) {
        const T ri = frcp(at);
        tt = ri * frcp(T(1) + fsqrt(T(1) + ri * ri));
    } else {
        tt = frcp(at + fsqrt(T(1) + at * at));
    }
    t = (tau >= T(0)) ? tt : -tt;
    c = frcp(fsqrt(T(1) + t * t));
    s = t * c;
}

SYLV_DEVINL int pair_first(int t, int bx, int by) { return t < JB ? bx * JB + t : by * JB + (t - JB); }

// 32x32x32 product on MFMA by the four wavefronts of a workgroup, wave w
// computing the 16x16 block (w & 1, w >> 1) of Out = op(A) B with A, B in
// LDS (column-major, ld JLD); op(A) = A^T when ta.  Lane l returns
// Out(16 (w & 1) + (l & 15), 16 (w >> 1) + orow(l, r)) in acc[r].
template <typename T>
SYLV_DEVINL typename mfma16<T>::v4 mm32(const T *A, bool ta, const T *B) {
    typedef typename mfma16<T>::v4 v4;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int i = 16 * (w & 1) + (l & 15), j = 16 * (w >> 1) + (l & 15);
    v4 acc = v4{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < JP / 4; ++kk) {
        const int k = 4 * kk + (l >> 4);
        const T fa = ta ? A[i * JLD + k] : A[k * JLD + i];
        const T fb = B[j * JLD + k];
        acc = mfma16<T>::op(fb, fa, acc);
    }
    return acc;
}

// One workgroup (four wavefronts) per pair g of round r: S(I_g, I_g) <- its
// rotated form, J (device) <- the JP x JP rotation J_g (column-major, ld
// JP), rot[g] = 1 if it is not the identity, count[0] += rotations taken,
// count[1] += 1 if any.  nrm: ||S||_F (binary64, device).
//
// In an inner round the 16 disjoint rotations act on the block as R^T P R,
// which splits into independent 2x2 sub-blocks: thread (p1, p2) owns rows
// {x1, y1} of rotation p1 and columns {x2, y2} of rotation p2 and applies
// R1^T B R2 to them in one pass (the diagonal sub-blocks p1 = p2 take the
// closed form), plus rotation p2 to two rows of the accumulated Q.  Every
// thread forms the two rotations it needs itself, in one loop, so all users
// of a rotation get bit-identical parameters.  Two barriers per round: all
// reads before any write, then the end of the round (which also counts the
// rotations).
template <typename T>
__global__ __launch_bounds__(256) void k_jac_pairs(int n, T *S, int lds, T *J, int *rot, int r, int m,
                                                  const double *nrm, int *count) {
    __shared__ T P[JP * JLD];
    __shared__ T Q[JP * JLD];
    __shared__ T M[JP * JLD];
    const int g = blockIdx.x, tid = threadIdx.x;
    int bx, by;
    rr_match(r, g, m, bx, by);
    const T thr = (T)((double)num<T>::ulp * (*nrm) / (double)(n > 0 ? n : 1));
    bool big = false;
    for (int e = tid; e < JP * JP; e += 256) {
        const int i = e % JP, j = e / JP;
        const int gi = pair_first(i, bx, by), gj = pair_first(j, bx, by);
        const T v = (gi < n && gj < n) ? CM(S, gi, gj, lds) : T(0);
        P[j * JLD + i] = v;
        Q[j * JLD + i] = (i == j) ? T(1) : T(0);
        big = big || (i != j && fabs(v) > thr);
    }
    // a block already below the threshold takes no rotation
    int total = 0;
    if (__syncthreads_or(big)) {
        const int p1 = tid >> 4, p2 = tid & 15;
        for (int sw = 0; sw < JIN; ++sw) {
            int taken = 0;
            for (int rr = 0; rr < JP - 1; ++rr) {
                int xs[2], ys[2];
                T app[2], aqq[2], apq[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    rr_match(rr, h ? p2 : p1, JP - 1, xs[h], ys[h]);
                    app[h] = P[xs[h] * JLD + xs[h]];
                    aqq[h] = P[ys[h] * JLD + ys[h]];
                    apq[h] = P[ys[h] * JLD + xs[h]];
                }
                const int x1 = xs[0], y1 = ys[0], x2 = xs[1], y2 = ys[1];
                T b00 = P[x2 * JLD + x1], b01 = P[y2 * JLD + x1];
                T b10 = P[x2 * JLD + y1], b11 = P[y2 * JLD + y1];
                const int q0 = 2 * p1, q1 = 2 * p1 + 1;
                T qa0 = Q[x2 * JLD + q0], qb0 = Q[y2 * JLD + q0];
                T qa1 = Q[x2 * JLD + q1], qb1 = Q[y2 * JLD + q1];
                __syncthreads();
                T sn[2], tr[2], tt[2];
                bool act[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    T c = T(1);
                    sn[h] = T(0);
                    tt[h] = T(0);
                    act[h] = fabs(apq[h]) > thr;
                    if (act[h]) jac_rot(app[h], aqq[h], apq[h], c, sn[h], tt[h]);
                    tr[h] = act[h] ? sn[h] * frcp(T(1) + c) : T(0);
                }
                if (p1 == p2) {
                    if (act[0]) {
                        P[x1 * JLD + x1] = app[0] - tt[0] * apq[0];
                        P[y1 * JLD + y1] = aqq[0] + tt[0] * apq[0];
                        P[y1 * JLD + x1] = T(0);
                        P[x1 * JLD + y1] = T(0);
                    }
                } else if (act[0] || act[1]) {
                    // rows x1, y1 by rotation 1, then columns x2, y2 by rotation 2
                    T u, v;
                    u = b00; v = b10;
                    b00 = u - sn[0] * (v + tr[0] * u);
                    b10 = v + sn[0] * (u - tr[0] * v);
                    u = b01; v = b11;
                    b01 = u - sn[0] * (v + tr[0] * u);
                    b11 = v + sn[0] * (u - tr[0] * v);
                    u = b00; v = b01;
                    b00 = u - sn[1] * (v + tr[1] * u);
                    b01 = v + sn[1] * (u - tr[1] * v);
                    u = b10; v = b11;
                    b10 = u - sn[1] * (v + tr[1] * u);
                    b11 = v + sn[1] * (u - tr[1] * v);
                    P[x2 * JLD + x1] = b00;
                    P[y2 * JLD + x1] = b01;
                    P[x2 * JLD + y1] = b10;
                    P[y2 * JLD + y1] = b11;
                }
                if (act[1]) {
                    Q[x2 * JLD + q0] = qa0 - sn[1] * (qb0 + tr[1] * qa0);
                    Q[y2 * JLD + q0] = qb0 + sn[1] * (qa0 - tr[1] * qb0);
                    Q[x2 * JLD + q1] = qa1 - sn[1] * (qb1 + tr[1] * qa1);
                    Q[y2 * JLD + q1] = qb1 + sn[1] * (qa1 - tr[1] * qb1);
                }
                taken += __syncthreads_count(p1 == p2 && act[0]);
            }
            total += taken;
            if (taken == 0) break;
        }
    }
    T *Jg = J + (size_t)g * JP * JP;
    if (total == 0) {
        for (int e = tid; e < JP * JP; e += 256) Jg[e] = ((e / JP) == (e % JP)) ? T(1) : T(0);
    } else {
        // The rotated pair block goes back as computed here (symmetrised),
        // not as J_g^T S J_g re-formed by the apply kernel: that product would
        // put rounding noise of order u |s_ii| back into the entries just
        // zeroed, which for close eigenvalues exceeds the rotation threshold.
        for (int e = tid; e < JP * JP; e += 256) {
            const int i = e % JP, j = e / JP;
            const int gi = pair_first(i, bx, by), gj = pair_first(j, bx, by);
            if (gi < n && gj < n) CM(S, gi, gj, lds) = T(0.5) * (P[j * JLD + i] + P[i * JLD + j]);
        }
        // One Newton-Schulz step J <- J (3I - J^T J) / 2 squares the
        // departure from orthogonality that the rotations accumulated, so
        // that the products of J's forming the eigenvectors do not drift.
        const int w = tid >> 6, l = tid & 63, oi = 16 * (w & 1) + (l & 15);
        auto acc = mm32<T>(Q, true, Q);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int oj = 16 * (w >> 1) + mfma16<T>::orow(l, q);
            M[oj * JLD + oi] = (oi == oj ? T(1.5) : T(0)) - T(0.5) * acc[q];
        }
        __syncthreads();
        acc = mm32<T>(Q, false, M);
#pragma unroll
        for (int q = 0; q < 4; ++q) Jg[(16 * (w >> 1) + mfma16<T>::orow(l, q)) * JP + oi] = acc[q];
    }
    if (tid == 0) {
        rot[g] = total > 0 ? 1 : 0;
        if (total > 0) {
            atomicAdd(count, total);
            atomicAdd(count + 1, 1);
        }
    }
}

// Tiles: [0, kp(kp-1)/2) are the off-diagonal S tiles (g < h; the pair
// kernel has already written the diagonal ones), then nrt * kp tiles of Q
// (row tile of JP rows x column pair h).  256 threads = 4 wavefronts.
template <typename T>
__global__ __launch_bounds__(256) void k_jac_apply(int n, T *S, int lds, T *Qm, int ldq, const T *J,
                                                  const int *rot, int r, int m, int kp) {
    __shared__ T X[JP * JLD];
    __shared__ T L[JP * JLD];
    __shared__ T R[JP * JLD];
    __shared__ T W[JP * JLD];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int ntri = kp * (kp - 1) / 2;
    const int oi = 16 * (w & 1) + (l & 15);   // output row of this lane
    int tile = blockIdx.x;
    if (tile < ntri) {
        // tile = h (h - 1) / 2 + g, 0 <= g < h
        int h = (int)((1.0 + sqrt(1.0 + 8.0 * tile)) * 0.5);
        while (h * (h - 1) / 2 > tile) --h;
        while ((h + 1) * h / 2 <= tile) ++h;
        const int g = tile - h * (h - 1) / 2;
        if (!rot[g] && !rot[h]) return;
        int gx, gy, hx, hy;
        rr_match(r, g, m, gx, gy);
        rr_match(r, h, m, hx, hy);
        const T *Jg = J + (size_t)g * JP * JP, *Jh = J + (size_t)h * JP * JP;
        for (int e = tid; e < JP * JP; e += 256) {
            const int a = e % JP, b = e / JP;
            const int ga = pair_first(a, gx, gy), hb = pair_first(b, hx, hy);
            X[b * JLD + a] = (ga < n && hb < n) ? CM(S, ga, hb, lds) : T(0);
            L[b * JLD + a] = Jg[e];
            R[b * JLD + a] = Jh[e];
        }
        __syncthreads();
        // W = Jg^T X
        auto acc = mm32<T>(L, true, X);
#pragma unroll
        for (int q = 0; q < 4; ++q) W[(16 * (w >> 1) + mfma16<T>::orow(l, q)) * JLD + oi] = acc[q];
        __syncthreads();
        // Out = W Jh, staged in X for the two coalesced stores
        acc = mm32<T>(W, false, R);
#pragma unroll
        for (int q = 0; q < 4; ++q) X[(16 * (w >> 1) + mfma16<T>::orow(l, q)) * JLD + oi] = acc[q];
        __syncthreads();
        for (int e = tid; e < JP * JP; e += 256) {
            int a = e % JP, b = e / JP;
            int ga = pair_first(a, gx, gy), hb = pair_first(b, hx, hy);
            if (ga < n && hb < n) CM(S, ga, hb, lds) = X[b * JLD + a];
            // transposed tile: consecutive threads walk down a column of S
            b = e % JP;
            a = e / JP;
            ga = pair_first(a, gx, gy);
            hb = pair_first(b, hx, hy);
            if (ga < n && hb < n) CM(S, hb, ga, lds) = X[b * JLD + a];
        }
    } else {
        tile -= ntri;
        const int h = tile % kp, rb = tile / kp;
        if (!rot[h]) return;
        int hx, hy;
        rr_match(r, h, m, hx, hy);
        const T *Jh = J + (size_t)h * JP * JP;
        for (int e = tid; e < JP * JP; e += 256) {
            const int a = e % JP, b = e / JP;
            const int ra = rb * JP + a, hb = pair_first(b, hx, hy);
            X[b * JLD + a] = (ra < n && hb < n) ? CM(Qm, ra, hb, ldq) : T(0);
            R[b * JLD + a] = Jh[e];
        }
        __syncthreads();
        const auto acc = mm32<T>(X, false, R);
        const int ra = rb * JP + oi;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int hb = pair_first(16 * (w >> 1) + mfma16<T>::orow(l, q), hx, hy);
            if (ra < n && hb < n) CM(Qm, ra, hb, ldq) = acc[q];
        }
    }
}

// dst = (src + src^T) / 2 in binary64, rounded to T
template <typename TS, typename T>
__global__ void k_sym_part(int n, const TS *A, int lda, T *D, int ldd) {
    const size_t total = (size_t)n * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        CM(D, i, j, ldd) = (T)(0.5 * ((double)CM(A, i, j, lda) + (double)CM(A, j, i, lda)));
    }
}

// keep only the diagonal
template <typename T>
__global__ void k_keep_diag(int n, T *D, int ldd) {
    const size_t total = (size_t)n * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        if (i != j) CM(D, i, j, ldd) = T(0);
    }
}

// ||A - A^T||_F^2 partial sums: out[b] per block (binary64)
__global__ __launch_bounds__(256) void k_asym_partial(int n, const double *A, int lda, double *part) {
    __shared__ double red[256];
    const size_t total = (size_t)n * n;
    double acc = 0.0;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        const double d = CM(A, i, j, lda) - CM(A, j, i, lda);
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_asym_final(int nb, const double *part, double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[b];
        *out = sqrt(s);
    }
}

static int grid_for(size_t total) {
    size_t b = (total + 255) / 256;
    return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

void asym_norm(hipStream_t s, int n, const double *A, int lda, double *out, double *scratch) {
    const int nb = 64;
    hipLaunchKernelGGL(k_asym_partial, dim3(nb), dim3(256), 0, s, n, A, lda, scratch);
    hipLaunchKernelGGL(k_asym_final, dim3(1), dim3(64), 0, s, nb, scratch, out);
}

template <typename TS, typename T>
void sym_part(hipStream_t s, int n, const TS *A, int lda, T *D, int ldd) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_sym_part<TS, T>), dim3(grid_for((size_t)n * n)), dim3(256), 0, s, n, A, lda, D, ldd);
}
template void sym_part<double, float>(hipStream_t, int, const double *, int, float *, int);
template void sym_part<double, double>(hipStream_t, int, const double *, int, double *, int);
template void sym_part<float, float>(hipStream_t, int, const float *, int, float *, int);

template <typename T>
__global__ void k_get_diag(int n, const T *D, int ldd, T *d) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) d[i] = CM(D, i, i, ldd);
}
template <typename T>
void get_diag(hipStream_t s, int n, const T *D, int ldd, T *d) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_get_diag<T>), dim3((n + 255) / 256), dim3(256), 0, s, n, D, ldd, d);
}
template void get_diag<float>(hipStream_t, int, const float *, int, float *);
template void get_diag<double>(hipStream_t, int, const double *, int, double *);

static int pair_blocks(int n) {
    int nb = (n + JB - 1) / JB;
    if (nb < 2) nb = 2;
    return nb + (nb & 1);
}

template <typename T>
size_t sym_eig_work_bytes(int n) {
    const size_t kp = (size_t)pair_blocks(n) / 2;
    return kp * JP * JP * sizeof(T) + 256 + kp * sizeof(int) + 256 + 4096;
}
template size_t sym_eig_work_bytes<float>(int);
template size_t sym_eig_work_bytes<double>(int);

// S (n x n, symmetric, overwritten: diagonal = eigenvalues, all other
// entries exact zeros) and Q (n x n, receives the eigenvectors).  ws:
// sym_eig_work_bytes(n) device bytes; hbuf: pinned host scratch (>= 8 bytes).
// Returns 0 with *sweeps = outer sweeps taken, 1 if max_sweeps ran out, or a
// negative HIP code.
template <typename T>
int sym_eig(hipStream_t s, int n, T *S, int lds, T *Q, int ldq, char *ws, char *hbuf, int max_sweeps,
            int *sweeps) {
    if (sweeps) *sweeps = 0;
    if (n <= 0) return 0;
    identity<T>(s, n, Q, ldq);
    const int nb2 = pair_blocks(n), kp = nb2 / 2, m = nb2 - 1;
    T *J = (T *)ws;
    int *rot = (int *)(ws + (((size_t)kp * JP * JP * sizeof(T) + 255) & ~(size_t)255));
    char *tail = (char *)rot + (((size_t)kp * sizeof(int) + 255) & ~(size_t)255);
    int *count = (int *)tail;
    double *nrm = (double *)(tail + 256);
    double *nscr = nrm + 1;
    matnorm<T>(s, n, n, S, lds, nrm, nscr, 0);
    const int nrt = (n + JP - 1) / JP;
    const int tiles = kp * (kp - 1) / 2 + nrt * kp;
    int sw = 0, conv = 0;
    for (; sw < max_sweeps; ++sw) {
        HIP_TRY(hipMemsetAsync(count, 0, 2 * sizeof(int), s));
        for (int r = 0; r < m; ++r) {
            {
                ProfScope ps(KID_JAC_PAIRS, s);
                hipLaunchKernelGGL((k_jac_pairs<T>), dim3(kp), dim3(256), 0, s, n, S, lds, J, rot, r, m, nrm,
                                   count);
            }
            {
                ProfScope ps(KID_JAC_APPLY, s);
                hipLaunchKernelGGL((k_jac_apply<T>), dim3(tiles), dim3(256), 0, s, n, S, lds, Q, ldq, J, rot,
                                   r, m, kp);
            }
        }
        HIP_TRY(hipMemcpyAsync(hbuf, count, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        int cnt[2] = {0, 0};
        std::memcpy(cnt, hbuf, 2 * sizeof(int));
        const int taken = cnt[0];
        // algorithmic work of the pair kernels of this sweep: every rotation
        // updates 32 element pairs of the block's rows, of its columns and of
        // the accumulated rotation (8 flops per pair in Rutishauser's form),
        // plus the Newton-Schulz step of each rotated block (two 32^3 products)
        if (prof_armed(KID_JAC_PAIRS))
            prof_add_work(KID_JAC_PAIRS, 768.0 * taken + 2.0 * 2.0 * JP * JP * JP * cnt[1]);
        if (taken == 0) { conv = 1; ++sw; break; }
    }
    hipLaunchKernelGGL((k_keep_diag<T>), dim3(grid_for((size_t)n * n)), dim3(256), 0, s, n, S, lds);
    if (sweeps) *sweeps = sw;
    return conv ? 0 : 1;
}
template int sym_eig<float>(hipStream_t, int, float *, int, float *, int, char *, char *, int, int *);
template int sym_eig<double>(hipStream_t, int, double *, int, double *, int, char *, char *, int, int *);

// Y(i, j) /= (TA(i,i) + TB(j,j)) with the tri-solve's pivot rule: a
// denominator below smin = u max(max|TA|, max|TB|) is replaced by +-smin and
// *flag set.
template <typename T>
__global__ void k_diag_solve(int m, int n, const T *TA, int ldta, const T *TB, int ldtb, T *Y, int ldy,
                             const double *maxab, int *flag) {
    const T smin = (T)fmax((double)num<T>::ulp * (*maxab), (double)num<T>::safmin);
    const size_t total = (size_t)m * n;
    int f = 0;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        T d = CM(TA, i, i, ldta) + CM(TB, j, j, ldtb);
        if (fabs(d) < smin) { d = (d >= T(0)) ? smin : -smin; f = 1; }
        CM(Y, i, j, ldy) = CM(Y, i, j, ldy) / d;
    }
    if (f) atomicOr(flag, 1);
}

template <typename T>
void diag_solve(hipStream_t s, int m, int n, const T *TA, int ldta, const T *TB, int ldtb, T *Y, int ldy,
                const double *maxab, int *flag) {
    if (m <= 0 || n <= 0) return;
    hipLaunchKernelGGL((k_diag_solve<T>), dim3(grid_for((size_t)m * n)), dim3(256), 0, s, m, n, TA, ldta, TB,
                       ldtb, Y, ldy, maxab, flag);
}
template void diag_solve<float>(hipStream_t, int, int, const float *, int, const float *, int, float *, int,
                                const double *, int *);
template void diag_solve<double>(hipStream_t, int, int, const double *, int, const double *, int, double *,
                                 int, const double *, int *);

}  // namespace sylv
