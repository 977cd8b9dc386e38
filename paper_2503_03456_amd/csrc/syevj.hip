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
//   k_jac_pairs  (one wavefront per pair) diagonalises the 2JB x 2JB pair
//                block in LDS by cyclic Jacobi sweeps of its own, keeping
//                the accumulated rotation J_g (2JB x 2JB);
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
constexpr int JIN = 12;       // cap on the inner sweeps of one pair block

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
    const T tau = (aqq - app) / (T(2) * apq);
    const T at = fabs(tau);
    T tt;
    if (at > T(1)) {
        const T ri = T(1) / at;
        tt = ri / (T(1) + sqrt(T(1) + ri * ri));
    } else {
        tt = T(1) / (at + sqrt(T(1) + at * at));
    }
    t = (tau >= T(0)) ? tt : -tt;
    c = T(1) / sqrt(T(1) + t * t);
    s = t * c;
}

SYLV_DEVINL int pair_first(int t, int bx, int by) { return t < JB ? bx * JB + t : by * JB + (t - JB); }

// One wavefront per pair g of round r: S(I_g, I_g) <- its diagonalised
// form, J (device) <- the JP x JP rotation J_g (column-major, ld JP),
// rot[g] = 1 if it is not the identity, *count += rotations taken.
// nrm: ||S||_F (binary64, device).
template <typename T>
__global__ __launch_bounds__(64) void k_jac_pairs(int n, T *S, int lds, T *J, int *rot, int r, int m,
                                                 const double *nrm, int *count) {
    __shared__ T P[JP * JLD];
    __shared__ T Q[JP * JLD];
    __shared__ T rs[JB], rtr[JB], rdx[JB], rdy[JB];
    __shared__ int ract[JB];
    const int g = blockIdx.x, lane = threadIdx.x;
    int bx, by;
    rr_match(r, g, m, bx, by);
    const T thr = (T)((double)num<T>::ulp * (*nrm) / (double)(n > 0 ? n : 1));
    for (int e = lane; e < JP * JP; e += 64) {
        const int i = e % JP, j = e / JP;
        const int gi = pair_first(i, bx, by), gj = pair_first(j, bx, by);
        P[j * JLD + i] = (gi < n && gj < n) ? CM(S, gi, gj, lds) : T(0);
        Q[j * JLD + i] = (i == j) ? T(1) : T(0);
    }
    __syncthreads();
    int total = 0;
    for (int sw = 0; sw < JIN; ++sw) {
        int taken = 0;
        for (int rr = 0; rr < JP - 1; ++rr) {
            bool act = false;
            if (lane < JB) {
                int x, y;
                rr_match(rr, lane, JP - 1, x, y);
                const T apq = P[y * JLD + x];
                T c = T(1), s = T(0), t = T(0);
                const T app = P[x * JLD + x], aqq = P[y * JLD + y];
                if (fabs(apq) > thr) {
                    jac_rot(app, aqq, apq, c, s, t);
                    act = true;
                }
                rs[lane] = s;
                rtr[lane] = s / (T(1) + c);
                rdx[lane] = app - t * apq;
                rdy[lane] = aqq + t * apq;
                ract[lane] = act ? 1 : 0;
            }
            const unsigned long long vote = __ballot(act);
            taken += __popcll(vote);
            __syncthreads();
            if (vote) {
                // rows: P <- R^T P (16 pairs x 32 columns, 8 per lane)
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int e = lane + 64 * q, pr = e >> 5, k = e & 31;
                    int x, y;
                    rr_match(rr, pr, JP - 1, x, y);
                    const T s = rs[pr], tr = rtr[pr];
                    const T a = P[k * JLD + x], b = P[k * JLD + y];
                    P[k * JLD + x] = a - s * (b + tr * a);
                    P[k * JLD + y] = b + s * (a - tr * b);
                }
                __syncthreads();
                // columns: P <- P R, Q <- Q R
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int e = lane + 64 * q, pr = e >> 5, k = e & 31;
                    int x, y;
                    rr_match(rr, pr, JP - 1, x, y);
                    const T s = rs[pr], tr = rtr[pr];
                    const T a = P[x * JLD + k], b = P[y * JLD + k];
                    P[x * JLD + k] = a - s * (b + tr * a);
                    P[y * JLD + k] = b + s * (a - tr * b);
                    const T qa = Q[x * JLD + k], qb = Q[y * JLD + k];
                    Q[x * JLD + k] = qa - s * (qb + tr * qa);
                    Q[y * JLD + k] = qb + s * (qa - tr * qb);
                }
                __syncthreads();
                // the rotated 2x2 diagonal block in closed form (Alg. 8.5.1):
                // s_pp - t s_pq, s_qq + t s_pq and an exact zero
                if (lane < JB && ract[lane]) {
                    int x, y;
                    rr_match(rr, lane, JP - 1, x, y);
                    P[x * JLD + x] = rdx[lane];
                    P[y * JLD + y] = rdy[lane];
                    P[x * JLD + y] = T(0);
                    P[y * JLD + x] = T(0);
                }
                __syncthreads();
            }
        }
        total += taken;
        if (taken == 0) break;
    }
    T *Jg = J + (size_t)g * JP * JP;
    // The diagonalised pair block goes back as computed here (symmetrised),
    // not as J_g^T S J_g re-formed by the apply kernel: that product would
    // put rounding noise of order u |s_ii| back into the entries just
    // zeroed, which for close eigenvalues exceeds the rotation threshold.
    if (total > 0)
        for (int e = lane; e < JP * JP; e += 64) {
            const int i = e % JP, j = e / JP;
            const int gi = pair_first(i, bx, by), gj = pair_first(j, bx, by);
            if (gi < n && gj < n)
                CM(S, gi, gj, lds) = T(0.5) * (P[j * JLD + i] + P[i * JLD + j]);
        }
    if (total == 0) {
        for (int e = lane; e < JP * JP; e += 64) Jg[e] = ((e / JP) == (e % JP)) ? T(1) : T(0);
    } else {
        // One Newton-Schulz step J <- J (3I - J^T J) / 2 squares the
        // departure from orthogonality that the rotations accumulated, so
        // that the products of J's forming the eigenvectors do not drift.
        // Lane -> column j, rows i0 .. i0+15.
        __syncthreads();
        const int jc = lane & 31, i0 = (lane >> 5) * 16;
        T acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = T(0);
        for (int k = 0; k < JP; ++k) {
            const T qj = Q[jc * JLD + k];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] += Q[(i0 + q) * JLD + k] * qj;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) P[jc * JLD + i0 + q] = ((i0 + q) == jc ? T(1.5) : T(0)) - T(0.5) * acc[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = T(0);
        for (int k = 0; k < JP; ++k) {
            const T mkj = P[jc * JLD + k];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] += Q[k * JLD + i0 + q] * mkj;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) Jg[jc * JP + i0 + q] = acc[q];
    }
    if (lane == 0) {
        rot[g] = total > 0 ? 1 : 0;
        if (total > 0) atomicAdd(count, total);
    }
}

// Tiles: [0, kp(kp-1)/2) are the off-diagonal S tiles (g < h; the pair
// kernel has already written the diagonal ones), then nrt * kp tiles of Q
// (row tile of JP rows x column pair h).  256 threads, 4 outputs each.
template <typename T>
__global__ __launch_bounds__(256) void k_jac_apply(int n, T *S, int lds, T *Qm, int ldq, const T *J,
                                                  const int *rot, int r, int m, int kp) {
    __shared__ T X[JP * JLD];
    __shared__ T L[JP * JLD];
    __shared__ T R[JP * JLD];
    const int tid = threadIdx.x;
    const int ntri = kp * (kp - 1) / 2;
    int tile = blockIdx.x;
    // thread -> column j, rows i0..i0+3 of the 32 x 32 output
    const int j = tid >> 3, i0 = (tid & 7) * 4;
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
        T w[4] = {T(0), T(0), T(0), T(0)};
        for (int k = 0; k < JP; ++k) {
            const T xv = X[j * JLD + k];
#pragma unroll
            for (int q = 0; q < 4; ++q) w[q] += L[(i0 + q) * JLD + k] * xv;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) X[j * JLD + i0 + q] = w[q];
        __syncthreads();
        // Out = W Jh
        T o[4] = {T(0), T(0), T(0), T(0)};
        for (int k = 0; k < JP; ++k) {
            const T rv = R[j * JLD + k];
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] += X[k * JLD + i0 + q] * rv;
        }
        const int hb = pair_first(j, hx, hy);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ga = pair_first(i0 + q, gx, gy);
            if (ga < n && hb < n) {
                CM(S, ga, hb, lds) = o[q];
                CM(S, hb, ga, lds) = o[q];
            }
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
        T o[4] = {T(0), T(0), T(0), T(0)};
        for (int k = 0; k < JP; ++k) {
            const T rv = R[j * JLD + k];
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] += X[k * JLD + i0 + q] * rv;
        }
        const int hb = pair_first(j, hx, hy);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ra = rb * JP + i0 + q;
            if (ra < n && hb < n) CM(Qm, ra, hb, ldq) = o[q];
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
        HIP_TRY(hipMemsetAsync(count, 0, sizeof(int), s));
        for (int r = 0; r < m; ++r) {
            {
                ProfScope ps(KID_JAC_PAIRS, s);
                hipLaunchKernelGGL((k_jac_pairs<T>), dim3(kp), dim3(64), 0, s, n, S, lds, J, rot, r, m, nrm,
                                   count);
            }
            {
                ProfScope ps(KID_JAC_APPLY, s);
                hipLaunchKernelGGL((k_jac_apply<T>), dim3(tiles), dim3(256), 0, s, n, S, lds, Q, ldq, J, rot,
                                   r, m, kp);
            }
        }
        HIP_TRY(hipMemcpyAsync(hbuf, count, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        int taken = 0;
        std::memcpy(&taken, hbuf, sizeof(int));
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
