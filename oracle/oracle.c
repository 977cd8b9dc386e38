/*
 * Plain CPU FP64 oracle for the Sylvester equation AX + XB = C and the
 * Lyapunov equation AX + XA^T = C.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may build, load or call this code.  It
 * shares nothing with the GPU library: no headers, no helpers, no tables.
 *
 * Everything here is written for clarity, not speed: single thread, no BLAS,
 * column-major storage with explicit leading dimensions, IEEE binary64.
 *
 * What it computes (paper: "Mixed-precision algorithms for solving the
 * Sylvester matrix equation", Dmytryshyn, Fasi, Higham, Liu):
 *   - the Bartels-Stewart algorithm (Sec. 2.2.1): real Schur forms of A and
 *     B, the transformed right-hand side U_A^T C U_B, the quasi-triangular
 *     substitution, and the back-transform X = U_A Y U_B^T;
 *   - the normwise relative residual of eq. (2.1) with Frobenius norms;
 *   - the Kronecker linear system of eq. (1.2), solved by Gaussian
 *     elimination with partial pivoting (tiny sizes only);
 *   - the symmetric-coefficient variant of Sec. 2.2.2 (diagonal Schur
 *     factors), with eigendecompositions from the cyclic Jacobi method.
 *
 * The Schur factorisation follows the textbook QR algorithm the paper cites
 * (Golub & Van Loan, 4th ed., Sec. 7.4-7.5): Householder reduction to upper
 * Hessenberg form, then implicit Francis double-shift sweeps with deflation
 * on negligible subdiagonal entries.  Exceptional shifts after 10 and 20
 * stagnating sweeps follow the published EISPACK/LAPACK heuristic.  2x2
 * diagonal blocks with real eigenvalues are split by one rotation so that
 * every remaining 2x2 block carries a complex-conjugate pair.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#define E(a, i, j, ld) ((a)[(size_t)(j) * (size_t)(ld) + (size_t)(i)])

static const double ORC_U = 1.1102230246251565e-16; /* 2^-53, binary64 unit roundoff */

/* ---------------------------------------------------------------- helpers */

/* 2-norm of x[0..k) by scaling with the largest magnitude (two passes). */
static double scaled_norm(int k, const double *x, int inc)
{
    double mx = 0.0;
    for (int i = 0; i < k; ++i) {
        double a = fabs(x[(size_t)i * inc]);
        if (a > mx) mx = a;
    }
    if (mx == 0.0) return 0.0;
    double s = 0.0;
    for (int i = 0; i < k; ++i) {
        double t = x[(size_t)i * inc] / mx;
        s += t * t;
    }
    return mx * sqrt(s);
}

/* Householder reflector P = I - tau v v^T with v[0] = 1 such that
 * P x = beta e_1 (GVL Alg. 5.1.1, sign chosen to avoid cancellation).
 * x has length k; v receives k entries.  tau = 0 means P = I. */
static void house(int k, const double *x, double *v, double *tau, double *beta)
{
    double alpha = x[0];
    double xn = (k > 1) ? scaled_norm(k - 1, x + 1, 1) : 0.0;
    v[0] = 1.0;
    if (xn == 0.0) {
        for (int i = 1; i < k; ++i) v[i] = 0.0;
        *tau = 0.0;
        *beta = alpha;
        return;
    }
    double nrm = hypot(alpha, xn);
    double b = (alpha >= 0.0) ? -nrm : nrm;
    *tau = (b - alpha) / b;
    double scal = 1.0 / (alpha - b);
    for (int i = 1; i < k; ++i) v[i] = x[i] * scal;
    *beta = b;
}

/* rows r0..r0+k-1, columns c0..c1 of A  <-  (I - tau v v^T) * A */
static void apply_left(double *A, int ld, int k, const double *v, double tau,
                       int r0, int c0, int c1)
{
    if (tau == 0.0) return;
    for (int j = c0; j <= c1; ++j) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s += v[i] * E(A, r0 + i, j, ld);
        s *= tau;
        for (int i = 0; i < k; ++i) E(A, r0 + i, j, ld) -= s * v[i];
    }
}

/* rows q0..q1, columns c0..c0+k-1 of A  <-  A * (I - tau v v^T) */
static void apply_right(double *A, int ld, int k, const double *v, double tau,
                        int q0, int q1, int c0)
{
    if (tau == 0.0) return;
    for (int i = q0; i <= q1; ++i) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s += E(A, i, c0 + j, ld) * v[j];
        s *= tau;
        for (int j = 0; j < k; ++j) E(A, i, c0 + j, ld) -= s * v[j];
    }
}

/* ---------------------------------------------------- Hessenberg (GVL 7.4) */

/* A (n x n) is overwritten by H = U^T A U (upper Hessenberg, exact zeros
 * below the first subdiagonal); U (n x n) receives the accumulated
 * orthogonal factor.  Returns 0. */
int orc_hessenberg(int n, double *A, int lda, double *U, int ldu)
{
    double *v = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *x = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) E(U, i, j, ldu) = (i == j) ? 1.0 : 0.0;
    for (int j = 0; j + 2 < n; ++j) {
        int k = n - j - 1;          /* reflector acts on rows/cols j+1..n-1 */
        for (int i = 0; i < k; ++i) x[i] = E(A, j + 1 + i, j, lda);
        double tau, beta;
        house(k, x, v, &tau, &beta);
        apply_left(A, lda, k, v, tau, j + 1, j, n - 1);
        apply_right(A, lda, k, v, tau, 0, n - 1, j + 1);
        apply_right(U, ldu, k, v, tau, 0, n - 1, j + 1);
        E(A, j + 1, j, lda) = beta;
        for (int i = j + 2; i < n; ++i) E(A, i, j, lda) = 0.0;
    }
    free(v);
    free(x);
    return 0;
}

/* ------------------------------------------- Francis double shift QR (7.5) */

/* True if the 2x2 block [[a,b],[c,d]] has real eigenvalues. */
static int real_eigs_2x2(double a, double b, double c, double d)
{
    double p = 0.5 * (a - d);
    double disc = p * p + b * c;
    return disc >= 0.0;
}

/* Split the 2x2 diagonal block at (k,k) of T if its eigenvalues are real:
 * one plane rotation G (first column = unit eigenvector of the block) makes
 * the block upper triangular.  Rows k,k+1 (columns k..n-1), columns k,k+1
 * (rows 0..k+1) of T and columns k,k+1 of U are updated. */
static void split_block(int n, double *T, int ldt, double *U, int ldu, int k)
{
    double a = E(T, k, k, ldt), b = E(T, k, k + 1, ldt);
    double c = E(T, k + 1, k, ldt), d = E(T, k + 1, k + 1, ldt);
    if (c == 0.0) return;
    if (!real_eigs_2x2(a, b, c, d)) return;
    double p = 0.5 * (a - d);
    double disc = p * p + b * c;
    double r = sqrt(disc);
    /* eigenvalue of larger |lambda - d| pairs well with vector (lambda-d, c) */
    double lam = d + p + (p >= 0.0 ? r : -r);
    double x1 = lam - d, x2 = c;     /* (T - lam I) v = 0 via 2nd row: c v1 + (d-lam) v2 = 0 */
    double nv = hypot(x1, x2);
    if (nv == 0.0) return;
    double cs = x1 / nv, sn = x2 / nv;
    /* G = [[cs, -sn], [sn, cs]]; T <- G^T T G, U <- U G */
    for (int j = k; j < n; ++j) {
        double t1 = E(T, k, j, ldt), t2 = E(T, k + 1, j, ldt);
        E(T, k, j, ldt) = cs * t1 + sn * t2;
        E(T, k + 1, j, ldt) = -sn * t1 + cs * t2;
    }
    for (int i = 0; i <= k + 1; ++i) {
        double t1 = E(T, i, k, ldt), t2 = E(T, i, k + 1, ldt);
        E(T, i, k, ldt) = cs * t1 + sn * t2;
        E(T, i, k + 1, ldt) = -sn * t1 + cs * t2;
    }
    for (int i = 0; i < n; ++i) {
        double t1 = E(U, i, k, ldu), t2 = E(U, i, k + 1, ldu);
        E(U, i, k, ldu) = cs * t1 + sn * t2;
        E(U, i, k + 1, ldu) = -sn * t1 + cs * t2;
    }
    E(T, k + 1, k, ldt) = 0.0;
}

/* Real Schur form of an upper Hessenberg H by the implicit double-shift QR
 * algorithm.  H is overwritten by T (upper quasi-triangular; every 2x2
 * diagonal block has a complex-conjugate pair of eigenvalues; entries below
 * the first subdiagonal are exact zeros, and so is every subdiagonal entry
 * that does not belong to a 2x2 block).  U (n x n) is post-multiplied by the
 * accumulated orthogonal factor.  Returns 0 on success, 1 if more than 30n
 * sweeps were needed. */
int orc_hqr(int n, double *H, int ldh, double *U, int ldu)
{
    int ihi = n - 1;
    int its = 0, total = 0;
    double v[3];
    while (ihi >= 0) {
        /* look for a negligible subdiagonal entry in the active block */
        int l;
        for (l = ihi; l > 0; --l) {
            double s = fabs(E(H, l - 1, l - 1, ldh)) + fabs(E(H, l, l, ldh));
            if (s == 0.0) {
                /* both diagonal entries zero: compare with the neighbours */
                if (l - 2 >= 0) s += fabs(E(H, l - 1, l - 2, ldh));
                if (l + 1 <= ihi) s += fabs(E(H, l + 1, l, ldh));
            }
            if (fabs(E(H, l, l - 1, ldh)) <= ORC_U * s) {
                E(H, l, l - 1, ldh) = 0.0;
                break;
            }
        }
        if (l == ihi) {                      /* 1x1 block converged */
            ihi -= 1;
            its = 0;
            continue;
        }
        if (l == ihi - 1) {                  /* 2x2 block converged */
            split_block(n, H, ldh, U, ldu, ihi - 1);
            ihi -= 2;
            its = 0;
            continue;
        }
        if (++total > 30 * n) return 1;
        ++its;
        /* shifts: eigenvalues of the trailing 2x2, as trace and determinant */
        double h11 = E(H, ihi - 1, ihi - 1, ldh), h12 = E(H, ihi - 1, ihi, ldh);
        double h21 = E(H, ihi, ihi - 1, ldh), h22 = E(H, ihi, ihi, ldh);
        if (its == 10 || its == 20) {
            /* exceptional shift (EISPACK hqr / LAPACK dlahqr heuristic) */
            double s = fabs(E(H, ihi, ihi - 1, ldh)) + fabs(E(H, ihi - 1, ihi - 2, ldh));
            h11 = 0.75 * s + E(H, ihi, ihi, ldh);
            h12 = -0.4375 * s;
            h21 = s;
            h22 = h11;
        }
        /* the two shifts: eigenvalues of the trailing 2x2, s1,2 = re +- r
         * (real pair) or re +- i im (complex pair) */
        double hp = 0.5 * (h11 - h22), disc = hp * hp + h12 * h21;
        int cplx = disc < 0.0;
        double sre = h22 + hp, srad = sqrt(fabs(disc));
        double s1 = sre + srad, s2 = sre - srad;
        /* first column of (H - s1 I)(H - s2 I), restricted to rows l..l+2,
         * formed from the differences a00 - s and a11 - s (no trace and
         * determinant): near a cluster of equal eigenvalues those
         * differences are exact while the expanded polynomial cancels to
         * rounding noise and the iteration would stagnate */
        double a00 = E(H, l, l, ldh), a01 = E(H, l, l + 1, ldh);
        double a10 = E(H, l + 1, l, ldh), a11 = E(H, l + 1, l + 1, ldh);
        double a21 = E(H, l + 2, l + 1, ldh);
        double x, y;
        if (cplx) {
            double d0 = a00 - sre;
            x = d0 * d0 + srad * srad + a01 * a10;
            y = a10 * (d0 + (a11 - sre));
        } else {
            x = (a00 - s1) * (a00 - s2) + a01 * a10;
            y = a10 * ((a00 - s1) + (a11 - s2));
        }
        double z = a10 * a21;
        for (int k = l; k <= ihi - 1; ++k) {
            int len = (k <= ihi - 2) ? 3 : 2;
            double xv[3] = {x, y, z}, tau, beta;
            house(len, xv, v, &tau, &beta);
            int c0 = (k > l) ? k - 1 : l;
            apply_left(H, ldh, len, v, tau, k, c0, n - 1);
            int rmax = (k + 3 <= ihi) ? k + 3 : ihi;
            apply_right(H, ldh, len, v, tau, 0, rmax, k);
            apply_right(U, ldu, len, v, tau, 0, n - 1, k);
            if (k > l) {
                E(H, k, k - 1, ldh) = beta;
                E(H, k + 1, k - 1, ldh) = 0.0;
                if (len == 3) E(H, k + 2, k - 1, ldh) = 0.0;
            }
            if (k <= ihi - 2) {
                x = E(H, k + 1, k, ldh);
                y = E(H, k + 2, k, ldh);
                z = (k <= ihi - 3) ? E(H, k + 3, k, ldh) : 0.0;
            }
        }
    }
    /* clean: exact zeros below the first subdiagonal */
    for (int j = 0; j < n; ++j)
        for (int i = j + 2; i < n; ++i) E(H, i, j, ldh) = 0.0;
    return 0;
}

/* Real Schur decomposition A = U T U^T.  A is not modified.  Returns the
 * status of orc_hqr. */
int orc_schur(int n, const double *A, int lda, double *T, int ldt, double *U, int ldu)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) E(T, i, j, ldt) = E(A, i, j, lda);
    orc_hessenberg(n, T, ldt, U, ldu);
    return orc_hqr(n, T, ldt, U, ldu);
}

/* ------------------------------- small dense solve, complete pivoting GE */

/* Solve the k x k system M z = r (k <= 4, M column-major with ld 4) by
 * Gaussian elimination with complete pivoting.  A pivot smaller than smin in
 * magnitude is replaced by smin (sign kept) and *perturbed is set. */
static void solve_small(int k, double M[16], double r[4], double smin, int *perturbed)
{
    int cperm[4] = {0, 1, 2, 3};
    for (int p = 0; p < k; ++p) {
        int bi = p, bj = p;
        double bv = -1.0;
        for (int j = p; j < k; ++j)
            for (int i = p; i < k; ++i)
                if (fabs(M[j * 4 + i]) > bv) { bv = fabs(M[j * 4 + i]); bi = i; bj = j; }
        if (bi != p) {
            for (int j = 0; j < k; ++j) { double t = M[j * 4 + p]; M[j * 4 + p] = M[j * 4 + bi]; M[j * 4 + bi] = t; }
            double t = r[p]; r[p] = r[bi]; r[bi] = t;
        }
        if (bj != p) {
            for (int i = 0; i < k; ++i) { double t = M[p * 4 + i]; M[p * 4 + i] = M[bj * 4 + i]; M[bj * 4 + i] = t; }
            int t = cperm[p]; cperm[p] = cperm[bj]; cperm[bj] = t;
        }
        if (fabs(M[p * 4 + p]) < smin) {
            M[p * 4 + p] = (M[p * 4 + p] >= 0.0) ? smin : -smin;
            *perturbed = 1;
        }
        for (int i = p + 1; i < k; ++i) {
            double f = M[p * 4 + i] / M[p * 4 + p];
            for (int j = p; j < k; ++j) M[j * 4 + i] -= f * M[j * 4 + p];
            r[i] -= f * r[p];
        }
    }
    double z[4];
    for (int i = k - 1; i >= 0; --i) {
        double s = r[i];
        for (int j = i + 1; j < k; ++j) s -= M[j * 4 + i] * z[j];
        z[i] = s / M[i * 4 + i];
    }
    for (int i = 0; i < k; ++i) r[cperm[i]] = z[i];
}

/* Block starts of a quasi-triangular matrix: blk[i] = size of the diagonal
 * block starting at i (1 or 2), or 0 for the second row of a 2x2 block. */
static void block_map(int n, const double *T, int ldt, int *blk)
{
    int i = 0;
    while (i < n) {
        if (i + 1 < n && E(T, i + 1, i, ldt) != 0.0) {
            blk[i] = 2; blk[i + 1] = 0; i += 2;
        } else {
            blk[i] = 1; i += 1;
        }
    }
}

static double max_abs(int r, int c, const double *A, int ld)
{
    double m = 0.0;
    for (int j = 0; j < c; ++j)
        for (int i = 0; i < r; ++i)
            if (fabs(E(A, i, j, ld)) > m) m = fabs(E(A, i, j, ld));
    return m;
}

/* Quasi-triangular Sylvester equation TA Y + Y TB = C (Bartels-Stewart
 * substitution, paper Sec. 2.2.1; GVL Sec. 7.6.3).
 *   TA: m x m upper quasi-triangular.
 *   lower_b = 0: TB is n x n upper quasi-triangular; block columns of Y are
 *                computed left to right.
 *   lower_b = 1: the coefficient on the right is TB^T (TB upper
 *                quasi-triangular), i.e. TA Y + Y TB^T = C; block columns of
 *                Y are computed right to left.
 * C (m x n) is overwritten by Y.  Returns 1 if a pivot of a small block
 * system was perturbed, else 0. */
int orc_trsyl(int m, int n, const double *TA, int ldta, const double *TB, int ldtb,
              int lower_b, double *C, int ldc)
{
    int *ba = (int *)malloc(sizeof(int) * (m > 0 ? m : 1));
    int *bb = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    block_map(m, TA, ldta, ba);
    block_map(n, TB, ldtb, bb);
    double smin = ORC_U * fmax(max_abs(m, m, TA, ldta), max_abs(n, n, TB, ldtb));
    if (smin < DBL_MIN) smin = DBL_MIN;
    int perturbed = 0;
    /* coefficient on the right, element (r, c) */
#define RB(r, c) (lower_b ? E(TB, (c), (r), ldtb) : E(TB, (r), (c), ldtb))
    /* list the block columns in processing order */
    int *jorder = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int nj = 0;
    for (int j = 0; j < n; ++j) if (bb[j]) jorder[nj++] = j;
    if (lower_b) for (int a = 0, b = nj - 1; a < b; ++a, --b) { int t = jorder[a]; jorder[a] = jorder[b]; jorder[b] = t; }
    for (int t = 0; t < nj; ++t) {
        int j = jorder[t], q = bb[j];
        /* G = C(:, J) - sum over solved block columns J' of Y(:, J') RB(J', J) */
        for (int jj = 0; jj < q; ++jj) {
            for (int s = 0; s < t; ++s) {
                int j2 = jorder[s], q2 = bb[j2];
                for (int kk = 0; kk < q2; ++kk) {
                    double b = RB(j2 + kk, j + jj);
                    if (b == 0.0) continue;
                    for (int i = 0; i < m; ++i) E(C, i, j + jj, ldc) -= E(C, i, j2 + kk, ldc) * b;
                }
            }
        }
        /* back substitution over the row blocks of TA, bottom to top */
        int i = m - 1;
        while (i >= 0) {
            int i0 = (ba[i] == 0) ? i - 1 : i;
            int p = ba[i0];
            /* rhs of the small block system (TA(I,I') Y(I',J) for I' > I already subtracted) */
            double M[16] = {0}, r[4];
            for (int jj = 0; jj < q; ++jj)
                for (int ii = 0; ii < p; ++ii) r[jj * p + ii] = E(C, i0 + ii, j + jj, ldc);
            /* (I_q (x) TA(I,I) + RB(J,J)^T (x) I_p) vec(Y_IJ) = vec(G_I) */
            int k = p * q;
            for (int jj = 0; jj < q; ++jj)
                for (int ii = 0; ii < p; ++ii) {
                    int row = jj * p + ii;
                    for (int kk = 0; kk < p; ++kk) M[(jj * p + kk) * 4 + row] += E(TA, i0 + ii, i0 + kk, ldta);
                    for (int ll = 0; ll < q; ++ll) M[(ll * p + ii) * 4 + row] += RB(j + ll, j + jj);
                }
            solve_small(k, M, r, smin, &perturbed);
            for (int jj = 0; jj < q; ++jj)
                for (int ii = 0; ii < p; ++ii) E(C, i0 + ii, j + jj, ldc) = r[jj * p + ii];
            /* rows above: G(r, J) -= TA(r, I) Y(I, J) */
            for (int jj = 0; jj < q; ++jj)
                for (int ii = 0; ii < p; ++ii) {
                    double y = E(C, i0 + ii, j + jj, ldc);
                    for (int rr = 0; rr < i0; ++rr) E(C, rr, j + jj, ldc) -= E(TA, rr, i0 + ii, ldta) * y;
                }
            i = i0 - 1;
        }
    }
#undef RB
    free(ba); free(bb); free(jorder);
    return perturbed;
}

/* Z = op(X) * op(Y) for square/rectangular plain triple loops (FP64).
 * ta/tb = 1 means transpose. Z is r x c, inner dimension k. */
static void matmul(int r, int c, int k, const double *X, int ldx, int ta,
                   const double *Y, int ldy, int tb, double *Z, int ldz)
{
    for (int j = 0; j < c; ++j)
        for (int i = 0; i < r; ++i) E(Z, i, j, ldz) = 0.0;
    for (int j = 0; j < c; ++j)
        for (int l = 0; l < k; ++l) {
            double y = tb ? E(Y, j, l, ldy) : E(Y, l, j, ldy);
            if (y == 0.0) continue;
            if (!ta) {
                for (int i = 0; i < r; ++i) E(Z, i, j, ldz) += E(X, i, l, ldx) * y;
            } else {
                for (int i = 0; i < r; ++i) E(Z, i, j, ldz) += E(X, l, i, ldx) * y;
            }
        }
}

/* Bartels-Stewart solve of AX + XB = C (lyap = 0) or AX + XA^T = C
 * (lyap = 1, B ignored).  X (m x n) receives the solution.
 * Returns bit 0: trsyl pivot perturbed; bit 1: QR iteration limit hit. */
int orc_bs_solve(int m, int n, const double *A, int lda, const double *B, int ldb,
                 const double *C, int ldc, double *X, int ldx, int lyap)
{
    int st = 0;
    double *TA = (double *)malloc(sizeof(double) * (size_t)m * m);
    double *UA = (double *)malloc(sizeof(double) * (size_t)m * m);
    double *W = (double *)malloc(sizeof(double) * (size_t)m * n);
    double *Y = (double *)malloc(sizeof(double) * (size_t)m * n);
    if (orc_schur(m, A, lda, TA, m, UA, m)) st |= 2;
    const double *TB = TA, *UB = UA;
    double *TBb = NULL, *UBb = NULL;
    if (!lyap) {
        TBb = (double *)malloc(sizeof(double) * (size_t)n * n);
        UBb = (double *)malloc(sizeof(double) * (size_t)n * n);
        if (orc_schur(n, B, ldb, TBb, n, UBb, n)) st |= 2;
        TB = TBb; UB = UBb;
    }
    /* C~ = UA^T C UB */
    matmul(m, n, m, UA, m, 1, C, ldc, 0, W, m);
    matmul(m, n, n, W, m, 0, UB, n, 0, Y, m);
    /* B = UB TB UB^T (Sylvester), or the right coefficient A^T = UA TA^T UA^T */
    if (orc_trsyl(m, n, TA, m, TB, lyap ? m : n, lyap, Y, m)) st |= 1;
    /* X = UA Y UB^T */
    matmul(m, n, m, UA, m, 0, Y, m, 0, W, m);
    matmul(m, n, n, W, m, 0, UB, n, 1, X, ldx);
    free(TA); free(UA); free(W); free(Y); free(TBb); free(UBb);
    return st;
}

/* Normwise relative residual of eq. (2.1), Frobenius norms, FP64:
 *   ||A X + X B - C||_F / (||C||_F + ||X||_F (||A||_F + ||B||_F)).
 * lyap = 1 uses B = A^T. */
double orc_rel_residual(int m, int n, const double *A, int lda, const double *B, int ldb,
                        const double *C, int ldc, const double *X, int ldx, int lyap)
{
    double *R = (double *)malloc(sizeof(double) * (size_t)m * n);
    double *P = (double *)malloc(sizeof(double) * (size_t)m * n);
    matmul(m, n, m, A, lda, 0, X, ldx, 0, R, m);
    if (lyap) matmul(m, n, n, X, ldx, 0, A, lda, 1, P, m);
    else      matmul(m, n, n, X, ldx, 0, B, ldb, 0, P, m);
    double rr = 0, cc = 0, xx = 0, aa = 0, bb = 0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            double r = E(R, i, j, m) + E(P, i, j, m) - E(C, i, j, ldc);
            rr += r * r;
            cc += E(C, i, j, ldc) * E(C, i, j, ldc);
            xx += E(X, i, j, ldx) * E(X, i, j, ldx);
        }
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) aa += E(A, i, j, lda) * E(A, i, j, lda);
    if (lyap) bb = aa;
    else
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) bb += E(B, i, j, ldb) * E(B, i, j, ldb);
    free(R); free(P);
    return sqrt(rr) / (sqrt(cc) + sqrt(xx) * (sqrt(aa) + sqrt(bb)));
}

/* ------------------------------------------------ Kronecker route (1.2) */

/* Solve M_f vec(X) = vec(C), M_f = I_n (x) A + B^T (x) I_m (eq. 1.2), by
 * dense Gaussian elimination with partial pivoting.  vec stacks columns.
 * Intended for mn <= a few thousand.  Returns 0, or 1 on an exactly zero
 * pivot. */
int orc_kron_solve(int m, int n, const double *A, int lda, const double *B, int ldb,
                   const double *C, int ldc, double *X, int ldx)
{
    int N = m * n;
    double *M = (double *)calloc((size_t)N * N, sizeof(double));
    double *r = (double *)malloc(sizeof(double) * (size_t)N);
    /* row index (j*m + i), column index (l*m + k):
     *   [I_n (x) A]   = delta_{jl} A(i,k)
     *   [B^T (x) I_m] = B(l, j) delta_{ik} */
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            int row = j * m + i;
            for (int k = 0; k < m; ++k) E(M, row, j * m + k, N) += E(A, i, k, lda);
            for (int l = 0; l < n; ++l) E(M, row, l * m + i, N) += E(B, l, j, ldb);
            r[row] = E(C, i, j, ldc);
        }
    int st = 0;
    for (int p = 0; p < N; ++p) {
        int bi = p;
        for (int i = p + 1; i < N; ++i) if (fabs(E(M, i, p, N)) > fabs(E(M, bi, p, N))) bi = i;
        if (E(M, bi, p, N) == 0.0) { st = 1; continue; }
        if (bi != p) {
            for (int j = 0; j < N; ++j) { double t = E(M, p, j, N); E(M, p, j, N) = E(M, bi, j, N); E(M, bi, j, N) = t; }
            double t = r[p]; r[p] = r[bi]; r[bi] = t;
        }
        double piv = E(M, p, p, N);
        for (int i = p + 1; i < N; ++i) E(M, i, p, N) /= piv;
        for (int j = p + 1; j < N; ++j) {
            double mpj = E(M, p, j, N);
            if (mpj == 0.0) continue;
            for (int i = p + 1; i < N; ++i) E(M, i, j, N) -= E(M, i, p, N) * mpj;
        }
        for (int i = p + 1; i < N; ++i) r[i] -= E(M, i, p, N) * r[p];
    }
    for (int i = N - 1; i >= 0; --i) {
        double s = r[i];
        for (int j = i + 1; j < N; ++j) s -= E(M, i, j, N) * r[j];
        r[i] = s / E(M, i, i, N);
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) E(X, i, j, ldx) = r[j * m + i];
    free(M); free(r);
    return st;
}

/* ------------------------------- symmetric coefficients (Sec. 2.2.2) */

/* Cyclic Jacobi eigenvalue method for a symmetric S (n x n): S is destroyed,
 * d receives the eigenvalues and V the orthonormal eigenvectors (S = V D V^T).
 * Rotation angles per GVL Alg. 8.5.1 (sym.schur2).  Returns sweeps used. */
int orc_sym_eig(int n, double *S, int lds, double *d, double *V, int ldv)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) E(V, i, j, ldv) = (i == j) ? 1.0 : 0.0;
    int sweep;
    for (sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double s = E(S, i, j, lds) * E(S, i, j, lds);
                tot += s;
                if (i != j) off += s;
            }
        if (off <= ORC_U * ORC_U * tot * 1e-2) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = E(S, p, q, lds);
                if (apq == 0.0) continue;
                double app = E(S, p, p, lds), aqq = E(S, q, q, lds);
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* S <- J^T S J with J = rotation in plane (p,q) */
                for (int k = 0; k < n; ++k) {
                    double skp = E(S, k, p, lds), skq = E(S, k, q, lds);
                    E(S, k, p, lds) = c * skp - s * skq;
                    E(S, k, q, lds) = s * skp + c * skq;
                }
                for (int k = 0; k < n; ++k) {
                    double spk = E(S, p, k, lds), sqk = E(S, q, k, lds);
                    E(S, p, k, lds) = c * spk - s * sqk;
                    E(S, q, k, lds) = s * spk + c * sqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = E(V, k, p, ldv), vkq = E(V, k, q, ldv);
                    E(V, k, p, ldv) = c * vkp - s * vkq;
                    E(V, k, q, ldv) = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) d[i] = E(S, i, i, lds);
    return sweep;
}

/* Symmetric A, B: X = U_A Y U_B^T with Y_ij = C~_ij / (d_i + e_j),
 * C~ = U_A^T C U_B (paper Sec. 2.2.2). */
int orc_sym_solve(int m, int n, const double *A, int lda, const double *B, int ldb,
                  const double *C, int ldc, double *X, int ldx)
{
    double *SA = (double *)malloc(sizeof(double) * (size_t)m * m);
    double *SB = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *UA = (double *)malloc(sizeof(double) * (size_t)m * m);
    double *UB = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *da = (double *)malloc(sizeof(double) * m);
    double *db = (double *)malloc(sizeof(double) * n);
    double *W = (double *)malloc(sizeof(double) * (size_t)m * n);
    double *Y = (double *)malloc(sizeof(double) * (size_t)m * n);
    for (int j = 0; j < m; ++j) for (int i = 0; i < m; ++i) E(SA, i, j, m) = E(A, i, j, lda);
    for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i) E(SB, i, j, n) = E(B, i, j, ldb);
    orc_sym_eig(m, SA, m, da, UA, m);
    orc_sym_eig(n, SB, n, db, UB, n);
    matmul(m, n, m, UA, m, 1, C, ldc, 0, W, m);
    matmul(m, n, n, W, m, 0, UB, n, 0, Y, m);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) E(Y, i, j, m) /= (da[i] + db[j]);
    matmul(m, n, m, UA, m, 0, Y, m, 0, W, m);
    matmul(m, n, n, W, m, 0, UB, n, 1, X, ldx);
    free(SA); free(SB); free(UA); free(UB); free(da); free(db); free(W); free(Y);
    return 0;
}

/* Eigenvalues of a real quasi-triangular T: wr/wi receive real and imaginary
 * parts (a 2x2 block [[a,b],[c,d]] contributes its two eigenvalues). */
void orc_quasi_eigs(int n, const double *T, int ldt, double *wr, double *wi)
{
    int i = 0;
    while (i < n) {
        if (i + 1 < n && E(T, i + 1, i, ldt) != 0.0) {
            double a = E(T, i, i, ldt), b = E(T, i, i + 1, ldt);
            double c = E(T, i + 1, i, ldt), d = E(T, i + 1, i + 1, ldt);
            double p = 0.5 * (a - d), disc = p * p + b * c;
            double mid = 0.5 * (a + d);
            if (disc >= 0.0) {
                double r = sqrt(disc);
                wr[i] = mid + r; wr[i + 1] = mid - r; wi[i] = wi[i + 1] = 0.0;
            } else {
                double r = sqrt(-disc);
                wr[i] = wr[i + 1] = mid; wi[i] = r; wi[i + 1] = -r;
            }
            i += 2;
        } else {
            wr[i] = E(T, i, i, ldt); wi[i] = 0.0;
            i += 1;
        }
    }
}
