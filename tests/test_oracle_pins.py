"""Pins for the CPU oracle: each test checks the oracle against something
other than itself — the Kronecker linear system of eq. (1.2) solved by a
library or by brute force, closed forms, invariants of the Schur form and of
the Lyapunov solution, and manufactured solutions."""
import numpy as np
import pytest

import oracle
import workloads

U = 2.0 ** -53


def kron_matrix(A, B):
    m, n = A.shape[0], B.shape[0]
    return np.kron(np.eye(n), A) + np.kron(B.T, np.eye(m))


def kron_np(A, B, C):
    """numpy/LAPACK dgesv solution of M_f vec(X) = vec(C) (eq. 1.2)."""
    m, n = C.shape
    x = np.linalg.solve(kron_matrix(A, B), np.asarray(C).ravel(order="F"))
    return x.reshape((m, n), order="F")


def relerr(X, Y):
    return np.linalg.norm(X - Y) / max(np.linalg.norm(Y), 1e-300)


def quasi_tri(n, rs, pattern):
    """Random upper quasi-triangular matrix with 2x2 blocks (complex pairs)
    where ``pattern`` (list of block sizes) says so."""
    T = np.triu(rs.standard_normal((n, n))) * 0.3
    i = 0
    for p in pattern:
        if p == 1:
            T[i, i] = rs.uniform(1.0, 3.0) * rs.choice([-1, 1])
        else:
            a, w = rs.uniform(1.0, 3.0), rs.uniform(0.5, 2.0)
            T[i, i] = T[i + 1, i + 1] = a
            T[i, i + 1] = w * rs.uniform(0.5, 2.0)
            T[i + 1, i] = -w * w / T[i, i + 1]
        i += p
    return T


def patterns(n):
    """All compositions of n into parts 1 and 2."""
    if n == 0:
        return [[]]
    out = [[1] + p for p in patterns(n - 1)]
    if n >= 2:
        out += [[2] + p for p in patterns(n - 2)]
    return out


# ------------------------------------------------------------ P1 Kronecker

@pytest.mark.parametrize("m,n", [(1, 1), (1, 5), (5, 1), (2, 2), (3, 4), (7, 5), (8, 8), (13, 11)])
def test_bs_matches_kronecker_brute_force(m, n):
    A, B, C = workloads.sylv_random(1000 + 10 * m + n, m, n, shift=1.0, scale=0.5)
    X, st = oracle.bs_solve(A, B, C)
    assert st == 0
    Xk, stk = oracle.kron_solve(A, B, C)
    assert stk == 0
    kappa = np.linalg.cond(kron_matrix(A, B))
    assert relerr(X, Xk) <= 100 * U * kappa
    # independent library route
    assert relerr(Xk, kron_np(A, B, C)) <= 100 * U * kappa


def test_config1_vs_library_kronecker_4096():
    """Config 1 (m=n=64): the 4096 x 4096 Kronecker system by LAPACK dgesv."""
    A, B, C = workloads.config1()
    X, st = oracle.bs_solve(A, B, C)
    assert st == 0
    M = kron_matrix(A, B)
    s = np.linalg.svd(M, compute_uv=False)
    kappa = s[0] / s[-1]
    Xk = np.linalg.solve(M, C.ravel(order="F")).reshape((64, 64), order="F")
    assert relerr(X, Xk) <= 100 * U * kappa
    assert oracle.rel_residual(A, B, C, X) <= 1e-15


def test_kronecker_pin_catches_transposed_operand():
    """A mistake planted in the oracle's output (X solving AX + XB^T = C)
    must fail the Kronecker pin."""
    A, B, C = workloads.sylv_random(7, 6, 6, shift=1.0, scale=0.5)
    Xwrong, _ = oracle.bs_solve(A, B.T, C)
    kappa = np.linalg.cond(kron_matrix(A, B))
    assert relerr(Xwrong, kron_np(A, B, C)) > 1e3 * 100 * U * kappa


# -------------------------------------------------------- P2 closed forms

def test_closed_form_diagonal():
    rs = np.random.RandomState(5)
    a = rs.uniform(0.5, 3, 9)
    b = rs.uniform(0.5, 3, 6)
    C = rs.standard_normal((9, 6))
    X, _ = oracle.bs_solve(np.diag(a), np.diag(b), C)
    Xc = C / (a[:, None] + b[None, :])
    assert relerr(X, Xc) <= 4 * U * 10


def test_closed_form_scalar_multiples():
    rs = np.random.RandomState(6)
    C = rs.standard_normal((7, 4))
    X, _ = oracle.bs_solve(1.75 * np.eye(7), 0.5 * np.eye(4), C)
    assert relerr(X, C / 2.25) <= 4 * U


def test_closed_form_triangular_2x1():
    A = np.array([[2.0, 0.7], [0.0, 1.5]])
    b = 0.25
    c = np.array([[1.3], [-0.4]])
    X, _ = oracle.bs_solve(A, np.array([[b]]), c)
    x2 = c[1, 0] / (A[1, 1] + b)
    x1 = (c[0, 0] - A[0, 1] * x2) / (A[0, 0] + b)
    assert relerr(X[:, 0], np.array([x1, x2])) <= 8 * U


def test_closed_form_rotation_block():
    """A = [[a, w], [-w, a]] (eigenvalues a +- i w), scalar B = b:
    (A + bI)^{-1} = [[a+b, -w], [w, a+b]] / ((a+b)^2 + w^2)."""
    a, w, b = 1.2, 0.9, 0.3
    A = np.array([[a, w], [-w, a]])
    C = np.array([[0.8, -1.1, 0.2], [0.3, 0.5, -0.7]])
    Bm = b * np.eye(3)
    X, _ = oracle.bs_solve(A, Bm, C)
    Xc = np.array([[a + b, -w], [w, a + b]]) @ C / ((a + b) ** 2 + w ** 2)
    assert relerr(X, Xc) <= 16 * U


def test_closed_form_lyapunov_diagonal():
    rs = np.random.RandomState(8)
    lam = -rs.uniform(0.1, 5, 10)
    C = rs.standard_normal((10, 10))
    X, _ = oracle.lyap_solve(np.diag(lam), C)
    Xc = C / (lam[:, None] + lam[None, :])
    assert relerr(X, Xc) <= 16 * U


def test_closed_form_rotated_normal_spectrum():
    """A = Q_A D_A Q_A^T with known block-diagonal D_A (complex pairs):
    X = Q_A Y Q_B^T where Y solves the block-diagonal equation block by block
    (2x2 blocks by an explicit 4x4 solve).  Exercises the oracle's full Schur
    path on matrices with 2x2 blocks."""
    m, n = 23, 17
    A, ea, QA, DA = workloads.normal_coeff(31, m, 0.5, 5.0)
    B, eb, QB, DB = workloads.normal_coeff(32, n, 0.5, 5.0)
    C = np.asfortranarray(np.random.RandomState(33).standard_normal((m, n)))
    X, st = oracle.bs_solve(A, B, C)
    assert st == 0
    Ct = QA.T @ C @ QB

    def blocks(D):
        out, i = [], 0
        while i < D.shape[0]:
            if i + 1 < D.shape[0] and D[i + 1, i] != 0:
                out.append((i, 2)); i += 2
            else:
                out.append((i, 1)); i += 1
        return out

    Y = np.zeros((m, n))
    for (i, p) in blocks(DA):
        for (j, q) in blocks(DB):
            Ab = DA[i:i + p, i:i + p]
            Bb = DB[j:j + q, j:j + q]
            M = np.kron(np.eye(q), Ab) + np.kron(Bb.T, np.eye(p))
            Y[i:i + p, j:j + q] = np.linalg.solve(M, Ct[i:i + p, j:j + q].ravel(order="F")).reshape((p, q), order="F")
    Xc = QA @ Y @ QB.T
    lam = ea[:, None] + eb[None, :]
    kappa = np.abs(lam).max() / np.abs(lam).min()
    assert relerr(X, Xc) <= 100 * U * kappa * max(m, n)


# ------------------------------------------------- P3 symmetric cross-route

def test_symmetric_cross_route():
    rs = np.random.RandomState(9)
    m, n = 14, 9
    GA = rs.standard_normal((m, m))
    GB = rs.standard_normal((n, n))
    A = GA + GA.T + 12 * np.eye(m)
    B = GB + GB.T + 12 * np.eye(n)
    C = rs.standard_normal((m, n))
    X1 = oracle.sym_solve(A, B, C)
    X2, _ = oracle.bs_solve(A, B, C)
    kappa = np.linalg.cond(kron_matrix(A, B))
    assert relerr(X1, X2) <= 100 * U * kappa * 10
    assert relerr(X1, kron_np(A, B, C)) <= 100 * U * kappa * 10


def test_jacobi_eigs_match_library():
    rs = np.random.RandomState(10)
    G = rs.standard_normal((12, 12))
    S = G + G.T
    d, V = oracle.sym_eig(S)
    assert np.allclose(np.sort(d), np.linalg.eigvalsh(S), rtol=0, atol=1e-13 * np.abs(d).max())
    assert np.linalg.norm(V.T @ V - np.eye(12)) < 1e-13
    assert np.linalg.norm(S - V @ np.diag(d) @ V.T) < 1e-13 * np.linalg.norm(S)


def test_jacobi_closed_form_tridiagonal_toeplitz():
    """tridiag(-1, 2, -1) of order n has eigenvalues 2 - 2 cos(k pi/(n+1))
    and eigenvectors sin(i k pi/(n+1)) (a textbook closed form)."""
    for n in (1, 2, 7, 30):
        S = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
        d, V = oracle.sym_eig(S)
        k = np.arange(1, n + 1)
        lam = np.sort(2 - 2 * np.cos(k * np.pi / (n + 1)))
        assert np.abs(np.sort(d) - lam).max() <= 1e-14 * 4
        i = np.argsort(d)[0]
        v = np.sin(np.arange(1, n + 1) * np.pi / (n + 1))
        v /= np.linalg.norm(v)
        assert abs(abs(V[:, i] @ v) - 1) <= 1e-13


def test_jacobi_closed_form_2x2_and_rank_one():
    a, b, c = 3.0, 1.5, -2.0
    d, V = oracle.sym_eig(np.array([[a, b], [b, c]]))
    mid, rad = (a + c) / 2, np.hypot((a - c) / 2, b)
    assert np.allclose(np.sort(d), [mid - rad, mid + rad], rtol=0, atol=1e-15 * 8)
    # I + v v^T: eigenvalue 1 (multiplicity n-1) and 1 + |v|^2 with vector v
    rs = np.random.RandomState(21)
    v = rs.standard_normal(9)
    d, V = oracle.sym_eig(np.eye(9) + np.outer(v, v))
    ds = np.sort(d)
    assert np.abs(ds[:-1] - 1).max() <= 1e-14 * 20 and abs(ds[-1] - (1 + v @ v)) <= 1e-13 * (1 + v @ v)
    i = np.argmax(d)
    assert abs(abs(V[:, i] @ v) / np.linalg.norm(v) - 1) <= 1e-13


def test_symmetric_route_closed_form_diagonal():
    """Diagonal A, B: X_ij = C_ij / (a_i + b_j) exactly (up to one rounding)."""
    rs = np.random.RandomState(22)
    a, b = rs.uniform(0.5, 5, 11), rs.uniform(0.5, 5, 6)
    C = rs.standard_normal((11, 6))
    X = oracle.sym_solve(np.diag(a), np.diag(b), C)
    assert np.abs(X - C / (a[:, None] + b[None, :])).max() <= 4 * U * np.abs(X).max()


def test_symmetric_route_planted_spectrum():
    """A = Q_A diag(la) Q_A^T, B likewise: X = Q_A ((Q_A^T C Q_B) / (la_i + lb_j)) Q_B^T
    from the planted factors agrees with the oracle's own eigen-decompositions."""
    A, la, QA = workloads.sym_coeff(23, 40, repeated=5)
    B, lb, QB = workloads.sym_coeff(24, 25)
    C = np.random.RandomState(25).standard_normal((40, 25))
    Xp = QA @ ((QA.T @ C @ QB) / (la[:, None] + lb[None, :])) @ QB.T
    X = oracle.sym_solve(A, B, C)
    assert relerr(X, Xp) <= 1e3 * U
    d, V = oracle.sym_eig(A)
    assert np.abs(np.sort(d) - np.sort(la)).max() <= 1e3 * U


# ------------------------------------------------ P4 Lyapunov invariants

def test_lyapunov_symmetry_and_psd():
    A, C, eig = workloads.config4_item(3, 40)
    X, st = oracle.lyap_solve(A, C)
    assert st == 0
    nx = np.linalg.norm(X)
    lam = eig[:, None] + eig[None, :]
    kappa = np.abs(lam).max() / np.abs(lam).min()
    assert np.linalg.norm(X - X.T) / nx <= 100 * U * kappa
    w = np.linalg.eigvalsh(0.5 * (X + X.T))
    assert w.min() >= -100 * U * np.abs(w).max()
    assert oracle.rel_residual(A, None, C, X, lyap=True) <= 1e-14
    # cross-route: Kronecker with B = A^T
    Xk = kron_np(A, A.T, C)
    assert relerr(X, Xk) <= 100 * U * kappa * 10


# --------------------------------------------- P5 manufactured solution

def test_manufactured_solution_forward_error():
    m, n = 30, 20
    A, B, Xs = workloads.manufactured(11, m, n)
    # right-hand side in extended precision, rounded once to binary64
    Al, Bl, Xl = (np.asarray(M, dtype=np.longdouble) for M in (A, B, Xs))
    C = np.asarray(Al @ Xl + Xl @ Bl, dtype=np.float64)
    X, _ = oracle.bs_solve(A, B, C)
    kappa = np.linalg.cond(kron_matrix(A, B))
    assert relerr(X, Xs) <= 100 * U * kappa


# ------------------------------------------------------ P6 Schur invariants

def check_schur(A, T, Uq, eig_true=None, tol_mult=10):
    n = A.shape[0]
    na = np.linalg.norm(A)
    assert np.linalg.norm(A - Uq @ T @ Uq.T) / na <= tol_mult * n * U
    assert np.linalg.norm(Uq.T @ Uq - np.eye(n)) <= tol_mult * n * U
    # quasi-triangular: zero below the subdiagonal, no two consecutive nonzero
    # subdiagonal entries, every 2x2 block has complex eigenvalues
    assert np.all(np.tril(T, -2) == 0)
    sub = np.diag(T, -1)
    assert not np.any((sub[:-1] != 0) & (sub[1:] != 0))
    for i in np.nonzero(sub)[0]:
        a, b, c, d = T[i, i], T[i, i + 1], T[i + 1, i], T[i + 1, i + 1]
        assert (0.5 * (a - d)) ** 2 + b * c < 0
    if eig_true is not None:
        ev = oracle.quasi_eigs(T)
        key = lambda z: (round(z.real, 6), z.imag)
        e1 = np.array(sorted(ev, key=key))
        e2 = np.array(sorted(eig_true, key=key))
        assert np.max(np.abs(e1 - e2)) <= 10 * n * U * np.linalg.norm(A, 2) * 10


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 64])
def test_schur_invariants_random(n):
    rs = np.random.RandomState(40 + n)
    A = rs.standard_normal((n, n))
    T, Uq, st = oracle.schur(A)
    assert st == 0
    check_schur(A, T, Uq)
    ev = oracle.quasi_eigs(T)
    ref = np.linalg.eigvals(A)
    # multiset comparison by optimal matching (greedy on sorted values is
    # enough for well separated random spectra at these sizes)
    for z in ref:
        assert np.min(np.abs(ev - z)) <= 1e-10 * max(1.0, np.abs(ref).max())


def test_schur_invariants_constructed_spectrum():
    A, ea, QA, DA = workloads.normal_coeff(2, 150, 0.5, 5.0)
    T, Uq, st = oracle.schur(A)
    assert st == 0
    check_schur(A, T, Uq, eig_true=ea)


@pytest.mark.parametrize("rep", [5, 13, 20])
def test_schur_repeated_eigenvalue_cluster(rep):
    """A symmetric matrix whose spectrum holds `rep` copies of one value:
    the QR iteration must still converge (no cap), with backward error and
    orthogonality at the n u level and the planted spectrum recovered."""
    A, lam, _ = workloads.sym_coeff(641, 40, repeated=rep)
    T, Uq, st = oracle.schur(A)
    assert st == 0
    check_schur(A, T, Uq, eig_true=lam)


def test_hessenberg_invariants():
    rs = np.random.RandomState(50)
    A = rs.standard_normal((30, 30))
    H, Uq = oracle.hessenberg(A)
    assert np.all(np.tril(H, -2) == 0)
    assert np.linalg.norm(A - Uq @ H @ Uq.T) <= 100 * U * np.linalg.norm(A)
    assert np.linalg.norm(Uq.T @ Uq - np.eye(30)) <= 100 * U


def test_schur_special_matrices():
    # already triangular, zero matrix, a Jordan-like block, a pure rotation
    for A in [np.triu(np.arange(1.0, 17.0).reshape(4, 4)), np.zeros((5, 5)),
              np.eye(6) + np.diag(np.ones(5), 1),
              np.array([[0.0, 1.0], [-1.0, 0.0]])]:
        T, Uq, st = oracle.schur(A)
        assert st == 0
        n = A.shape[0]
        assert np.linalg.norm(A - Uq @ T @ Uq.T) <= 10 * n * U * max(1.0, np.linalg.norm(A))


# -------------------------------------------- quasi-triangular substitution

@pytest.mark.parametrize("m,n", [(1, 1), (2, 2), (3, 3), (4, 2), (2, 4), (4, 4), (5, 3)])
def test_trsyl_all_block_patterns_vs_kronecker(m, n):
    rs = np.random.RandomState(60 + m * 7 + n)
    for pa in patterns(m):
        for pb in patterns(n):
            TA = quasi_tri(m, rs, pa)
            TB = quasi_tri(n, rs, pb)
            C = rs.standard_normal((m, n))
            Y, st = oracle.trsyl(TA, TB, C)
            assert st == 0
            kappa = np.linalg.cond(kron_matrix(TA, TB))
            assert relerr(Y, kron_np(TA, TB, C)) <= 100 * U * kappa
            # transposed right coefficient (Lyapunov-type ordering)
            Yl, _ = oracle.trsyl(TA, TB, C, lower_b=True)
            kappa = np.linalg.cond(kron_matrix(TA, TB.T))
            assert relerr(Yl, kron_np(TA, TB.T, C)) <= 100 * U * kappa


def test_trsyl_singular_pivot_is_perturbed():
    """lambda(TA) = -mu(TB) exactly: the small system is singular; the pivot
    is replaced by s_min and the flag is raised (result finite)."""
    TA = np.array([[1.0, 0.5], [0.0, 2.0]])
    TB = np.array([[-2.0]])
    C = np.array([[1.0], [1.0]])
    Y, st = oracle.trsyl(TA, TB, C)
    assert st == 1
    assert np.all(np.isfinite(Y))


# ------------------------------------------------------- P7 sep by design

def test_sep_construction_equals_delta():
    """Config-3 recipe at a small size: normal A and B, so sep_F(A,-B) =
    sigma_min(M_f) = min |lambda_i + mu_j| = delta (Varah)."""
    for delta in [1e-1, 1e-3]:
        A, ea, _, _ = workloads.normal_coeff(70, 12, 0.5, 5.0, planted=0.5, shift=delta - 1.0)
        B, eb, _, _ = workloads.normal_coeff(71, 8, 0.5, 5.0, planted=0.5)
        s = np.linalg.svd(kron_matrix(A, B), compute_uv=False)
        assert abs(s[-1] - delta) <= 1e-12
        assert abs(np.abs(ea[:, None] + eb[None, :]).min() - delta) <= 1e-14


# ---------------------------------------------------- P10 degenerate shapes

def test_degenerate_column_and_row():
    rs = np.random.RandomState(80)
    A = rs.standard_normal((6, 6)) * 0.3 + 2 * np.eye(6)
    b = 0.7
    c = rs.standard_normal((6, 1))
    X, _ = oracle.bs_solve(A, np.array([[b]]), c)
    assert relerr(X, np.linalg.solve(A + b * np.eye(6), c)) <= 1e-14
    r = rs.standard_normal((1, 6))
    X2, _ = oracle.bs_solve(np.array([[b]]), A, r)
    assert relerr(X2, np.linalg.solve((A + b * np.eye(6)).T, r.T).T) <= 1e-14


def test_empty_shapes():
    X, st = oracle.bs_solve(np.zeros((0, 0)), np.zeros((3, 3)) + np.eye(3), np.zeros((0, 3)))
    assert X.shape == (0, 3) and st == 0
