"""Independent large-size reference for the normal constructions of the
workloads: A = Q_A D_A Q_A^T, B = Q_B D_B Q_B^T with Q orthogonal and D block
diagonal (1x1 real eigenvalues, 2x2 blocks [[a, w], [-w, a]]).  Then
X = Q_A Y Q_B^T where Y solves D_A Y + Y D_B = Q_A^T C Q_B block pair by
block pair in closed form (vectorised numpy).  No Schur factorisation and no
solver code is involved, so it pins results at sizes the C oracle cannot
reach quickly."""
import numpy as np


def blocks(D):
    n = D.shape[0]
    one, two = [], []
    i = 0
    while i < n:
        if i + 1 < n and D[i + 1, i] != 0.0:
            two.append(i)
            i += 2
        else:
            one.append(i)
            i += 1
    return np.array(one, dtype=int), np.array(two, dtype=int)


def solve_block_diagonal(DA, DB, Ct):
    m, n = Ct.shape
    Y = np.zeros((m, n))
    a1, a2 = blocks(DA)
    b1, b2 = blocks(DB)
    da = np.diag(DA)
    db = np.diag(DB)
    # 1x1 / 1x1
    if len(a1) and len(b1):
        Y[np.ix_(a1, b1)] = Ct[np.ix_(a1, b1)] / (da[a1][:, None] + db[b1][None, :])
    # 2x2 (A) / 1x1 (B): (Ab + b I) y = c
    if len(a2) and len(b1):
        a = DA[a2, a2][:, None]; w12 = DA[a2, a2 + 1][:, None]; w21 = DA[a2 + 1, a2][:, None]
        d = DA[a2 + 1, a2 + 1][:, None]
        b = db[b1][None, :]
        c0 = Ct[np.ix_(a2, b1)]; c1 = Ct[np.ix_(a2 + 1, b1)]
        p, q, r, s = a + b, w12, w21, d + b
        det = p * s - q * r
        Y[np.ix_(a2, b1)] = (s * c0 - q * c1) / det
        Y[np.ix_(a2 + 1, b1)] = (-r * c0 + p * c1) / det
    # 1x1 (A) / 2x2 (B): y (a I + Bb) = c  ->  (a I + Bb)^T y^T = c^T
    if len(a1) and len(b2):
        a = da[a1][:, None]
        p = a + DB[b2, b2][None, :]; q = DB[b2 + 1, b2][None, :]   # transposed entries
        r = DB[b2, b2 + 1][None, :]; s = a + DB[b2 + 1, b2 + 1][None, :]
        c0 = Ct[np.ix_(a1, b2)]; c1 = Ct[np.ix_(a1, b2 + 1)]
        det = p * s - q * r
        Y[np.ix_(a1, b2)] = (s * c0 - q * c1) / det
        Y[np.ix_(a1, b2 + 1)] = (-r * c0 + p * c1) / det
    # 2x2 / 2x2: 4x4 systems (I (x) Ab + Bb^T (x) I) vec(Yb) = vec(Cb)
    if len(a2) and len(b2):
        na, nb = len(a2), len(b2)
        M = np.zeros((na, nb, 4, 4))
        Ab = np.stack([DA[np.ix_([i, i + 1], [i, i + 1])] for i in a2])  # na x 2 x 2
        Bb = np.stack([DB[np.ix_([j, j + 1], [j, j + 1])] for j in b2])
        I2 = np.eye(2)
        KA = np.einsum("ab,ncd->nacbd", I2, Ab).reshape(na, 4, 4)        # I (x) Ab
        KB = np.einsum("nba,cd->nacbd", Bb, I2).reshape(nb, 4, 4)        # Bb^T (x) I
        M = KA[:, None] + KB[None, :]
        rhs = np.stack([Ct[np.ix_(a2, b2)], Ct[np.ix_(a2 + 1, b2)],
                        Ct[np.ix_(a2, b2 + 1)], Ct[np.ix_(a2 + 1, b2 + 1)]], axis=-1)
        sol = np.linalg.solve(M, rhs[..., None])[..., 0]
        Y[np.ix_(a2, b2)] = sol[..., 0]
        Y[np.ix_(a2 + 1, b2)] = sol[..., 1]
        Y[np.ix_(a2, b2 + 1)] = sol[..., 2]
        Y[np.ix_(a2 + 1, b2 + 1)] = sol[..., 3]
    return Y


def exact_solution(cfg):
    """X for a workloads.config2/config3-style dict (normal coefficients)."""
    QA, DA, QB, DB, C = cfg["QA"], cfg["DA"], cfg["QB"], cfg["DB"], cfg["C"]
    Ct = QA.T @ C @ QB
    Y = solve_block_diagonal(DA, DB, Ct)
    return QA @ Y @ QB.T
