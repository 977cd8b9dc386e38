"""CPU oracle for the Sylvester / Lyapunov solver — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library.  The numerical core is the plain C file ``oracle.c`` (FP64, single
thread, no BLAS), loaded here through ctypes; ``mlp.py`` holds the numpy FP64
oracle of the precision selector and ``flops.py`` the paper's flop model in
exact rational arithmetic.

Parity status of each function (what pins it is listed in the tests):
  bs_solve / schur / trsyl / kron_solve / sym_solve / rel_residual — pinned
  (Kronecker brute force, closed forms, invariants, cross-routes);
  mlp — pinned by central finite differences;
  flops — pinned by the values printed in the paper.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i = ctypes.c_int


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_hessenberg.argtypes = [_i, _dp, _i, _dp, _i]
    lib.orc_hqr.argtypes = [_i, _dp, _i, _dp, _i]
    lib.orc_schur.argtypes = [_i, _dp, _i, _dp, _i, _dp, _i]
    lib.orc_trsyl.argtypes = [_i, _i, _dp, _i, _dp, _i, _i, _dp, _i]
    lib.orc_bs_solve.argtypes = [_i, _i, _dp, _i, _dp, _i, _dp, _i, _dp, _i, _i]
    lib.orc_rel_residual.argtypes = [_i, _i, _dp, _i, _dp, _i, _dp, _i, _dp, _i, _i]
    lib.orc_rel_residual.restype = ctypes.c_double
    lib.orc_kron_solve.argtypes = [_i, _i, _dp, _i, _dp, _i, _dp, _i, _dp, _i]
    lib.orc_sym_eig.argtypes = [_i, _dp, _i, _dp, _dp, _i]
    lib.orc_sym_solve.argtypes = [_i, _i, _dp, _i, _dp, _i, _dp, _i, _dp, _i]
    lib.orc_quasi_eigs.argtypes = [_i, _dp, _i, _dp, _dp]
    lib.orc_quasi_eigs.restype = None
    _lib = lib
    return lib


def _F(a):
    """float64 Fortran-ordered copy (column-major), as the C code expects."""
    return np.array(a, dtype=np.float64, order="F", copy=True)


def _p(a):
    return a.ctypes.data_as(_dp)


def hessenberg(A):
    """H = U^T A U (Householder, GVL 7.4); returns (H, U)."""
    H = _F(A)
    n = H.shape[0]
    U = np.zeros((n, n), order="F")
    _load().orc_hessenberg(n, _p(H), max(n, 1), _p(U), max(n, 1))
    return H, U


def schur(A):
    """Real Schur form A = U T U^T by the Francis double-shift QR algorithm.
    Returns (T, U, status) with status 0 on success."""
    A = _F(A)
    n = A.shape[0]
    T = np.zeros((n, n), order="F")
    U = np.zeros((n, n), order="F")
    st = _load().orc_schur(n, _p(A), max(n, 1), _p(T), max(n, 1), _p(U), max(n, 1))
    return T, U, st


def quasi_eigs(T):
    """Eigenvalues of a quasi-triangular matrix (complex array)."""
    T = _F(T)
    n = T.shape[0]
    wr = np.zeros(n)
    wi = np.zeros(n)
    _load().orc_quasi_eigs(n, _p(T), max(n, 1), _p(wr), _p(wi))
    return wr + 1j * wi


def trsyl(TA, TB, C, lower_b=False):
    """Quasi-triangular Sylvester TA Y + Y TB = C (lower_b=False) or
    TA Y + Y TB^T = C (lower_b=True).  Returns (Y, perturbed_flag)."""
    TA = _F(TA)
    TB = _F(TB)
    Y = _F(C)
    m, n = Y.shape
    st = _load().orc_trsyl(m, n, _p(TA), max(m, 1), _p(TB), max(TB.shape[0], 1),
                           int(bool(lower_b)), _p(Y), max(m, 1))
    return Y, st


def bs_solve(A, B, C):
    """Bartels-Stewart solution of AX + XB = C in FP64.  Returns (X, status)."""
    A, B, C = _F(A), _F(B), _F(C)
    m, n = C.shape
    X = np.zeros((m, n), order="F")
    st = _load().orc_bs_solve(m, n, _p(A), max(m, 1), _p(B), max(n, 1), _p(C),
                              max(m, 1), _p(X), max(m, 1), 0)
    return X, st


def lyap_solve(A, C):
    """Bartels-Stewart solution of AX + XA^T = C in FP64 (one Schur form)."""
    A, C = _F(A), _F(C)
    n = C.shape[0]
    X = np.zeros((n, n), order="F")
    st = _load().orc_bs_solve(n, n, _p(A), max(n, 1), _p(A), max(n, 1), _p(C),
                              max(n, 1), _p(X), max(n, 1), 1)
    return X, st


def rel_residual(A, B, C, X, lyap=False):
    """Normwise relative residual, eq. (2.1), Frobenius norms, FP64."""
    A, C, X = _F(A), _F(C), _F(X)
    B = A if lyap else _F(B)
    m, n = C.shape
    return _load().orc_rel_residual(m, n, _p(A), max(m, 1), _p(B), max(n, 1), _p(C),
                                    max(m, 1), _p(X), max(m, 1), int(bool(lyap)))


def kron_solve(A, B, C):
    """Dense GEPP solution of M_f vec(X) = vec(C), M_f = I (x) A + B^T (x) I."""
    A, B, C = _F(A), _F(B), _F(C)
    m, n = C.shape
    X = np.zeros((m, n), order="F")
    st = _load().orc_kron_solve(m, n, _p(A), max(m, 1), _p(B), max(n, 1), _p(C),
                                max(m, 1), _p(X), max(m, 1))
    return X, st


def sym_eig(S):
    """Cyclic Jacobi eigen-decomposition of a symmetric matrix: (d, V)."""
    S = _F(S)
    n = S.shape[0]
    d = np.zeros(n)
    V = np.zeros((n, n), order="F")
    _load().orc_sym_eig(n, _p(S), max(n, 1), _p(d), _p(V), max(n, 1))
    return d, V


def sym_solve(A, B, C):
    """Symmetric-coefficient route (Sec. 2.2.2): Y_ij = C~_ij/(d_i + e_j)."""
    A, B, C = _F(A), _F(B), _F(C)
    m, n = C.shape
    X = np.zeros((m, n), order="F")
    _load().orc_sym_solve(m, n, _p(A), max(m, 1), _p(B), max(n, 1), _p(C),
                          max(m, 1), _p(X), max(m, 1))
    return X


def residual_matrix(A, B, C, X, lyap=False):
    """R = C - A X - X B (numpy FP64 products), used for forward checks."""
    A = np.asarray(A)
    Bm = A.T if lyap else np.asarray(B)
    return np.asarray(C) - A @ X - X @ Bm


def block_exact(Q_A, D_A, Q_B, D_B, C):
    """Exact-route solution for A = Q_A D_A Q_A^T, B = Q_B D_B Q_B^T with
    orthogonal Q and block-diagonal (or block upper triangular) D: solve the
    quasi-triangular equation D_A Y + Y D_B = Q_A^T C Q_B with the oracle
    substitution and back-transform.  No Schur factorisation is involved, so
    it is an independent route to X at large sizes."""
    Ct = np.asarray(Q_A).T @ np.asarray(C) @ np.asarray(Q_B)
    Y, _ = trsyl(D_A, D_B, Ct)
    return np.asarray(Q_A) @ Y @ np.asarray(Q_B).T
