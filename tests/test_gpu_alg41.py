"""Algs. 4.1 (SYLV_ALG_ORTH: binary64-orthonormalised Schur vectors) and 4.2
(SYLV_ALG_INV: the low-precision Schur vectors with binary64 inverses) of the
paper -- triangular-basis coefficients and the stationary iteration of
Alg. 3.1 with binary64 tri-solves -- against the FP64 oracle and against the
original-basis refinement on the same equations."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_common import U64, binding, dev, host, relerr, say

pytestmark = pytest.mark.gpu

TOL = 1e-14


def kron_cond(A, B):
    m, n = A.shape[0], B.shape[0]
    return np.linalg.cond(np.kron(np.eye(n), A) + np.kron(B.T, np.eye(m)))


@pytest.mark.parametrize("alg", ["orth", "inv"])
def test_alg41_config1(alg):
    sy = binding()
    A, B, C = workloads.config1()
    X, info = sy.solve(dev(A), dev(B), dev(C), alg=alg)
    torch.cuda.synchronize()
    say("alg41 config1", info)
    assert info["status"] == 0 and info["fell_back"] == 0 and info["rel_res"] <= TOL, info
    assert info["iterations"] >= 1
    Xo, _ = oracle.bs_solve(A, B, C)
    assert relerr(host(X), Xo) <= 100 * U64 * kron_cond(A, B)


@pytest.mark.parametrize("alg", ["orth", "inv"])
@pytest.mark.parametrize("low", ["fp32", "bf16"])
@pytest.mark.parametrize("m,n", [(1, 1), (2, 7), (33, 17), (150, 90), (301, 257)])
def test_alg41_shapes(alg, low, m, n):
    sy = binding()
    A, B, C = workloads.sylv_random(700 + m + n, m, n, scale=0.5 / np.sqrt(max(m, n)))
    X, info = sy.solve(dev(A), dev(B), dev(C), alg=alg, low=low)
    X2, info2 = sy.solve(dev(A), dev(B), dev(C), alg="orig", low=low)
    torch.cuda.synchronize()
    say("alg4x", alg, low, m, n, info["iterations"], info2["iterations"], info["rel_res"])
    assert info["rel_res"] <= TOL and info["fell_back"] == 0, info
    Xo, _ = oracle.bs_solve(A, B, C)
    kap = kron_cond(A, B) if m * n <= 2500 else 10.0
    assert relerr(host(X), Xo) <= 100 * U64 * kap * max(1.0, np.sqrt(m + n) / 8)
    assert relerr(host(X), host(X2)) <= 200 * U64 * kap * max(1.0, np.sqrt(m + n) / 8)


@pytest.mark.parametrize("alg", ["orth", "inv"])
@pytest.mark.parametrize("n", [16, 100, 256])
def test_alg41_lyapunov(alg, n):
    sy = binding()
    A, C, eig = workloads.config4_item(n + 3, n)
    X, info = sy.lyap(dev(A), dev(C), alg=alg)
    torch.cuda.synchronize()
    assert info["rel_res"] <= TOL and info["fell_back"] == 0, info
    Xo, _ = oracle.lyap_solve(A, C)
    lam = eig[:, None] + eig[None, :]
    kap = np.abs(lam).max() / np.abs(lam).min()
    assert relerr(host(X), Xo) <= 100 * U64 * kap
    Xg = host(X)
    assert np.linalg.norm(Xg - Xg.T) <= 100 * U64 * kap * np.linalg.norm(Xg)


@pytest.mark.parametrize("alg", ["orth", "inv"])
def test_alg41_small_sep(alg):
    """sep = 1e-3 (kappa ~ 1e4): the triangular-basis iteration still reaches
    the binary64 residual level."""
    sy = binding()
    cfg = workloads.config3(2, m=300, n=200)
    X, info = sy.solve(dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"]), alg=alg)
    torch.cuda.synchronize()
    say("alg41 small sep", info)
    assert info["rel_res"] <= TOL and info["fell_back"] == 0, info
    Xo, _ = oracle.bs_solve(cfg["A"], cfg["B"], cfg["C"])
    assert relerr(host(X), Xo) <= 1e-9


@pytest.mark.parametrize("n", [1, 63, 64, 65, 300])
def test_cholqr_is_the_qr_factor(n):
    """sylv_cholqr (the binary64 QR step of Alg. 4.1) returns the QR factor
    with positive diag(R) of a nearly orthogonal matrix: equal to numpy's
    Householder QR after its signs are made positive."""
    sy = binding()
    rs = np.random.RandomState(40 + n)
    U = workloads.haar_orthogonal(rs, n) + 1e-5 * rs.standard_normal((n, n))
    Q, R, st = sy.cholqr(dev(U))
    torch.cuda.synchronize()
    assert st == 0
    Qh, Rh = host(Q), host(R)
    Qn, Rn = np.linalg.qr(U)
    d = np.sign(np.diag(Rn))
    Qn, Rn = Qn * d[None, :], Rn * d[:, None]
    assert np.all(np.tril(Rh, -1) == 0) and np.all(np.diag(Rh) > 0)
    assert np.linalg.norm(Qh - Qn) <= 20 * n * U64
    assert np.linalg.norm(Rh - Rn) <= 20 * n * U64 * np.linalg.norm(Rn)
    assert np.linalg.norm(Qh.T @ Qh - np.eye(n)) <= 10 * n * U64
    assert np.linalg.norm(Qh @ Rh - U) <= 10 * n * U64 * np.linalg.norm(U)


def test_cholqr_reports_a_breakdown():
    sy = binding()
    U = np.eye(70)
    U[:, 5] = 0.0    # rank deficient: G has a zero pivot
    _, _, st = sy.cholqr(dev(U))
    torch.cuda.synchronize()
    assert st == 2
