"""Symmetric-coefficient variant (Sec. 2.2.2) on the GPU: the block-Jacobi
eigen-decomposition against the oracle's cyclic Jacobi and against planted
spectra, and the elementwise-solve route with original-basis refinement
(SYLV_ALG_SYM) against the oracle's symmetric route and Bartels-Stewart."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_common import U32, U64, binding, dev, host, relerr, say

pytestmark = pytest.mark.gpu

TOL = 1e-14


def _eig_checks(S, d, Q, u, mult):
    n = S.shape[0]
    ns = max(np.linalg.norm(S), 1e-300)
    orth = np.linalg.norm(Q.T @ Q - np.eye(n))
    bwd = np.linalg.norm(S - (Q * d[None, :]) @ Q.T) / ns
    assert orth <= mult * n * u, ("orthogonality", orth / u)
    assert bwd <= mult * n * u, ("backward error", bwd / u)
    do, _ = oracle.sym_eig(S)
    # Weyl: eigenvalues move by at most the 2-norm of the backward error
    err = np.abs(np.sort(d) - np.sort(do)).max()
    assert err <= 2 * mult * n * u * ns, ("eigenvalues", err / (u * ns))
    return orth / u, bwd / u


@pytest.mark.parametrize("dt", ["fp32", "fp64"])
@pytest.mark.parametrize("n,kind", [(1, "rand"), (2, "rand"), (17, "rand"), (32, "rand"), (33, "planted"),
                                    (100, "planted"), (131, "repeated"), (257, "planted")])
def test_sym_eig_parity(n, kind, dt):
    sy = binding()
    say(f"sym_eig n={n} {kind} {dt}")
    if kind == "rand":
        G = np.random.RandomState(400 + n).standard_normal((n, n))
        S = G + G.T
    else:
        S, lam, _ = workloads.sym_coeff(410 + n, n, repeated=(n // 3 if kind == "repeated" else 0))
    tdt = torch.float32 if dt == "fp32" else torch.float64
    u = U32 if dt == "fp32" else U64
    d, Q, sweeps, st = sy.sym_eig(dev(S, tdt))
    torch.cuda.synchronize()
    assert st == 0 and 1 <= sweeps <= 30, (st, sweeps)
    Sr = S.astype(np.float32).astype(np.float64) if dt == "fp32" else S
    o, b = _eig_checks(Sr, host(d), host(Q), u, mult=4)
    say(f"  sweeps {sweeps} orth/u {o:.1f} bwd/u {b:.1f}")
    if kind != "rand":
        assert np.abs(np.sort(host(d)) - np.sort(lam)).max() <= 8 * n * u * np.linalg.norm(S) + 1e-15


@pytest.mark.parametrize("dt", ["fp32", "fp64"])
def test_sym_eig_diagonal_and_identity_are_exact(dt):
    sy = binding()
    tdt = torch.float32 if dt == "fp32" else torch.float64
    a = np.random.RandomState(5).uniform(-3, 3, 70)
    for S in (np.diag(a), 2.0 * np.eye(70)):
        d, Q, sweeps, st = sy.sym_eig(dev(S, tdt))
        torch.cuda.synchronize()
        assert st == 0 and sweeps == 1
        assert np.array_equal(host(d), np.diag(S).astype(np.float32 if dt == "fp32" else np.float64))
        assert np.array_equal(host(Q), np.eye(70))


def test_sym_eig_uses_symmetric_part():
    sy = binding()
    G = np.random.RandomState(6).standard_normal((45, 45))
    d, Q, _, st = sy.sym_eig(dev(G))
    torch.cuda.synchronize()
    _eig_checks(0.5 * (G + G.T), host(d), host(Q), U64, mult=4)


def test_sym_eig_empty():
    sy = binding()
    d, Q, sweeps, st = sy.sym_eig(torch.empty((0, 0), dtype=torch.float64, device="cuda"))
    assert d.numel() == 0 and sweeps == 0 and st == 0


@pytest.mark.parametrize("m,n", [(1, 1), (2, 3), (40, 40), (100, 67), (257, 130)])
@pytest.mark.parametrize("low", ["fp32", "bf16"])
def test_sym_solve_parity(m, n, low):
    sy = binding()
    say(f"sym solve m={m} n={n} low={low}")
    A, la, _ = workloads.sym_coeff(500 + m, m)
    B, lb, _ = workloads.sym_coeff(600 + n, n, repeated=n // 4)
    C = np.random.RandomState(700 + m + n).standard_normal((m, n))
    X, info = sy.solve(dev(A), dev(B), dev(C), low=low, alg="sym")
    torch.cuda.synchronize()
    assert info["rel_res"] <= TOL and info["fell_back"] == 0 and info["status"] == 0, info
    assert info["iterations"] <= (6 if low == "fp32" else 16), info
    kappa = (la.max() + lb.max()) / (la.min() + lb.min())
    Xo = oracle.sym_solve(A, B, C)
    assert relerr(host(X), Xo) <= 50 * kappa * max(m, n) * U64
    Xb, _ = oracle.bs_solve(A, B, C)
    assert relerr(host(X), Xb) <= 50 * kappa * max(m, n) * U64
    # sep estimate from the diagonal forms: min(la) + min(lb) to binary32 accuracy
    assert abs(info["sep_est"] - (la.min() + lb.min())) <= 1e-4 * (la.max() + lb.max())


def test_sym_plain_fp64_path():
    sy = binding()
    A, la, _ = workloads.sym_coeff(31, 150)
    B, lb, _ = workloads.sym_coeff(32, 90)
    C = np.random.RandomState(33).standard_normal((150, 90))
    X, info = sy.solve(dev(A), dev(B), dev(C), low="fp64", alg="sym")
    torch.cuda.synchronize()
    assert info["iterations"] == 0 and info["precision_used"] == "fp64" and info["status"] == 0
    assert info["rel_res"] <= TOL, info
    Xo = oracle.sym_solve(A, B, C)
    assert relerr(host(X), Xo) <= 1e-12


def test_sym_lyapunov_symmetric_solution():
    sy = binding()
    A, la, _ = workloads.sym_coeff(41, 120)
    G = np.random.RandomState(42).standard_normal((120, 4))
    C = G @ G.T
    X, info = sy.lyap(dev(A), dev(C), alg="sym")
    torch.cuda.synchronize()
    assert info["rel_res"] <= TOL and info["fell_back"] == 0, info
    Xh = host(X)
    Xo, _ = oracle.lyap_solve(A, C)
    kappa = la.max() / la.min()
    assert relerr(Xh, Xo) <= 100 * kappa * 120 * U64
    assert np.linalg.norm(Xh - Xh.T) <= 100 * kappa * 120 * U64 * np.linalg.norm(Xh)


def test_sym_rejects_nonsymmetric_coefficients():
    sy = binding()
    A, _, _ = workloads.sym_coeff(51, 30)
    B, _, _ = workloads.sym_coeff(52, 20)
    C = np.random.RandomState(53).standard_normal((30, 20))
    An = A.copy()
    An[0, 1] += 1e-3
    with pytest.raises(sy.SylvError):
        sy.solve(dev(An), dev(B), dev(C), alg="sym")
    Bn = B.copy()
    Bn[3, 0] -= 1e-3
    with pytest.raises(sy.SylvError):
        sy.solve(dev(A), dev(Bn), dev(C), alg="sym")
    # rounding-level asymmetry is accepted
    Ar = A.copy()
    Ar[0, 1] *= 1 + 1e-15
    X, info = sy.solve(dev(Ar), dev(B), dev(C), alg="sym")
    torch.cuda.synchronize()
    assert info["rel_res"] <= TOL


def test_sym_failure_falls_back_to_general_fp64():
    """Eigenvalues of A and -B 1e-9 apart (kappa ~ 1e10, beyond binary32):
    the refinement cannot converge and the general binary64 path answers."""
    sy = binding()
    A, la, QA = workloads.sym_coeff(61, 60)
    B, lb, QB = workloads.sym_coeff(62, 40, lo=-5.0, hi=-0.5)
    # plant lb[0] = -(la[0] - 1e-9)
    lb = lb.copy()
    lb[0] = -la[0] + 1e-9
    B = (QB * lb[None, :]) @ QB.T
    B = 0.5 * (B + B.T)
    C = np.random.RandomState(63).standard_normal((60, 40))
    X, info = sy.solve(dev(A), dev(B), dev(C), alg="sym")
    torch.cuda.synchronize()
    assert info["fell_back"] == 1 and info["precision_used"] == "fp64", info


@pytest.mark.parametrize("dt", ["fp32", "fp64"])
@pytest.mark.parametrize("n,rep", [(40, 13), (300, 60), (700, 200)])
def test_general_schur_on_eigenvalue_cluster(n, rep, dt):
    """The general path's Schur factorisation (small-matrix Francis kernel
    for n = 40, multishift chase + AED above) on symmetric matrices whose
    spectrum holds `rep` equal eigenvalues: no iteration cap, invariants at
    the n u level."""
    sy = binding()
    from gpu_common import check_schur
    say(f"schur cluster n={n} rep={rep} {dt}")
    A, lam, _ = workloads.sym_coeff(800 + n, n, repeated=rep)
    tdt = torch.float32 if dt == "fp32" else torch.float64
    u = U32 if dt == "fp32" else U64
    T, Uq, st = sy.schur(dev(A, tdt))
    torch.cuda.synchronize()
    assert st == 0
    Ar = A.astype(np.float32).astype(np.float64) if dt == "fp32" else A
    check_schur(Ar, host(T), host(Uq), u)


def test_batched_lyapunov_on_eigenvalue_cluster():
    """Batched Lyapunov path (one workgroup per equation) on symmetric
    coefficients with repeated eigenvalues: every equation converges without
    the binary64 fallback."""
    sy = binding()
    eqs, ref = [], []
    for i, (n, rep) in enumerate([(24, 8), (64, 30), (150, 40), (256, 100)]):
        A, lam, _ = workloads.sym_coeff(900 + i, n, lo=-5.0, hi=-0.5, repeated=rep)
        G = np.random.RandomState(950 + i).standard_normal((n, 4))
        C = -G @ G.T
        eqs.append((dev(A), dev(C)))
        ref.append((A, C))
    Xs, infos = sy.solve_batched(eqs)
    torch.cuda.synchronize()
    for (A, C), X, info in zip(ref, Xs, infos):
        assert info["rel_res"] <= TOL and info["fell_back"] == 0, info


@pytest.mark.parametrize("low", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [1, 64, 65, 200, 300])
def test_lyapunov_symmetric_rhs_specialisation(n, low):
    """lyap_solve with a symmetric right-hand side takes the symmetric
    specialisation (one-product residual, mirrored half tri-solve, iterate
    kept exactly symmetric); a general right-hand side of the same equation
    takes the general path.  Both against the oracle."""
    sy = binding()
    say(f"lyap symmetric rhs n={n} {low}")
    A, C, eig = workloads.config4_item(1000 + n, n)
    lam = eig[:, None] + eig[None, :]
    kap = np.abs(lam).max() / np.abs(lam).min()
    for general in (False, True):
        Cc = np.random.RandomState(n).standard_normal((n, n)) if general else C
        X, info = sy.lyap(dev(A), dev(Cc), low=low)
        torch.cuda.synchronize()
        Xh = host(X)
        assert info["rel_res"] <= TOL and info["fell_back"] == 0, info
        Xo, st = oracle.lyap_solve(A, Cc)
        assert st == 0
        assert relerr(Xh, Xo) <= 200 * kap * n * U64 + 1e-15
        if not general:
            assert np.array_equal(Xh, Xh.T)
