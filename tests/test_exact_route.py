"""Pin the vectorised block-diagonal reference against the C oracle (Kronecker
route at small size) so it can stand in at large sizes."""
import numpy as np

import oracle
import workloads
from exact_route import exact_solution, solve_block_diagonal


def test_block_diagonal_solver_vs_kronecker():
    rs = np.random.RandomState(3)
    _, ea, QA, DA = workloads.normal_coeff(11, 9, 0.5, 5.0)
    _, eb, QB, DB = workloads.normal_coeff(12, 7, 0.5, 5.0)
    Ct = rs.standard_normal((9, 7))
    Y = solve_block_diagonal(DA, DB, Ct)
    M = np.kron(np.eye(7), DA) + np.kron(DB.T, np.eye(9))
    Yk = np.linalg.solve(M, Ct.ravel(order="F")).reshape((9, 7), order="F")
    assert np.linalg.norm(Y - Yk) <= 1e-13 * np.linalg.norm(Yk)


def test_exact_route_matches_oracle_bs():
    cfg = workloads.config2(m=60, n=45)
    X = exact_solution(cfg)
    Xo, st = oracle.bs_solve(cfg["A"], cfg["B"], cfg["C"])
    assert st == 0
    assert np.linalg.norm(X - Xo) <= 1e-13 * np.linalg.norm(Xo)
    assert oracle.rel_residual(cfg["A"], cfg["B"], cfg["C"], X) <= 1e-15


def test_exact_route_config3_small():
    cfg = workloads.config3(2, m=40, n=20)
    X = exact_solution(cfg)
    Xo, _ = oracle.bs_solve(cfg["A"], cfg["B"], cfg["C"])
    kappa = 13.5 / cfg["delta"]
    assert np.linalg.norm(X - Xo) <= 100 * 2.0 ** -53 * kappa * 10 * np.linalg.norm(Xo)
