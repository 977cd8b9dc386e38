"""Pins of the relative residual of eq. (2.1) (Frobenius norms, as in the
experiments of Sec. 7):

    rel_res = ||A X + X B - C||_F / (||C||_F + ||X||_F (||A||_F + ||B||_F)),

with B = A^T for the Lyapunov equation (1.3).  Every expected value below is
worked out by hand from integer matrices (the residual entries are written
out as literals), so a dropped term, a transposed operand, a swapped product
order or a different norm in the oracle fails at least one test."""
import math

import numpy as np
import pytest

import oracle

A2 = np.array([[1.0, 2.0], [3.0, 4.0]])
B2 = np.array([[0.0, 1.0], [5.0, 0.0]])
X2 = np.array([[1.0, 2.0], [0.0, 1.0]])
C2 = np.array([[1.0, 1.0], [1.0, 1.0]])


def test_zero_iterate_gives_exactly_one():
    # X = 0: the residual is -C and the denominator is ||C||_F.
    rs = np.random.RandomState(5)
    for m, n in [(1, 1), (3, 5), (6, 2)]:
        A, B, C = rs.standard_normal((m, m)), rs.standard_normal((n, n)), rs.standard_normal((m, n))
        assert oracle.rel_residual(A, B, C, np.zeros((m, n))) == 1.0
    A, C = rs.standard_normal((4, 4)), rs.standard_normal((4, 4))
    assert oracle.rel_residual(A, None, C, np.zeros((4, 4)), lyap=True) == 1.0


def test_sylvester_integer_case_by_hand():
    # A X = [[1, 4], [3, 10]],  X B = [[10, 1], [5, 0]],
    # R = A X + X B - C = [[10, 4], [7, 9]]  ->  ||R||_F^2 = 246;
    # ||C||_F = 2, ||X||_F^2 = 6, ||A||_F^2 = 30, ||B||_F^2 = 26.
    want = math.sqrt(246.0) / (2.0 + math.sqrt(6.0) * (math.sqrt(30.0) + math.sqrt(26.0)))
    got = oracle.rel_residual(A2, B2, C2, X2)
    assert abs(got - want) <= 4e-16 * want


def test_sylvester_case_is_sensitive_to_operand_order():
    # The same data with B X (instead of X B) or X B^T would give
    #   B X = [[0, 1], [5, 10]]  -> R = [[0, 4], [7, 19]], ||R||^2 = 426
    #   X B^T = [[2, 5], [1, 0]] -> R = [[2, 8], [3, 9]],  ||R||^2 = 158
    # neither of which is what the oracle returns.
    got = oracle.rel_residual(A2, B2, C2, X2)
    den = 2.0 + math.sqrt(6.0) * (math.sqrt(30.0) + math.sqrt(26.0))
    for wrong in (426.0, 158.0):
        assert abs(got - math.sqrt(wrong) / den) > 1e-3


def test_lyapunov_integer_case_by_hand():
    # X A^T = [[5, 11], [2, 4]], R = A X + X A^T - C = [[5, 14], [4, 13]]
    # -> ||R||_F^2 = 406; denominator ||C||_F + ||X||_F (||A||_F + ||A^T||_F).
    want = math.sqrt(406.0) / (2.0 + math.sqrt(6.0) * 2.0 * math.sqrt(30.0))
    got = oracle.rel_residual(A2, None, C2, X2, lyap=True)
    assert abs(got - want) <= 4e-16 * want
    # X A (the wrong right coefficient) = [[7, 10], [3, 4]] -> R = [[7, 13], [5, 13]],
    # ||R||^2 = 412.
    assert abs(got - math.sqrt(412.0) / (2.0 + math.sqrt(6.0) * 2.0 * math.sqrt(30.0))) > 1e-3


def test_lyapunov_equals_sylvester_with_transposed_coefficient():
    rs = np.random.RandomState(11)
    A = rs.standard_normal((7, 7))
    X = rs.standard_normal((7, 7))
    C = rs.standard_normal((7, 7))
    ly = oracle.rel_residual(A, None, C, X, lyap=True)
    assert ly == pytest.approx(oracle.rel_residual(A, np.ascontiguousarray(A.T), C, X), rel=1e-14)
    # for a nonsymmetric A, B = A is a different equation
    assert abs(ly - oracle.rel_residual(A, A, C, X)) > 1e-3 * ly


@pytest.mark.parametrize("s", [2.0 ** -30, 0.37, 3.0, 2.0 ** 40])
def test_invariant_under_common_scaling_of_coefficients(s):
    # (A, B, C, X) -> (sA, sB, sC, X) scales the residual and the denominator
    # by |s|.
    rs = np.random.RandomState(3)
    A, B = rs.standard_normal((5, 5)), rs.standard_normal((4, 4))
    C, X = rs.standard_normal((5, 4)), rs.standard_normal((5, 4))
    r0 = oracle.rel_residual(A, B, C, X)
    assert oracle.rel_residual(s * A, s * B, s * C, X) == pytest.approx(r0, rel=1e-13)


def test_exact_solution_of_diagonal_equation_has_zero_residual():
    # A, B diagonal and C_ij = a_i + b_j, so X = C ./ (a_i + b_j) is all ones,
    # exactly, and the residual is exactly zero.
    a = np.array([1.0, 3.0, 7.0])
    b = np.array([1.0, 5.0])
    C = np.array([[2.0, 6.0], [4.0, 8.0], [8.0, 12.0]])
    X = C / (a[:, None] + b[None, :])
    assert oracle.rel_residual(np.diag(a), np.diag(b), C, X) == 0.0
