"""The paper's flop model in exact rational arithmetic — TEST INFRASTRUCTURE.

Notation: alpha = m^3 + n^3, beta = m n (m + n), gamma = n^3, rho = cost of a
low-precision flop relative to a high-precision one, i = refinement steps.

  Bartels-Stewart (Sec. 2.2.1):   25 alpha + 5 beta   (Lyapunov 35 n^3)
  Hermitian variant (Sec. 2.2.2): 26 n^3 at m = n
  Stationary iteration (Sec. 3.1): 3 k beta  (Lyapunov 6 k n^3)
  Table 4.1: Alg. 4.1 low 25 alpha + beta, high 6 alpha + (4+3i) beta;
             Lyapunov low 27 gamma, high (14 + 6i) gamma.
             Alg. 4.2 low 25 alpha + beta, high (4+2/3) alpha + (4+3i) beta;
             Lyapunov low 27 gamma, high (12 + 2/3 + 6i) gamma.
  Break-even iteration counts, eqs. (5.1)-(5.4).
"""
from __future__ import annotations

from fractions import Fraction as Fr


def bs_sylv(m, n):
    return 25 * (m ** 3 + n ** 3) + 5 * m * n * (m + n)


def bs_lyap(n):
    return 35 * n ** 3


def stationary(m, n, k, lyap=False):
    return 6 * k * n ** 3 if lyap else 3 * k * m * n * (m + n)


def alg41(m, n, i, lyap=False):
    """(low, high) flops of the orthonormalisation-based algorithm."""
    if lyap:
        return 27 * n ** 3, (14 + 6 * i) * n ** 3
    a, b = m ** 3 + n ** 3, m * n * (m + n)
    return 25 * a + b, 6 * a + (4 + 3 * i) * b


def alg42(m, n, i, lyap=False):
    """(low, high) flops of the inversion-based algorithm."""
    if lyap:
        return 27 * n ** 3, (Fr(38, 3) + 6 * i) * n ** 3
    a, b = m ** 3 + n ** 3, m * n * (m + n)
    return 25 * a + b, Fr(14, 3) * a + (4 + 3 * i) * b


def phi_S1(rho, m, n):
    rho = Fr(rho)
    a, b = m ** 3 + n ** 3, m * n * (m + n)
    return ((19 - 25 * rho) * a + (1 - rho) * b) / (3 * b)


def phi_L1(rho):
    return (21 - 27 * Fr(rho)) / 6


def phi_S2(rho, m, n):
    rho = Fr(rho)
    a, b = m ** 3 + n ** 3, m * n * (m + n)
    return ((Fr(61, 3) - 25 * rho) * a + (1 - rho) * b) / (3 * b)


def phi_L2(rho):
    return (Fr(67, 3) - 27 * Fr(rho)) / 6


def cost_ratio(alg, rho, m, n, i, lyap=False):
    """Cost in high-precision-flop equivalents relative to Bartels-Stewart."""
    low, high = (alg41 if alg == 1 else alg42)(m, n, i, lyap)
    bs = bs_lyap(n) if lyap else bs_sylv(m, n)
    return (Fr(rho) * low + high) / bs
