"""Seeded synthetic inputs for the Sylvester / Lyapunov workloads.

This module only draws random numbers and assembles coefficient matrices
with a prescribed spectrum; it contains none of the solver's arithmetic.
Both the GPU path and the CPU oracle read their inputs from here.

All matrices are returned as column-major (Fortran-ordered) float64 numpy
arrays.  Every generator uses numpy's legacy ``RandomState`` whose stream is
frozen, so a given seed always yields the same data.

Recipes (readings of the workload descriptions are marked in the design doc):

* ``config1``  m=n=64, A=G1/8+2I, B=G2/8+2I, C=G3, G_i iid N(0,1), seed 1.
* ``normal_coeff``  Q D Q^T with Q Haar-orthogonal (QR of a Gaussian matrix,
  signs of diag(R) folded into Q) and D block diagonal: real eigenvalues and
  2x2 blocks [[a, w], [-w, a]] (complex pair a +- i w), in random order.
* ``config2``  m=n=2048, real parts U[0.5, 5], 30% of eigenvalues in complex
  pairs with w ~ U[0.5, 5]; C ~ N(0,1).  Seeds 2 (A), 3 (B), 4 (C).
* ``config3``  m=4096, n=1024, same construction; one real eigenvalue 0.5
  planted in each spectrum, then A <- A + (delta-1) I so that
  min |lambda_i(A) + mu_j(B)| = delta exactly.
* ``config4``  batched Lyapunov, sizes U{16..256}, Re(eig) in U[-5, -0.1],
  30% complex pairs, C = -B B^T with B n x 4 Gaussian.
* ``sym_coeff``  symmetric Q diag(lam) Q^T, Q Haar, lam ~ U[lo, hi] (the
  real-part range of ``config2``), optionally with a repeated eigenvalue;
  ``config_sym`` m=n=2048, lam in U[0.5, 5], seeds 12 (A), 13 (B), 14 (C).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "haar_orthogonal", "block_spectrum", "normal_coeff", "config1", "config2",
    "config3", "config4_sizes", "config4_item", "sylv_random", "manufactured",
    "config2_nonnormal", "sym_coeff", "config_sym",
]


def _f(a):
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def haar_orthogonal(rs: np.random.RandomState, n: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix (Mezzadri 2007): QR of a Gaussian
    matrix with the signs of diag(R) folded into Q."""
    g = rs.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def block_spectrum(rs, n, re_lo, re_hi, frac_complex=0.30, w_lo=0.5, w_hi=5.0,
                   planted=None):
    """Block-diagonal D (n x n) and its eigenvalues.

    floor(frac_complex * n / 2) 2x2 blocks [[a, w], [-w, a]] with a ~ U[re_lo,
    re_hi], w ~ U[w_lo, w_hi]; the remaining eigenvalues are real ~ U[re_lo,
    re_hi].  ``planted`` (a real value) replaces one real eigenvalue.  The
    blocks are placed in random order.  Returns (D, eigenvalues as complex).
    """
    npair = int(np.floor(frac_complex * n / 2.0))
    nreal = n - 2 * npair
    reals = rs.uniform(re_lo, re_hi, size=nreal)
    if planted is not None and nreal > 0:
        reals[0] = planted
    pa = rs.uniform(re_lo, re_hi, size=npair)
    pw = rs.uniform(w_lo, w_hi, size=npair)
    blocks = [("r", x) for x in reals] + [("c", (a, w)) for a, w in zip(pa, pw)]
    order = rs.permutation(len(blocks))
    D = np.zeros((n, n))
    eig = []
    i = 0
    for k in order:
        kind, val = blocks[k]
        if kind == "r":
            D[i, i] = val
            eig.append(complex(val, 0.0))
            i += 1
        else:
            a, w = val
            D[i, i] = a
            D[i + 1, i + 1] = a
            D[i, i + 1] = w
            D[i + 1, i] = -w
            eig.extend([complex(a, w), complex(a, -w)])
            i += 2
    return D, np.array(eig)


def normal_coeff(seed, n, re_lo, re_hi, frac_complex=0.30, planted=None,
                 shift=0.0, eta=0.0):
    """A = Q (D + eta*N) Q^T + shift*I with Q Haar, D from ``block_spectrum``
    and N strictly block-upper Gaussian (only when eta != 0).

    Returns (A, eigenvalues, Q, D_total) where D_total = D + eta*N + shift*I.
    """
    rs = np.random.RandomState(seed)
    D, eig = block_spectrum(rs, n, re_lo, re_hi, frac_complex, planted=planted)
    Q = haar_orthogonal(rs, n)
    if eta != 0.0:
        N = rs.standard_normal((n, n))
        # strictly block-upper: zero the diagonal blocks and everything below
        mask = np.triu(np.ones((n, n)), 1).astype(bool)
        for i in range(n - 1):
            if D[i + 1, i] != 0.0:      # inside a 2x2 block: keep it intact
                mask[i, i + 1] = False
        D = D + eta * N * mask
    D = D + shift * np.eye(n)
    A = Q @ D @ Q.T
    return _f(A), eig + shift, _f(Q), _f(D)


def config1(seed: int = 1, m: int = 64, n: int = 64):
    """A=G1/8+2I, B=G2/8+2I, C=G3 with G1, G2, G3 drawn in this order."""
    rs = np.random.RandomState(seed)
    g1 = rs.standard_normal((m, m))
    g2 = rs.standard_normal((n, n))
    g3 = rs.standard_normal((m, n))
    A = g1 / 8.0 + 2.0 * np.eye(m)
    B = g2 / 8.0 + 2.0 * np.eye(n)
    return _f(A), _f(B), _f(g3)


def config2(m: int = 2048, n: int = 2048, seeds=(2, 3, 4)):
    """Normal coefficients with Re(eig) ~ U[0.5, 5], 30% complex pairs."""
    A, ea, QA, DA = normal_coeff(seeds[0], m, 0.5, 5.0)
    B, eb, QB, DB = normal_coeff(seeds[1], n, 0.5, 5.0)
    C = np.random.RandomState(seeds[2]).standard_normal((m, n))
    return dict(A=A, B=B, C=_f(C), eigA=ea, eigB=eb, QA=QA, QB=QB, DA=DA, DB=DB)


def config2_nonnormal(m: int = 2048, n: int = 2048, seeds=(2, 3, 4)):
    """Non-normal twin of config 2: D + eta*N with eta = 1/sqrt(n)."""
    A, ea, QA, DA = normal_coeff(seeds[0], m, 0.5, 5.0, eta=1.0 / np.sqrt(m))
    B, eb, QB, DB = normal_coeff(seeds[1], n, 0.5, 5.0, eta=1.0 / np.sqrt(n))
    C = np.random.RandomState(seeds[2]).standard_normal((m, n))
    return dict(A=A, B=B, C=_f(C), eigA=ea, eigB=eb, QA=QA, QB=QB, DA=DA, DB=DB)


def config3(j: int, m: int = 4096, n: int = 1024):
    """sep sweep: delta = 10**-(j+1), j = 0..5, seeds 10+j (A), 10+j+100 (B),
    10+j+200 (C).  One real eigenvalue 0.5 is planted in each spectrum and A
    is shifted by (delta - 1) I, so min |lambda + mu| = delta."""
    delta = 10.0 ** (-(j + 1))
    s = 10 + j
    A, ea, QA, DA = normal_coeff(s, m, 0.5, 5.0, planted=0.5, shift=delta - 1.0)
    B, eb, QB, DB = normal_coeff(s + 100, n, 0.5, 5.0, planted=0.5)
    C = np.random.RandomState(s + 200).standard_normal((m, n))
    return dict(A=A, B=B, C=_f(C), eigA=ea, eigB=eb, QA=QA, QB=QB, DA=DA,
                DB=DB, delta=delta)


def config4_sizes(count: int = 4096, lo: int = 16, hi: int = 256,
                  seed: int = 99999):
    """Equation orders n_i ~ U{lo..hi} (inclusive)."""
    return np.random.RandomState(seed).randint(lo, hi + 1, size=count)


def config4_item(i: int, n: int, nrhs: int = 4):
    """Stable A = Q D Q^T (Re(eig) ~ U[-5, -0.1], 30% complex pairs) and
    C = -B B^T with B n x nrhs Gaussian; seed 100000 + i."""
    rs = np.random.RandomState(100000 + i)
    D, eig = block_spectrum(rs, n, -5.0, -0.1)
    Q = haar_orthogonal(rs, n)
    Bf = rs.standard_normal((n, nrhs))
    A = Q @ D @ Q.T
    C = -(Bf @ Bf.T)
    return _f(A), _f(C), eig


def sylv_random(seed, m, n, shift=2.0, scale=0.125):
    """Generic well-conditioned non-normal Sylvester instance (config 1
    recipe at any shape)."""
    rs = np.random.RandomState(seed)
    A = rs.standard_normal((m, m)) * scale + shift * np.eye(m)
    B = rs.standard_normal((n, n)) * scale + shift * np.eye(n)
    C = rs.standard_normal((m, n))
    return _f(A), _f(B), _f(C)


def manufactured(seed, m, n):
    """A, B and a known solution X* (the right-hand side is formed by the
    caller in the precision it needs)."""
    rs = np.random.RandomState(seed)
    A = rs.standard_normal((m, m)) * 0.125 + 2.0 * np.eye(m)
    B = rs.standard_normal((n, n)) * 0.125 + 2.0 * np.eye(n)
    X = rs.standard_normal((m, n))
    return _f(A), _f(B), _f(X)


def selector_sizes(i: int, lo: int = 32, hi: int = 1024, seed_base: int = 200000):
    """Orders of selector instance i: m, n independently log-uniform integers
    in [lo, hi]; sep target delta log-uniform in [1e-8, 1e-1]; 10% of the
    instances are Lyapunov (then n = m)."""
    rs = np.random.RandomState(seed_base + i)
    m = int(round(np.exp(rs.uniform(np.log(lo), np.log(hi)))))
    n = int(round(np.exp(rs.uniform(np.log(lo), np.log(hi)))))
    delta = float(10.0 ** rs.uniform(-8.0, -1.0))
    lyap = bool(rs.uniform() < 0.10)
    return m, (m if lyap else n), delta, lyap


def selector_instance(i: int, lo: int = 32, hi: int = 1024, seed_base: int = 200000):
    """Instance i of the selector recipe (config-3 construction at the drawn
    sizes and sep).  Sylvester: A = Q_A D_A Q_A^T + (delta - 1) I and B with
    planted eigenvalue 0.5, so min |l + m| = delta.  Lyapunov: A with Re(eig)
    in [0.5, 5] and a planted eigenvalue delta/2 (min |l_i + l_j| = delta).
    Returns dict(A, B (None for Lyapunov), C, delta, lyap)."""
    m, n, delta, lyap = selector_sizes(i, lo, hi, seed_base)
    s = seed_base + i
    if lyap:
        A, ea, _, _ = normal_coeff(s + 1, m, 0.5, 5.0, planted=0.5, shift=delta / 2 - 0.5)
        C = np.random.RandomState(s + 3).standard_normal((m, m))
        C = C + C.T
        return dict(A=A, B=None, C=_f(C), delta=delta, lyap=True, eigA=ea)
    A, ea, _, _ = normal_coeff(s + 1, m, 0.5, 5.0, planted=0.5, shift=delta - 1.0)
    B, eb, _, _ = normal_coeff(s + 2, n, 0.5, 5.0, planted=0.5)
    C = np.random.RandomState(s + 3).standard_normal((m, n))
    return dict(A=A, B=B, C=_f(C), delta=delta, lyap=False, eigA=ea, eigB=eb)


def selector_lyap_mix(i: int, lo: int = 16, hi: int = 256, seed_base: int = 400000):
    """Equation i of the batched evaluation mix: a Lyapunov equation of order
    n uniform in [lo, hi], sep target delta log-uniform in [1e-8, 1e-1], the
    Lyapunov construction of selector_instance (Re(eig) in [0.5, 5] with a
    planted eigenvalue delta/2, C = G + G^T)."""
    rs = np.random.RandomState(seed_base + i)
    n = int(rs.randint(lo, hi + 1))
    delta = float(10.0 ** rs.uniform(-8.0, -1.0))
    s = seed_base + i
    A, ea, _, _ = normal_coeff(s + 1, n, 0.5, 5.0, planted=0.5, shift=delta / 2 - 0.5)
    G = np.random.RandomState(s + 3).standard_normal((n, n))
    return dict(A=A, C=_f(G + G.T), delta=delta, n=n, eigA=ea)


def sym_coeff(seed, n, lo=0.5, hi=5.0, repeated=0, rep_value=None):
    """Symmetric A = Q diag(lam) Q^T, Q Haar, lam ~ U[lo, hi] in random
    order; the first ``repeated`` entries of lam equal ``rep_value`` (default
    the middle of the range), a cluster of identical eigenvalues.  A is
    symmetrised exactly ((A + A^T)/2).  Returns (A, lam, Q)."""
    rs = np.random.RandomState(seed)
    lam = rs.uniform(lo, hi, n)
    if repeated:
        lam[:repeated] = 0.5 * (lo + hi) if rep_value is None else rep_value
    Q = haar_orthogonal(rs, n)
    A = (Q * lam[None, :]) @ Q.T
    A = 0.5 * (A + A.T)
    return _f(A), lam, _f(Q)


def config_sym(m: int = 2048, n: int = 2048, seeds=(12, 13, 14)):
    """Symmetric-coefficient Sylvester workload: A, B from ``sym_coeff`` with
    eigenvalues U[0.5, 5], C ~ N(0, 1)."""
    A, la, QA = sym_coeff(seeds[0], m)
    B, lb, QB = sym_coeff(seeds[1], n)
    C = np.random.RandomState(seeds[2]).standard_normal((m, n))
    return dict(A=A, B=B, C=_f(C), eigA=la, eigB=lb, QA=QA, QB=QB)
