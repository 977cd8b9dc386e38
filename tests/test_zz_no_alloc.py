"""sylv_solve_noalloc (workspace in the library's static device scratch, no
allocation) against sylv_solve (the same kernels with a caller workspace) on
the same equations: two calls in a row, the second smaller, each bit-equal to
sylv_solve and at the tolerance against the FP64 oracle; a problem beyond
the scratch is refused with SYLV_ERR_SCRATCH before any device work."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_common import U64, binding, dev, host, relerr, say

pytestmark = pytest.mark.gpu

TOL = 1e-14
SYLV_ERR_SCRATCH = -2000


def kappa_est(A, B):
    lam = np.abs(np.linalg.eigvals(A)[:, None] + np.linalg.eigvals(B)[None, :])
    return lam.max() / lam.min()


def test_noalloc_matches_sylv_solve_two_calls():
    sy = binding()
    sy.init()
    for seed, (m, n) in ((31, (300, 257)), (32, (90, 61))):
        say(f"noalloc m={m} n={n}")
        A, B, C = workloads.sylv_random(seed, m, n, scale=0.5 / np.sqrt(max(m, n)))
        dA, dB, dC = dev(A), dev(B), dev(C)
        X0, i0 = sy.solve(dA, dB, dC)
        X1 = torch.full((n, m), np.nan, dtype=torch.float64, device="cuda").t()
        X1, i1 = sy.solve_noalloc(dA, dB, dC, X1)
        torch.cuda.synchronize()
        x0, x1 = host(X0), host(X1)
        assert i1["status"] == 0 and i1["fell_back"] == 0 and i1["rel_res"] <= TOL, i1
        assert i1["iterations"] == i0["iterations"] and i1["rel_res"] == i0["rel_res"], (i0, i1)
        # same kernels on the same inputs: the same bits
        assert np.array_equal(x1, x0)
        Xo, st = oracle.bs_solve(A, B, C)
        assert st == 0
        assert relerr(x1, Xo) <= 100 * U64 * kappa_est(A, B)


def test_noalloc_refuses_problem_beyond_scratch():
    sy = binding()
    sy.init()
    A = torch.eye(640, dtype=torch.float64, device="cuda")
    X = torch.empty((640, 640), dtype=torch.float64, device="cuda").t()
    with pytest.raises(sy.SylvError) as e:
        sy.solve_noalloc(A, A, A, X)
    assert f"code {SYLV_ERR_SCRATCH}" in str(e.value)
