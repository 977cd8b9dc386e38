"""Orthogonality check of the binary32 Schur vectors (Sec. 2.1: U is
orthogonal to about the low-precision unit roundoff).  orth_check = 2 is
the exact binary64 ||U^T U - I||_F, compared with numpy on the factor
sylv_schur returns for the same matrix (the solve runs the same kernels on
the same input); orth_check = 1 is the randomised probe estimate, which must
agree with the exact value within the spread of an 8-probe trace estimate;
the batched path reports the probe of its own factors."""
import numpy as np
import pytest
import torch

import workloads
from gpu_common import U32, binding, dev, host, say

pytestmark = pytest.mark.gpu


def exact_orth(sy, A):
    _, U, st = sy.schur(dev(A, torch.float32))
    torch.cuda.synchronize()
    assert st == 0
    Uh = host(U)
    return np.linalg.norm(Uh.T @ Uh - np.eye(Uh.shape[0]))


@pytest.mark.parametrize("m,n", [(300, 200), (97, 64)])
def test_orth_full_and_probe_against_numpy(m, n):
    sy = binding()
    A, B, C = workloads.sylv_random(900 + m, m, n, scale=0.5 / np.sqrt(max(m, n)))
    ea, eb = exact_orth(sy, A), exact_orth(sy, B)
    say(f"orth m={m} n={n}: numpy {ea:.3e} {eb:.3e}")
    _, full = sy.solve(dev(A), dev(B), dev(C), orth_check="full")
    _, prb = sy.solve(dev(A), dev(B), dev(C), orth_check="probe")
    _, prb2 = sy.solve(dev(A), dev(B), dev(C), orth_check="probe")
    _, off = sy.solve(dev(A), dev(B), dev(C), orth_check="off")
    torch.cuda.synchronize()
    say(f"  full {full['orth_u']:.3e} {full['orth_v']:.3e}  probe {prb['orth_u']:.3e} {prb['orth_v']:.3e}")
    # exact mode: the binary64 product of the exact binary32 entries
    assert full["orth_u"] == pytest.approx(ea, rel=1e-6)
    assert full["orth_v"] == pytest.approx(eb, rel=1e-6)
    # probe: an unbiased estimate of ||E||_F^2 from 8 sign vectors
    for est, ex in ((prb["orth_u"], ea), (prb["orth_v"], eb)):
        assert 0.25 * ex <= est <= 4.0 * ex, (est, ex)
    assert prb["orth_u"] == prb2["orth_u"] and prb["orth_v"] == prb2["orth_v"]
    assert off["orth_u"] == 0.0 and off["orth_v"] == 0.0
    for inf in (full, prb, off):
        assert inf["status"] == 0 and inf["rel_res"] <= 1e-14


def test_orth_probe_batched():
    """Batched Lyapunov equations report the probe of their own binary32
    factors: of the order of the binary32 orthogonality level (the factor of
    the single-equation Schur form of the same A, within a factor 20), and 0
    with the check off."""
    sy = binding()
    sizes = [200, 64, 17]
    its = [workloads.config4_item(1200 + i, n) for i, n in enumerate(sizes)]
    eqs = [(dev(A), dev(C)) for A, C, _ in its]
    _, infos = sy.solve_batched(eqs)
    _, off = sy.solve_batched(eqs, orth_check="off")
    torch.cuda.synchronize()
    for (A, C, _), inf, o in zip(its, infos, off):
        ex = exact_orth(sy, A)
        n = A.shape[0]
        say(f"batched orth n={n}: probe {inf['orth_u']:.3e} single-equation factor {ex:.3e}")
        assert inf["rel_res"] <= 1e-14
        assert inf["orth_u"] == inf["orth_v"]
        assert 0.0 < inf["orth_u"] <= 10 * n * U32
        assert ex / 20 <= inf["orth_u"] <= 20 * ex
        assert o["orth_u"] == 0.0
