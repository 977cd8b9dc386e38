"""BF16 option: the GEMM-shaped products take bfloat16-rounded inputs on BF16
MFMA with binary32 accumulation; the refinement still reaches the binary64
residual level when the problem is well conditioned (Table 3.1: FP32/BF16
pairs converge for kappa * u_low well below 1), and otherwise the ladder
BF16 -> FP32 -> FP64 takes over."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_common import U64, binding, dev, host, relerr, say

pytestmark = pytest.mark.gpu

TOL = 1e-14
U32 = 2.0 ** -24


def bf16_round(a):
    """Round to bfloat16, nearest even, via binary32 (written from the format's
    definition: keep the top 16 bits of the binary32 pattern)."""
    x = np.ascontiguousarray(a, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (70, 33, 45), (130, 257, 300), (64, 64, 32)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_bf16_gemm_matches_rounded_product(m, n, k, ta, tb):
    sy = binding()
    rs = np.random.RandomState(1000 + m + 3 * n + 7 * k + 11 * ta + 13 * tb)
    A = rs.standard_normal((k, m) if ta else (m, k))
    B = rs.standard_normal((n, k) if tb else (k, n))
    C0 = rs.standard_normal((m, n))
    Ad, Bd = dev(A, torch.float32), dev(B, torch.float32)
    Cd = dev(C0, torch.float32)
    lib = sy.lib()
    import ctypes
    rc = lib.sylv_gemm(2, ta, tb, m, n, k, ctypes.c_double(1.5), ctypes.c_void_p(Ad.data_ptr()),
                       sy._ld(Ad), ctypes.c_void_p(Bd.data_ptr()), sy._ld(Bd), ctypes.c_double(-0.5),
                       ctypes.c_void_p(Cd.data_ptr()), sy._ld(Cd),
                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == 0
    Ar, Br = bf16_round(A), bf16_round(B)
    opA = Ar.T if ta else Ar
    opB = Br.T if tb else Br
    C32 = C0.astype(np.float32).astype(np.float64)
    ref = 1.5 * (opA @ opB) - 0.5 * C32
    bound = (k + 4) * U32 * (1.5 * np.abs(opA) @ np.abs(opB) + 0.5 * np.abs(C32)) + 1e-30
    err = np.abs(host(Cd) - ref)
    assert np.all(err <= bound), (err / bound).max()
    # and it is not the binary32 product of the unrounded operands
    if k >= 32:
        full = 1.5 * ((A.T if ta else A) @ (B.T if tb else B)) - 0.5 * C32
        assert np.abs(host(Cd) - full).max() > 10 * np.abs(host(Cd) - ref).max()


def test_bf16_solve_well_conditioned():
    sy = binding()
    A, B, C = workloads.config1()
    X, info = sy.solve(dev(A), dev(B), dev(C), low="bf16")
    _, info32 = sy.solve(dev(A), dev(B), dev(C), low="fp32")
    torch.cuda.synchronize()
    say("bf16 config1", info)
    assert info["rel_res"] <= TOL and info["fell_back"] == 0, info
    assert info["precision_used"] == "bf16"
    assert info["iterations"] > info32["iterations"]
    Xo, _ = oracle.bs_solve(A, B, C)
    assert relerr(host(X), Xo) <= 1e-12


def test_bf16_escalates_when_sep_is_small():
    """sep(A,-B) = 1e-4 (kappa ~ 1e5): kappa * u_bf16 > 1, so the BF16 forms
    cannot drive the refinement; the ladder must still deliver 1e-14."""
    sy = binding()
    cfg = workloads.config3(3, m=300, n=200)
    X, info = sy.solve(dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"]), low="bf16")
    torch.cuda.synchronize()
    say("bf16 small sep", info)
    assert info["fell_back"] == 1 and info["precision_used"] in ("fp32", "fp64"), info
    assert info["rel_res"] <= TOL
    Xo, _ = oracle.bs_solve(cfg["A"], cfg["B"], cfg["C"])
    assert relerr(host(X), Xo) <= 1e-8


def test_bf16_batched_lyapunov():
    sy = binding()
    sizes = [120, 40, 200, 17]
    its = [workloads.config4_item(950 + i, n) for i, n in enumerate(sizes)]
    Xs, infos = sy.solve_batched([(dev(A), dev(C)) for A, C, _ in its], low="bf16")
    torch.cuda.synchronize()
    for (A, C, eig), X, info in zip(its, Xs, infos):
        say("bf16 batched", A.shape[0], info)
        assert info["rel_res"] <= TOL, info
        assert (info["precision_used"] == "bf16") == (info["fell_back"] == 0)
        Xo, _ = oracle.lyap_solve(A, C)
        lam = eig[:, None] + eig[None, :]
        kap = np.abs(lam).max() / np.abs(lam).min()
        assert relerr(host(X), Xo) <= 100 * U64 * kap
