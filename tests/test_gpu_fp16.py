"""FP16 option (Table 2.1's binary16): the GEMM-shaped products take
binary16-rounded operands on FP16 MFMA with binary32 accumulation, every
operand brought into binary16 range by an exact power of two; the
refinement reaches the binary64 residual level for well-conditioned
problems and escalates otherwise.  Also the power-of-two scaling of the
right-hand side in the binary32 path (C scaled by 2^127 or 2^-130 converges as the
unscaled C does)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_common import U64, binding, dev, host, relerr, say

pytestmark = pytest.mark.gpu

TOL = 1e-14
U16 = 2.0 ** -11
U32 = 2.0 ** -24


def kron_cond(A, B):
    m, n = A.shape[0], B.shape[0]
    return np.linalg.cond(np.kron(np.eye(n), A) + np.kron(B.T, np.eye(m)))


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (70, 33, 45), (130, 257, 300)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1)])
def test_fp16_gemm_matches_rounded_product(m, n, k, ta, tb):
    sy = binding()
    rs = np.random.RandomState(2000 + m + 3 * n + 7 * k + 11 * ta)
    A = rs.standard_normal((k, m) if ta else (m, k))
    B = rs.standard_normal((n, k) if tb else (k, n))
    C0 = rs.standard_normal((m, n))
    Ad, Bd, Cd = dev(A, torch.float32), dev(B, torch.float32), dev(C0, torch.float32)
    rc = sy.lib().sylv_gemm(3, ta, tb, m, n, k, ctypes.c_double(1.5), ctypes.c_void_p(Ad.data_ptr()),
                            sy._ld(Ad), ctypes.c_void_p(Bd.data_ptr()), sy._ld(Bd), ctypes.c_double(-0.5),
                            ctypes.c_void_p(Cd.data_ptr()), sy._ld(Cd),
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == 0
    # binary16 rounding of the binary32 operands (numpy's conversion rounds to nearest even)
    Ar = A.astype(np.float32).astype(np.float16).astype(np.float64)
    Br = B.astype(np.float32).astype(np.float16).astype(np.float64)
    opA, opB = (Ar.T if ta else Ar), (Br.T if tb else Br)
    C32 = C0.astype(np.float32).astype(np.float64)
    ref = 1.5 * (opA @ opB) - 0.5 * C32
    bound = (k + 4) * U32 * (1.5 * np.abs(opA) @ np.abs(opB) + 0.5 * np.abs(C32)) + 1e-30
    assert np.all(np.abs(host(Cd) - ref) <= bound)
    if k >= 32:
        full = 1.5 * ((A.T if ta else A) @ (B.T if tb else B)) - 0.5 * C32
        assert np.abs(host(Cd) - full).max() > 10 * np.abs(host(Cd) - ref).max()


def test_fp16_solve_well_conditioned():
    sy = binding()
    A, B, C = workloads.config1()
    X, info = sy.solve(dev(A), dev(B), dev(C), low="fp16")
    torch.cuda.synchronize()
    say("fp16 config1", info)
    assert info["status"] == 0 and info["rel_res"] <= TOL, info
    assert info["precision_used"] == "fp16" and info["fell_back"] == 0
    Xo, _ = oracle.bs_solve(A, B, C)
    assert relerr(host(X), Xo) <= 100 * U64 * kron_cond(A, B)


@pytest.mark.parametrize("e", [20, -20])
def test_fp16_range_scaling(e):
    """A, B, C scaled by 2^e (same X): entries far outside binary16's range
    (2^20 * 2 > 65504; 2^-20 below its normal range), yet the binary16 path
    converges in about the iterations of the unscaled problem."""
    sy = binding()
    A, B, C = workloads.config1()
    s = 2.0 ** e
    _, i0 = sy.solve(dev(A), dev(B), dev(C), low="fp16")
    X, i1 = sy.solve(dev(s * A), dev(s * B), dev(s * C), low="fp16")
    torch.cuda.synchronize()
    say(f"fp16 scaled 2^{e}", i0["iterations"], i1["iterations"], i1["rel_res"])
    assert i1["status"] == 0 and i1["rel_res"] <= TOL and i1["precision_used"] == "fp16", i1
    assert abs(i1["iterations"] - i0["iterations"]) <= 1
    Xo, _ = oracle.bs_solve(A, B, C)
    assert relerr(host(X), Xo) <= 100 * U64 * kron_cond(A, B)


@pytest.mark.parametrize("e", [127, -130])
def test_fp32_rhs_power_of_two_scaling(e):
    """C scaled by 2^127 or 2^-130 (binary32 overflow or underflow of an unscaled
    cast): the binary32 path takes the same corrections as for C."""
    sy = binding()
    A, B, C = workloads.config1()
    _, i0 = sy.solve(dev(A), dev(B), dev(C), low="fp32")
    X, i1 = sy.solve(dev(A), dev(B), dev(2.0 ** e * C), low="fp32")
    torch.cuda.synchronize()
    say(f"fp32 rhs 2^{e}", i0["iterations"], i1["iterations"], i1["rel_res"])
    assert i1["status"] == 0 and i1["fell_back"] == 0 and i1["rel_res"] <= TOL, i1
    assert i1["iterations"] == i0["iterations"]
    Xo, _ = oracle.bs_solve(A, B, C)
    assert relerr(2.0 ** -e * host(X), Xo) <= 100 * U64 * kron_cond(A, B)


def test_fp16_escalates_when_sep_is_small():
    """sep(A,-B) = 1e-4: kappa * u_16 >> 1, so the binary16-update forms
    cannot converge; the ladder FP16 -> FP32 (-> FP64) answers."""
    sy = binding()
    cfg = workloads.config3(3, m=300, n=120)
    X, info = sy.solve(dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"]), low="fp16")
    torch.cuda.synchronize()
    say("fp16 small sep", info)
    assert info["rel_res"] <= TOL and info["fell_back"] == 1, info
    assert info["precision_used"] in ("fp32", "fp64")


def test_fp16_batched_lyapunov():
    sy = binding()
    sizes = [120, 40, 200, 17]
    its = [workloads.config4_item(1950 + i, n) for i, n in enumerate(sizes)]
    Xs, infos = sy.solve_batched([(dev(A), dev(C)) for A, C, _ in its], low="fp16")
    torch.cuda.synchronize()
    for (A, C, eig), X, info in zip(its, Xs, infos):
        say("fp16 batched", A.shape[0], info)
        assert info["rel_res"] <= TOL, info
        assert (info["precision_used"] == "fp16") == (info["fell_back"] == 0)
        Xo, _ = oracle.lyap_solve(A, C)
        lam = eig[:, None] + eig[None, :]
        kap = np.abs(lam).max() / np.abs(lam).min()
        assert relerr(host(X), Xo) <= 100 * U64 * kap
