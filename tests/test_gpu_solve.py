"""End-to-end parity of sylv_solve / lyap_solve on the GPU against the FP64
oracle (and, at the workload's full sizes, against the independent
block-diagonal route and the binary64 residual property)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from exact_route import exact_solution
from gpu_common import U64, binding, dev, host, relerr, say

pytestmark = pytest.mark.gpu

TOL = 1e-14


def kron_cond(A, B):
    m, n = A.shape[0], B.shape[0]
    M = np.kron(np.eye(n), A) + np.kron(B.T, np.eye(m))
    return np.linalg.cond(M)


@pytest.mark.parametrize("low", ["fp64", "fp32"])
def test_config1_sylvester(low):
    sy = binding()
    say("config1", low)
    A, B, C = workloads.config1()
    X, info = sy.solve(dev(A), dev(B), dev(C), low=low)
    torch.cuda.synchronize()
    Xg = host(X)
    Xo, st = oracle.bs_solve(A, B, C)
    assert st == 0
    assert info["status"] == 0, info
    assert info["rel_res"] <= TOL, info
    assert oracle.rel_residual(A, B, C, Xg) <= max(TOL, 10 * oracle.rel_residual(A, B, C, Xo))
    assert relerr(Xg, Xo) <= 100 * U64 * kron_cond(A, B)
    if low == "fp32":
        assert info["fell_back"] == 0 and info["iterations"] >= 1
        assert info["orth_u"] < 1e-4 and info["orth_v"] < 1e-4


@pytest.mark.parametrize("low", ["fp64", "fp32"])
@pytest.mark.parametrize("m,n", [(1, 1), (1, 7), (9, 1), (2, 2), (33, 17), (150, 90), (301, 257)])
def test_sylvester_shapes(low, m, n):
    sy = binding()
    say("sylv shapes", low, m, n)
    # spectra kept in discs of radius ~0.5 around 2 (|lambda + mu| >= ~3),
    # so the Sylvester operator is well conditioned at every shape
    A, B, C = workloads.sylv_random(500 + m + n, m, n, scale=0.5 / np.sqrt(max(m, n)))
    X, info = sy.solve(dev(A), dev(B), dev(C), low=low)
    torch.cuda.synchronize()
    Xg = host(X)
    Xo, _ = oracle.bs_solve(A, B, C)
    assert info["rel_res"] <= TOL, info
    assert oracle.rel_residual(A, B, C, Xg) <= TOL
    kap = kron_cond(A, B) if m * n <= 2500 else 10.0
    assert relerr(Xg, Xo) <= 100 * U64 * kap * max(1.0, np.sqrt(m + n) / 8)


@pytest.mark.parametrize("low", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [16, 100, 256])
def test_lyapunov_config4_items(low, n):
    sy = binding()
    say("lyap", low, n)
    A, C, eig = workloads.config4_item(n, n)
    X, info = sy.lyap(dev(A), dev(C), low=low)
    torch.cuda.synchronize()
    Xg = host(X)
    Xo, _ = oracle.lyap_solve(A, C)
    assert info["rel_res"] <= TOL, info
    lam = eig[:, None] + eig[None, :]
    kappa = np.abs(lam).max() / np.abs(lam).min()
    assert relerr(Xg, Xo) <= 100 * U64 * kappa
    assert np.linalg.norm(Xg - Xg.T) <= 100 * U64 * kappa * np.linalg.norm(Xg)


def test_nonnormal_twin_medium():
    sy = binding()
    cfg = workloads.config2_nonnormal(m=400, n=300)
    X, info = sy.solve(dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"]), low="fp32")
    torch.cuda.synchronize()
    Xo, _ = oracle.bs_solve(cfg["A"], cfg["B"], cfg["C"])
    assert info["rel_res"] <= TOL and info["fell_back"] == 0, info
    assert relerr(host(X), Xo) <= 1e-12


def test_info_reports_sep_estimate():
    sy = binding()
    cfg = workloads.config3(1, m=300, n=200)   # delta = 1e-2
    X, info = sy.solve(dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"]), low="fp32")
    torch.cuda.synchronize()
    assert abs(info["sep_est"] - cfg["delta"]) <= 1e-4 + 1e-3 * cfg["delta"] * 100
    assert info["rel_res"] <= TOL
    Xe = exact_solution(cfg)
    assert relerr(host(X), Xe) <= 100 * U64 * 13.5 / cfg["delta"] * 10


def test_fallback_path_when_no_iterations_allowed():
    """max_iter = 0: the binary32 first iterate cannot meet 1e-14, so the
    binary64 path must take over (fell_back = 1)."""
    sy = binding()
    A, B, C = workloads.sylv_random(9, 80, 60)
    X, info = sy.solve(dev(A), dev(B), dev(C), low="fp32", max_iter=0)
    torch.cuda.synchronize()
    assert info["fell_back"] == 1 and info["precision_used"] == "fp64"
    assert info["rel_res"] <= TOL
    X2, info2 = sy.solve(dev(A), dev(B), dev(C), low="fp32", max_iter=0, fallback=False)
    torch.cuda.synchronize()
    assert info2["fell_back"] == 0 and info2["status"] == 2


def test_nan_input_reports_status():
    sy = binding()
    A, B, C = workloads.sylv_random(10, 30, 20)
    C[3, 4] = np.nan
    X, info = sy.solve(dev(A), dev(B), dev(C), low="fp32", fallback=False)
    torch.cuda.synchronize()
    assert info["status"] == 3


def test_determinism():
    sy = binding()
    A, B, C = workloads.sylv_random(12, 200, 150)
    X1, _ = sy.solve(dev(A), dev(B), dev(C), low="fp32")
    X2, _ = sy.solve(dev(A), dev(B), dev(C), low="fp32")
    torch.cuda.synchronize()
    assert torch.equal(X1, X2)


def test_caller_workspace():
    sy = binding()
    A, B, C = workloads.sylv_random(13, 70, 50)
    nbytes = sy.workspace_size(70, 50)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    X, info = sy.solve(dev(A), dev(B), dev(C), work=work)
    torch.cuda.synchronize()
    assert info["rel_res"] <= TOL
    small = torch.empty(nbytes // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(sy.SylvError):
        sy.solve(dev(A), dev(B), dev(C), work=small)


def test_info_in_device_memory():
    """sylv_info may be a device array: the solve fills it by a copy on its
    stream (single and batched calls)."""
    import ctypes
    sy = binding()
    A, B, C = workloads.sylv_random(61, 50, 40)
    dA, dB, dC = dev(A), dev(B), dev(C)
    X = torch.empty((40, 50), dtype=torch.float64, device="cuda").t()
    nbytes = ctypes.sizeof(sy.Info)
    dinfo = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    o = sy.make_opts()
    rc = sy.lib().sylv_solve(50, 40, dA.data_ptr(), sy._ld(dA), dB.data_ptr(), sy._ld(dB), dC.data_ptr(),
                             sy._ld(dC), X.data_ptr(), sy._ld(X), ctypes.byref(o),
                             ctypes.cast(ctypes.c_void_p(dinfo.data_ptr()), ctypes.POINTER(sy.Info)), None, 0,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == 0
    got = sy.Info.from_buffer_copy(bytes(dinfo.cpu().numpy())).as_dict()
    _, ref = sy.solve(dA, dB, dC)
    torch.cuda.synchronize()
    assert got["status"] == 0 and got["rel_res"] == ref["rel_res"] and got["iterations"] == ref["iterations"]
