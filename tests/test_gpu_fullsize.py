"""Parity at the benchmark workloads' full sizes, in the configuration
bench.py times (caller-resident binary64 inputs, default options).

References: the independent block-diagonal route of tests/exact_route.py
(closed-form block solves on the constructed factors, pinned against the
oracle and Kronecker at small sizes) for the normal constructions, the
planted eigen-decompositions for the symmetric workload, and the C oracle
on sampled equations of the batched workload."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from exact_route import exact_solution
from gpu_common import U64, binding, dev, host, relerr, say

pytestmark = pytest.mark.gpu

TOL = 1e-14


def kappa(eig_a, eig_b):
    """kappa_est = max|l + m| / min|l + m| over the constructed spectra (exact
    2-norm condition number of the Kronecker operator for normal A, B)."""
    lam = np.abs(np.asarray(eig_a)[:, None] + np.asarray(eig_b)[None, :])
    return lam.max() / lam.min()


def test_sylvester_2048_benchmark_workload():
    """Config 2 (m = n = 2048), binary32 forms + binary64 refinement."""
    sy = binding()
    say("full size: sylvester 2048")
    cfg = workloads.config2()
    X, info = sy.solve(dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"]), low="fp32")
    torch.cuda.synchronize()
    assert info["rel_res"] <= TOL and info["fell_back"] == 0 and info["status"] == 0, info
    Xe = exact_solution(cfg)
    kap = kappa(cfg["eigA"], cfg["eigB"])
    err = relerr(host(X), Xe)
    say(f"  rel_res {info['rel_res']:.2e} iterations {info['iterations']} forward {err:.2e} kappa {kap:.1f}")
    # forward error at the binary64 level: 100 u kappa_est
    assert err <= 100 * U64 * kap


@pytest.mark.parametrize("j", [1, 5])
def test_sylvester_4096x1024_sep_sweep(j):
    """Config 3 at full size: delta = 1e-2 (binary32 refinement converges)
    and delta = 1e-6 (beyond binary32: the binary64 fallback answers).
    Forward error against the exact route within 100 u kappa_est."""
    sy = binding()
    cfg = workloads.config3(j)
    say(f"full size: config3 delta={cfg['delta']:.0e}")
    X, info = sy.solve(dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"]), low="fp32")
    torch.cuda.synchronize()
    assert info["rel_res"] <= TOL, info
    assert info["fell_back"] == (1 if cfg["delta"] < 1e-4 else 0), info
    Xe = exact_solution(cfg)
    err = relerr(host(X), Xe)
    kap = kappa(cfg["eigA"], cfg["eigB"])
    say(f"  rel_res {info['rel_res']:.2e} fell_back {info['fell_back']} forward {err:.2e} "
        f"bound {100 * U64 * kap:.2e}")
    assert err <= 100 * U64 * kap


def test_batched_lyapunov_4096_full_batch():
    """Config 4: all 4096 equations in one batched call; every equation at
    the tolerance without fallback; 16 sampled equations (every 256th of the
    longest-first order, so all sizes are covered) against the oracle."""
    sy = binding()
    say("full size: 4096 batched Lyapunov")
    sizes = workloads.config4_sizes()
    items = [workloads.config4_item(i, int(n)) for i, n in enumerate(sizes)]
    Xs, infos = sy.solve_batched([(dev(A), dev(C)) for A, C, _ in items])
    torch.cuda.synchronize()
    bad = [k for k, inf in enumerate(infos) if not (inf["rel_res"] <= TOL and inf["fell_back"] == 0)]
    assert not bad, (len(bad), infos[bad[0]])
    order = np.argsort(-np.asarray(sizes), kind="stable")
    for k in order[::256]:
        A, C, eig = items[k]
        Xo, st = oracle.lyap_solve(A, C)
        assert st == 0
        kap = kappa(eig, eig)
        n = A.shape[0]
        err = relerr(host(Xs[k]), Xo)
        assert err <= 100 * U64 * kap, (k, n, err, kap)


def test_symmetric_2048_workload():
    """Symmetric workload (m = n = 2048): the symmetric route against the
    solution formed from the planted eigen-decompositions."""
    sy = binding()
    say("full size: symmetric 2048")
    cfg = workloads.config_sym()
    X, info = sy.solve(dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"]), low="fp32", alg="sym")
    torch.cuda.synchronize()
    assert info["rel_res"] <= TOL and info["fell_back"] == 0 and info["status"] == 0, info
    QA, QB, la, lb = cfg["QA"], cfg["QB"], cfg["eigA"], cfg["eigB"]
    Xe = QA @ ((QA.T @ cfg["C"] @ QB) / (la[:, None] + lb[None, :])) @ QB.T
    kap = (la.max() + lb.max()) / (la.min() + lb.min())
    err = relerr(host(X), Xe)
    say(f"  rel_res {info['rel_res']:.2e} iterations {info['iterations']} forward {err:.2e}")
    assert err <= 100 * U64 * kap
