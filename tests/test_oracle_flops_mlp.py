"""Pins for the flop-model oracle (values printed in the paper) and the MLP
oracle (finite differences)."""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import flops, mlp

GOLD = os.path.join(os.path.dirname(__file__), "golden", "flop_model.json")


def test_flop_model_golden():
    """Every entry of the golden file carries its citation in the paper."""
    with open(GOLD) as f:
        g = json.load(f)
    n = 1000
    for e in g["entries"]:
        kind = e["kind"]
        if kind == "phi":
            fn = {"S1": lambda r: flops.phi_S1(r, n, n), "S2": lambda r: flops.phi_S2(r, n, n),
                  "L1": flops.phi_L1, "L2": flops.phi_L2}[e["which"]]
            val = fn(Fr(e["rho"]))
        elif kind == "ratio":
            val = flops.cost_ratio(e["alg"], Fr(e["rho"]), n, n, e["i"], e.get("lyap", False))
        elif kind == "equiv":
            low, high = (flops.alg41 if e["alg"] == 1 else flops.alg42)(n, n, e["i"])
            val = (Fr(e["rho"]) * low + high) / Fr(n ** 3)
        else:
            raise AssertionError(kind)
        if "exact" in e:
            assert Fr(val) == Fr(e["exact"]), e
        assert abs(float(val) - e["value"]) <= e["tol"], (e, float(val))


def test_bs_counts():
    assert flops.bs_sylv(10, 10) == 60 * 1000          # Sec. 2.2.1: 60 n^3 at m = n
    assert flops.bs_lyap(10) == 35 * 1000
    assert flops.stationary(10, 10, 2) == 3 * 2 * 10 * 10 * 20
    assert flops.stationary(10, 10, 2, lyap=True) == 6 * 2 * 1000
    # Table 4.1 at m = n: alpha = beta = 2 n^3
    lo, hi = flops.alg41(10, 10, 1)
    assert lo == 26 * 2000 and hi == 13 * 2000
    lo, hi = flops.alg42(10, 10, 1)
    assert lo == 26 * 2000 and hi == Fr(14, 3) * 2000 + 7 * 2000


def test_break_even_consistency():
    """At i = phi(rho) the mixed cost equals Bartels-Stewart exactly."""
    for rho in [Fr(0), Fr(1, 10), Fr(1, 2)]:
        for m, n in [(100, 100), (400, 100)]:
            i = flops.phi_S1(rho, m, n)
            low, high = flops.alg41(m, n, i)
            assert rho * low + high == flops.bs_sylv(m, n)
            i = flops.phi_S2(rho, m, n)
            low, high = flops.alg42(m, n, i)
            assert rho * low + high == flops.bs_sylv(m, n)
        i = flops.phi_L1(rho)
        low, high = flops.alg41(10, 10, i, lyap=True)
        assert rho * low + high == flops.bs_lyap(10)


def _theta(seed):
    rs = np.random.RandomState(seed)
    return rs.standard_normal(mlp.NPARAM) * 0.3


def test_mlp_param_count():
    assert mlp.NPARAM == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3 == 5443


def test_mlp_gradient_finite_differences():
    rs = np.random.RandomState(3)
    th = _theta(4)
    X = rs.standard_normal((7, 16))
    y = rs.randint(0, 3, size=7)
    g = mlp.backward(th, X, y)
    # sample coordinates from every tensor; skip points near ReLU kinks
    _, (Xc, z1, _, z2, _, _) = mlp.forward(th, X)
    assert np.abs(z1).min() > 1e-4 and np.abs(z2).min() > 1e-4
    idx = np.concatenate([rs.choice(mlp.NPARAM, 40, replace=False), [0, 1024, 1087, 5183, 5442]])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(th)
        e[k] = h
        fd = (mlp.loss(th + e, X, y) - mlp.loss(th - e, X, y)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-8, (k, fd, g[k])


def test_mlp_probabilities_and_adam():
    th = _theta(5)
    X = np.random.RandomState(6).standard_normal((4, 16))
    p, _ = mlp.forward(th, X)
    assert np.allclose(p.sum(axis=1), 1.0)
    g = np.ones(mlp.NPARAM)
    th2, m, v = mlp.adam_step(th, g, np.zeros_like(th), np.zeros_like(th), 1, lr=1e-3)
    # first Adam step with constant gradient moves every weight by lr (bias-corrected)
    assert np.allclose(th - th2, 1e-3 * 1 / (1 + 1e-8), rtol=1e-6)
