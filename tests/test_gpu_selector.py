"""Selector plumbing on the GPU: the features of constructed equations
(sizes, norms, sep_est = delta by construction, fraction of complex pairs),
SYLV_PREC_AUTO with weights that force each class, the escalation that
overrules a wrong choice, and the kappa_est rule expressed as weights of the
same network."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_common import binding, dev, host, relerr, say

pytestmark = pytest.mark.gpu

TOL = 1e-14


@pytest.fixture
def sel():
    binding()
    from paper_2503_03456_amd import selector
    yield selector
    selector.uninstall()


def test_features_of_constructed_equation(sel):
    cfg = workloads.config3(2, m=300, n=200)    # delta = 1e-3, normal A and B
    A, B, C = dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"])
    f = sel.features(A, B, C)
    torch.cuda.synchronize()
    assert abs(f[0] - np.log2(300)) < 1e-5 and abs(f[1] - np.log2(200)) < 1e-5
    assert abs(f[2] - np.log10(np.linalg.norm(cfg["A"]) / np.sqrt(300))) < 1e-4
    assert abs(f[4] - np.log10(np.linalg.norm(cfg["C"]) / np.sqrt(300 * 200))) < 1e-4
    # sep(A, -B) = delta exactly (normal coefficients); binary32 forms resolve it
    assert abs(f[5] - np.log10(cfg["delta"])) < 0.02
    na, nb = np.linalg.norm(cfg["A"]), np.linalg.norm(cfg["B"])
    assert abs(f[6] - np.log10((na + nb) / cfg["delta"])) < 0.02
    # normal coefficients: T is block diagonal up to rounding
    assert f[7] < 1e-3 and f[8] < 1e-3
    # fraction of eigenvalues in complex pairs, from the constructed spectra
    fa = np.mean(np.abs(cfg["eigA"].imag) > 0)
    fb = np.mean(np.abs(cfg["eigB"].imag) > 0)
    assert abs(f[9] - fa) < 1e-6 and abs(f[10] - fb) < 1e-6
    # ||U^T U - I||_F of binary32 forms: about sqrt(n) u_32 .. n u_32
    assert -8 < f[13] < -3 and -8 < f[14] < -3
    assert f[15] == 0.0
    fl = sel.features(A, None, dev(np.eye(300)))   # Lyapunov form: n = m, flag set
    assert fl[15] == 1.0 and abs(fl[1] - np.log2(300)) < 1e-5


def test_auto_requires_installed_weights(sel):
    sy = binding()
    A, B, C = workloads.sylv_random(3, 40, 30)
    sel.uninstall()
    with pytest.raises(sy.SylvError):
        sy.solve(dev(A), dev(B), dev(C), low="auto")


@pytest.mark.parametrize("k", [0, 1, 2])
def test_auto_forced_class(sel, k):
    sy = binding()
    A, B, C = workloads.sylv_random(4, 120, 90, scale=0.5 / np.sqrt(120))
    sel.install(*sel.forced_params(k))
    X, info = sy.solve(dev(A), dev(B), dev(C), low="auto")
    torch.cuda.synchronize()
    assert info["chosen"] == k and info["rel_res"] <= TOL and info["fell_back"] == 0, info
    assert info["precision_used"] == ("bf16", "fp32", "fp64")[k]
    Xo, _ = oracle.bs_solve(A, B, C)
    assert relerr(host(X), Xo) <= 1e-12


def test_wrong_choice_is_overruled(sel):
    """Class 0 forced on an equation with kappa ~ 1e7: bfloat16 transforms
    cannot converge, the same binary32 forms then cannot either within the
    stagnation rule, and the binary64 path delivers."""
    sy = binding()
    cfg = workloads.config3(5, m=200, n=150)    # delta = 1e-6
    sel.install(*sel.forced_params(0))
    X, info = sy.solve(dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"]), low="auto")
    torch.cuda.synchronize()
    assert info["chosen"] == 0 and info["fell_back"] == 1, info
    assert info["rel_res"] <= TOL
    Xo, _ = oracle.bs_solve(cfg["A"], cfg["B"], cfg["C"])
    assert relerr(host(X), Xo) <= 1e-6


@pytest.mark.parametrize("j,expect", [(0, 1), (6, 2)])
def test_kappa_rule_as_weights(sel, j, expect):
    """log10 kappa_est = log10((||A||_F + ||B||_F)/delta) of config-3
    equations at m = 160, n = 96: ~2.8 for delta = 1e-1 (class 1), ~8.8 for
    delta = 1e-7 (class 2)."""
    sy = binding()
    cfg = workloads.config3(j, m=160, n=96)
    sel.install(*sel.rule_params(lo=1.5, hi=6.0))
    X, info = sy.solve(dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"]), low="auto")
    torch.cuda.synchronize()
    assert info["chosen"] == expect and info["rel_res"] <= TOL, info


def test_trained_weights_gain_time_on_held_out(sel):
    """The committed weights (trained on the GPU from solver-generated
    instances, seeds 200000+, sizes up to 1024) on held-out instances of the
    same recipe (seeds 300000+, orders 128..1024): every solve reaches the
    tolerance, the selector escalates less often than the method without it
    (binary32 forms + refinement, binary64 on failure), and the total solve
    time is lower (each equation timed under both policies back to back, best
    of two, after an untimed solve that sizes the workspace)."""
    import time
    sy = binding()
    params, mean, std = sel.load()
    eqs = []
    for i in range(40):
        d = workloads.selector_instance(i, 128, 1024, 300000)
        eqs.append((dev(d["A"]), None if d["B"] is None else dev(d["B"]), dev(d["C"])))

    def run(eq, **kw):
        A, B, C = eq
        return sy.lyap(A, C, **kw) if B is None else sy.solve(A, B, C, **kw)

    sel.install(params, mean, std)
    t = {"auto": 0.0, "fp32": 0.0}
    esc = {"auto": 0, "fp32": 0}
    for eq in eqs:
        run(eq, low="auto")
        torch.cuda.synchronize()
        for name in ("auto", "fp32"):
            best = None
            for _ in range(2):
                t0 = time.perf_counter()
                _, info = run(eq, low=name)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
                assert info["rel_res"] <= TOL, (name, info)
            t[name] += best
            esc[name] += info["fell_back"]
    say(f"held-out 40: auto {t['auto']:.3f} s ({esc['auto']} escalations), "
        f"fp32 {t['fp32']:.3f} s ({esc['fp32']} escalations)")
    assert esc["fp32"] >= 5
    assert esc["auto"] < esc["fp32"], esc
    assert t["auto"] < t["fp32"], t


def test_selector_train_entry_point(sel):
    """sylv_selector_train: the feature statistics it computes on the device
    equal numpy's, the loss falls, a separable synthetic set is learnt, the
    same seed gives the same weights, and the blob installs."""
    rs = np.random.RandomState(5)
    n = 1500
    F = rs.standard_normal((n, 16)).astype(np.float32) * 3.0 + 1.5
    # class by two standardised coordinates: a task the network must fit
    y = np.where(F[:, 6] < 0.5, 0, np.where(F[:, 6] < 3.5, 1, 2)).astype(np.int32)
    p1, m1, s1, h1 = sel.train_device(F, y, epochs=80, batch=256, seed=7)
    p2, m2, s2, h2 = sel.train_device(F, y, epochs=80, batch=256, seed=7)
    torch.cuda.synchronize()
    np.testing.assert_allclose(m1, F.astype(np.float64).mean(axis=0), rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(s1, F.astype(np.float64).std(axis=0), rtol=1e-5)
    assert h1[-1] < 0.5 * h1[0]
    assert np.array_equal(p1, p2) and h1 == h2
    P = sel.predict(p1, m1, s1, F)
    # the majority class is 45% of the set; the learnt boundaries are near-exact
    assert np.mean(P.argmax(1) == y) > 0.9
    sel.install(p1, m1, s1)


def test_selector_load_file(sel, tmp_path):
    """sylv_selector_load: a file written by save_blob installs the same
    weights (forced class 2 chosen by AUTO); a wrong header is refused."""
    sy = binding()
    path = str(tmp_path / "w.bin")
    sel.save_blob(path, *sel.forced_params(2))
    sel.load_file(path)
    A, B, C = workloads.sylv_random(9, 30, 20)
    X, info = sy.solve(dev(A), dev(B), dev(C), low="auto")
    torch.cuda.synchronize()
    assert info["chosen"] == 2 and info["precision_used"] == "fp64" and info["rel_res"] <= TOL
    bad = str(tmp_path / "bad.bin")
    with open(bad, "wb") as fh:
        fh.write(b"SYLVSEL0" + b"\0" * 64)
    assert sy.lib().sylv_selector_load(bad.encode()) == -2
    assert sy.lib().sylv_selector_load(str(tmp_path / "missing.bin").encode()) == -1


@pytest.mark.parametrize("k", [0, 1, 2])
def test_batched_auto_forced_class(sel, k):
    """sylv_solve_batched with AUTO: one forward pass over the batch; with
    weights that force class k every equation takes it (0: bfloat16-operand
    transforms, 1: binary32, 2: the binary64 path) and meets the oracle."""
    sy = binding()
    sel.install(*sel.forced_params(k))
    sizes = [150, 40, 17, 256]
    its = [workloads.config4_item(2500 + i, n) for i, n in enumerate(sizes)]
    Xs, infos = sy.solve_batched([(dev(A), dev(C)) for A, C, _ in its], low="auto")
    torch.cuda.synchronize()
    for (A, C, eig), X, info in zip(its, Xs, infos):
        assert info["chosen"] == k, info
        assert info["rel_res"] <= TOL, info
        if k == 2:
            assert info["precision_used"] == "fp64" and info["fell_back"] == 0
        Xo, st = oracle.lyap_solve(A, C)
        lam = eig[:, None] + eig[None, :]
        kap = np.abs(lam).max() / np.abs(lam).min()
        assert relerr(host(X), Xo) <= 100 * 2.0 ** -53 * kap


def test_batched_auto_kappa_rule_uses_device_features(sel):
    """The kappa_est rule as network weights (feature 6 = log10 kappa_est,
    computed by the batched feature kernel): a well-separated equation gets
    class 0 or 1, one with sep 2e-7 (kappa_est ~ 1e8.5) class 2."""
    sy = binding()
    # hi = 4: the class-2 logit exceeds class 1's by ~4.5 at kappa_est ~ 1e8.5,
    # above the batched decision's margin of ln 20
    sel.install(*sel.rule_params(lo=2.0, hi=4.0))
    A1, C1, e1 = workloads.config4_item(2600, 90)
    A2, C2, e2 = workloads.config4_item(2601, 90)
    shift = -e2.real.max() - 1e-7
    A2 = A2 + shift * np.eye(90)
    _, infos = sy.solve_batched([(dev(A1), dev(C1)), (dev(A2), dev(C2))], low="auto")
    torch.cuda.synchronize()
    assert infos[0]["chosen"] in (0, 1) and infos[1]["chosen"] == 2, infos
    assert all(i["rel_res"] <= TOL for i in infos)
