"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/sylv.h declares, and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2503_03456_amd", "libsylv.so")
HEADER = os.path.join(ROOT, "include", "sylv.h")


def declared():
    with open(HEADER) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:sylv|lyap)_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libsylv.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_solver_calls():
    names = declared()
    for must in ["sylv_solve", "lyap_solve", "sylv_solve_batched", "sylv_workspace_size",
                 "sylv_default_opts", "sylv_status_string", "sylv_schur", "sylv_trsyl",
                 "sylv_residual", "sylv_gemm", "sylv_mlp_forward", "sylv_mlp_train_step"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    missing = [s for s in declared() if s not in exported]
    assert not missing, missing
    for s in declared():
        getattr(lib, s)


class Opts(ctypes.Structure):
    _fields_ = [("low", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("fallback", ctypes.c_int), ("orth_check", ctypes.c_int)]


def test_default_opts(lib):
    o = Opts()
    lib.sylv_default_opts(ctypes.byref(o))
    assert o.low == 1 and o.tol == 1e-14 and o.max_iter == 20 and o.fallback == 1


def test_argument_errors_are_synchronous(lib):
    vp = ctypes.c_void_p
    lib.sylv_solve.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int, vp,
                               ctypes.c_int, vp, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    # negative m
    assert lib.sylv_solve(-1, 3, None, 1, None, 3, None, 1, None, 1, None, None, None, 0, None) == -1
    # lda too small
    assert lib.sylv_solve(4, 3, 8, 2, 8, 3, 8, 4, 8, 4, None, None, None, 0, None) == -4
    # ldb too small
    assert lib.sylv_solve(4, 3, 8, 4, 8, 2, 8, 4, 8, 4, None, None, None, 0, None) == -6
    # null A
    assert lib.sylv_solve(4, 3, None, 4, 8, 3, 8, 4, 8, 4, None, None, None, 0, None) == -3
    # empty problem is a no-op success
    assert lib.sylv_solve(0, 3, None, 1, 8, 3, None, 1, None, 1, None, None, None, 0, None) == 0
    lib.lyap_solve.argtypes = [ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int,
                               vp, vp, vp, ctypes.c_size_t, vp]
    assert lib.lyap_solve(-2, None, 1, None, 1, None, 1, None, None, None, 0, None) == -1
    assert lib.lyap_solve(5, 8, 4, 8, 5, 8, 5, None, None, None, 0, None) == -3


def test_workspace_size_monotone(lib):
    lib.sylv_workspace_size.restype = ctypes.c_size_t
    lib.sylv_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    a = lib.sylv_workspace_size(64, 64, 0, None)
    b = lib.sylv_workspace_size(128, 64, 0, None)
    c = lib.sylv_workspace_size(64, 64, 1, None)
    assert 0 < a < b and c > 0
    assert lib.sylv_workspace_size(-1, 4, 0, None) == 0


def test_status_strings(lib):
    lib.sylv_status_string.restype = ctypes.c_char_p
    lib.sylv_status_string.argtypes = [ctypes.c_int]
    assert lib.sylv_status_string(0) == b"ok"
    assert b"invalid" in lib.sylv_status_string(-3)


def test_status_strings_of_library_codes(lib):
    lib.sylv_status_string.restype = ctypes.c_char_p
    lib.sylv_status_string.argtypes = [ctypes.c_int]
    assert b"captured" in lib.sylv_status_string(-2002) and b"allocate" in lib.sylv_status_string(-2002)
    assert b"captured" in lib.sylv_status_string(-2003)
    assert b"scratch" in lib.sylv_status_string(-2000)
    assert b"sylv_init" in lib.sylv_status_string(-2001)


def test_batched_tune_validation(lib):
    """sylv_batched_tune checks its arguments on the host (no GPU needed)
    and keeps the defaults on rejection."""
    v = (ctypes.c_int * 6)()
    assert lib.sylv_batched_tune_get(v) == 0
    before = list(v)
    assert lib.sylv_batched_tune(129, 64, 180, 128, 0, 3) == -1   # beyond the 128-capacity kernel
    assert lib.sylv_batched_tune(128, 65, 180, 128, 0, 3) == -2   # beyond the 64-capacity kernel
    assert lib.sylv_batched_tune(128, 64, 128, 180, 0, 3) == -3   # bands not descending
    assert lib.sylv_batched_tune(128, 64, 180, 0, 128, 3) == -3   # entry after the terminating 0
    assert lib.sylv_batched_tune(128, 64, 256, 0, 0, 3) == -3     # must be below the top bucket
    assert lib.sylv_batched_tune(128, 64, 180, 128, 0, 0) == -4
    assert lib.sylv_batched_tune_get(v) == 0 and list(v) == before
    assert lib.sylv_batched_tune(*before) == 0


def test_schur_tune_bounds_as_documented(lib):
    """sylv_schur_tune validates on the host against the bounds the header
    states (FP32: nsmall, nw <= 140, nb <= 44, window adv + 3 ceil(nb /
    chains) + 1 <= 141; FP64: 98, 32 and 99; adv >= 4; 1..4 chains; nibble
    0..100; 4 or 7 AED waves, 8 or 16 chase waves), at each edge, and a
    rejected call keeps the current values."""
    caps = {1: (140, 44, 141), 0: (98, 32, 99)}   # prec -> (nsmall/nw cap, nb cap, window cap)
    for prec, (ns, nbmax, wmax) in caps.items():
        v = (ctypes.c_int * 8)()
        assert lib.sylv_schur_tune_get(prec, v) == 0
        before = list(v)
        # (nsmall, nw, nb, adv, nibble, aed_waves, chase_waves, chains)
        base = [64, 48, 8, 16, 50, 7, 8, 2]
        ok = [
            dict(nsmall=ns), dict(nw=ns), dict(nb=nbmax, chains=4, adv=wmax - 3 * (nbmax // 4) - 1),
            dict(nb=nbmax, chains=2, adv=wmax - 3 * ((nbmax + 1) // 2) - 1), dict(adv=4), dict(aedw=4),
            dict(chasew=16), dict(chains=1), dict(nibble=0), dict(nibble=100),
        ]
        bad = [
            dict(nsmall=ns + 1), dict(nw=ns + 1), dict(nb=nbmax + 1, chains=4, adv=8),
            dict(nb=nbmax, chains=2, adv=wmax - 3 * ((nbmax + 1) // 2)), dict(adv=3), dict(chains=5),
            dict(aedw=5), dict(chasew=12), dict(nibble=101),
        ]
        keys = ["nsmall", "nw", "nb", "adv", "nibble", "aedw", "chasew", "chains"]
        for case in ok:
            args = [case.get(k, base[i]) for i, k in enumerate(keys)]
            assert lib.sylv_schur_tune(prec, *args) == 0, (prec, case)
            assert lib.sylv_schur_tune_get(prec, v) == 0 and list(v) == args, (prec, case)
        for case in bad:
            args = [case.get(k, base[i]) for i, k in enumerate(keys)]
            assert lib.sylv_schur_tune(prec, *[base[i] for i in range(8)]) == 0
            assert lib.sylv_schur_tune(prec, *args) == -2, (prec, case)
            assert lib.sylv_schur_tune_get(prec, v) == 0 and list(v) == base, (prec, case)
        # zeros keep the current values; a bad precision is refused
        assert lib.sylv_schur_tune(prec, 0, 0, 0, 0, -1, 0, 0, 0) == 0
        assert lib.sylv_schur_tune_get(prec, v) == 0 and list(v) == base
        assert lib.sylv_schur_tune(2, *base) == -1
        assert lib.sylv_schur_tune(prec, *before) == 0
        assert lib.sylv_schur_tune_get(prec, v) == 0 and list(v) == before


def test_batched_workspace_size(lib):
    """sylv_batched_workspace_size (host only): 0 for invalid arguments; a
    batch of Lyapunov equations of order <= 256 needs at least the per-equation
    buffers the batched path carves (one binary64 and six binary32 n x n
    arrays, 32 n^2 bytes); a Sylvester equation or an order above 256 goes to
    the single-equation path, 8 pooled slices of its workspace; adding
    equations never shrinks it."""
    lib.sylv_batched_workspace_size.restype = ctypes.c_size_t
    lib.sylv_workspace_size.restype = ctypes.c_size_t
    arr = lambda v: (ctypes.c_int * len(v))(*v)

    def size(kinds, ms, ns):
        return lib.sylv_batched_workspace_size(len(kinds), arr(kinds), arr(ms), arr(ns), None)

    assert lib.sylv_batched_workspace_size(-1, None, None, None, None) == 0
    assert lib.sylv_batched_workspace_size(2, None, arr([8, 8]), arr([8, 8]), None) == 0
    ns = [16, 40, 100, 256, 17, 200]
    s = size([1] * len(ns), ns, ns)
    assert s >= 32 * sum(n * n for n in ns)
    grow = [size([1] * k, ns[:k], ns[:k]) for k in range(1, len(ns) + 1)]
    assert all(b >= a for a, b in zip(grow, grow[1:]))
    # outside the batched kernels: one Sylvester equation, one order-300 Lyapunov
    big = lib.sylv_workspace_size(300, 300, 1, None)
    assert size([1], [300], [300]) >= 8 * big
    sylv = lib.sylv_workspace_size(120, 90, 0, None)
    assert size([0], [120], [90]) >= 8 * sylv
