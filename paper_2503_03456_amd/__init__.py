"""Python binding of libsylv.so, the gfx950 mixed-precision Sylvester /
Lyapunov solver.

Argument marshalling only: every arithmetic step runs in the HIP library.
PyTorch provides device memory and streams.  Matrices are float64 (or
float32 for the stage-level calls) CUDA tensors; they are passed to the
library column-major.  A tensor that is not column-major is copied into a
column-major buffer first (``colmajor``).

The library must be built (``python paper_2503_03456_amd/build.py`` or
``__graft_entry__.build()``).  Importing this module raises ImportError if it
is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsylv.so")
HEADER = os.path.join(_HERE, "..", "include", "sylv.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_2503_03456_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "auto": 4}
PREC_NAME = {v: k for k, v in PREC.items()}
KIND = {"sylv": 0, "lyap": 1}


class Opts(ctypes.Structure):
    _fields_ = [("low", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("fallback", ctypes.c_int), ("orth_check", ctypes.c_int), ("alg", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("rel_res", ctypes.c_double), ("orth_u", ctypes.c_double),
                ("orth_v", ctypes.c_double), ("sep_est", ctypes.c_double),
                ("corr_ratio", ctypes.c_double), ("iterations", ctypes.c_int),
                ("precision_used", ctypes.c_int), ("fell_back", ctypes.c_int),
                ("status", ctypes.c_int), ("chosen", ctypes.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["precision_used"] = PREC_NAME.get(d["precision_used"], d["precision_used"])
        return d


_vp, _i, _d, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
_ip = ctypes.POINTER(ctypes.c_int)
_dp = ctypes.POINTER(ctypes.c_double)

_lib.sylv_default_opts.argtypes = [ctypes.POINTER(Opts)]
_lib.sylv_default_opts.restype = None
_lib.sylv_workspace_size.argtypes = [_i, _i, _i, ctypes.POINTER(Opts)]
_lib.sylv_workspace_size.restype = _sz
_lib.sylv_solve.argtypes = [_i, _i, _vp, _i, _vp, _i, _vp, _i, _vp, _i, ctypes.POINTER(Opts),
                            ctypes.POINTER(Info), _vp, _sz, _vp]
_lib.sylv_solve.restype = _i
_lib.lyap_solve.argtypes = [_i, _vp, _i, _vp, _i, _vp, _i, ctypes.POINTER(Opts),
                            ctypes.POINTER(Info), _vp, _sz, _vp]
_lib.lyap_solve.restype = _i
NFEAT, NCLASS, NPARAM = 16, 3, 5443
_fp = ctypes.POINTER(ctypes.c_float)
_lib.sylv_selector_features.argtypes = [_i, _i, _vp, _i, _vp, _i, _vp, _i, _fp, _vp]
_lib.sylv_selector_features.restype = _i
_lib.sylv_selector_set.argtypes = [_fp, _i]
_lib.sylv_selector_set.restype = _i
_lib.sylv_mlp_forward.argtypes = [_i, _vp, _vp, _vp, _vp]
_lib.sylv_mlp_forward.restype = _i
_lib.sylv_mlp_train_step.argtypes = [_i, _vp, _vp, _vp, _vp, _vp, _i, ctypes.c_float, _vp, _fp, _vp]
_lib.sylv_mlp_train_step.restype = _i
_lib.sylv_schur_tune.argtypes = [_i, _i, _i, _i, _i, _i, _i, _i, _i]
_lib.sylv_schur_tune.restype = _i
_lib.sylv_schur_tune_get.argtypes = [_i, _ip]
_lib.sylv_schur_tune_get.restype = _i
_pp = ctypes.POINTER(ctypes.c_void_p)
_lib.sylv_solve_batched.argtypes = [_i, _ip, _ip, _ip, _pp, _ip, _pp, _ip, _pp, _ip, _pp, _ip,
                                    ctypes.POINTER(Opts), ctypes.POINTER(Info), _vp, _sz, _vp]
_lib.sylv_solve_batched.restype = _i
_lib.sylv_batched_workspace_size.argtypes = [_i, _ip, _ip, _ip, ctypes.POINTER(Opts)]
_lib.sylv_batched_workspace_size.restype = _sz
_lib.sylv_init.argtypes = []
_lib.sylv_init.restype = _i
_lib.sylv_solve_noalloc.argtypes = [_i, _i, _vp, _i, _vp, _i, _vp, _i, _vp, _i, ctypes.POINTER(Opts),
                                    ctypes.POINTER(Info), _vp]
_lib.sylv_solve_noalloc.restype = _i
_lib.sylv_batched_tune.argtypes = [_i, _i, _i, _i, _i, _i]
_lib.sylv_batched_tune.restype = _i
_lib.sylv_batched_tune_get.argtypes = [_ip]
_lib.sylv_batched_tune_get.restype = _i
_lib.sylv_cholqr.argtypes = [_i, _vp, _i, _vp, _i, _ip, _vp]
_lib.sylv_cholqr.restype = _i
_lib.sylv_selector_load.argtypes = [ctypes.c_char_p]
_lib.sylv_selector_load.restype = _i
_lib.sylv_status_string.argtypes = [_i]
_lib.sylv_status_string.restype = ctypes.c_char_p
_lib.sylv_schur.argtypes = [_i, _vp, _i, _vp, _i, _vp, _i, _i, _ip, _vp]
_lib.sylv_schur.restype = _i
_lib.sylv_sym_eig.argtypes = [_i, _vp, _i, _vp, _vp, _i, _i, _ip, _ip, _vp]
_lib.sylv_sym_eig.restype = _i
_lib.sylv_trsyl.argtypes = [_i, _i, _vp, _i, _vp, _i, _i, _vp, _i, _i, _ip, _vp]
_lib.sylv_trsyl.restype = _i
_lib.sylv_residual.argtypes = [_i, _i, _vp, _i, _vp, _i, _vp, _i, _vp, _i, _vp, _i, _i, _dp, _vp]
_lib.sylv_residual.restype = _i
_lib.sylv_gemm.argtypes = [_i, _i, _i, _i, _i, _i, _d, _vp, _i, _vp, _i, _d, _vp, _i, _vp]
_lib.sylv_gemm.restype = _i


class SylvError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise SylvError(f"{what} failed with code {rc}: {_lib.sylv_status_string(rc).decode()}")


def lib():
    """The loaded ctypes library (for direct C-ABI calls)."""
    return _lib


def exported_symbols():
    """Function names declared in include/sylv.h."""
    with open(HEADER) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sylv_\w+|lyap_\w+)\s*\(", src)))


def colmajor(t: torch.Tensor) -> torch.Tensor:
    """Column-major (stride (1, rows)) version of a 2-D tensor (copy if needed)."""
    if t.dim() != 2:
        raise ValueError("expected a matrix")
    r, c = t.shape
    if t.stride(0) == 1 and (t.stride(1) >= max(1, r) or c <= 1):
        return t
    return t.t().contiguous().t()


def _ld(t):
    return max(1, t.stride(1) if t.shape[1] > 1 else t.shape[0])


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


ALG = {"orig": 0, "orth": 1, "inv": 2, "sym": 3}


def make_opts(low="fp32", tol=1e-14, max_iter=20, fallback=True, orth_check=1, alg="orig"):
    o = Opts()
    _lib.sylv_default_opts(ctypes.byref(o))
    o.alg = ALG[alg] if isinstance(alg, str) else int(alg)
    o.low = PREC[low] if isinstance(low, str) else int(low)
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.fallback = int(bool(fallback))
    o.orth_check = int({"off": 0, "probe": 1, "full": 2}.get(orth_check, orth_check))
    return o


def workspace_size(m, n, lyap=False, **kw):
    return int(_lib.sylv_workspace_size(m, n, int(lyap), ctypes.byref(make_opts(**kw))))


def solve(A, B, C, X=None, work=None, stream=None, **kw):
    """AX + XB = C on the GPU.  Returns (X, info dict)."""
    A, B, C = colmajor(A), colmajor(B), colmajor(C)
    m, n = C.shape
    if X is None:
        X = torch.empty((n, m), dtype=torch.float64, device=C.device).t()
    o = make_opts(**kw)
    info = Info()
    wp = ctypes.c_void_p(work.data_ptr()) if work is not None else None
    wb = work.numel() * work.element_size() if work is not None else 0
    rc = _lib.sylv_solve(m, n, A.data_ptr(), _ld(A), B.data_ptr(), _ld(B), C.data_ptr(), _ld(C),
                         X.data_ptr(), _ld(X), ctypes.byref(o), ctypes.byref(info), wp, wb,
                         _stream(stream))
    _check(rc, "sylv_solve")
    return X, info.as_dict()


def init():
    """Per-device set-up of the current device (needed before solve_noalloc)."""
    _check(_lib.sylv_init(), "sylv_init")


def solve_noalloc(A, B, C, X, stream=None, **kw):
    """AX + XB = C with the library's static scratch: no allocation by the
    library or here (X must be a column-major float64 CUDA tensor)."""
    A, B, C = colmajor(A), colmajor(B), colmajor(C)
    m, n = C.shape
    if X.stride(0) != 1:
        raise ValueError("X must be column-major")
    o = make_opts(**kw)
    info = Info()
    rc = _lib.sylv_solve_noalloc(m, n, A.data_ptr(), _ld(A), B.data_ptr(), _ld(B), C.data_ptr(), _ld(C),
                                 X.data_ptr(), _ld(X), ctypes.byref(o), ctypes.byref(info), _stream(stream))
    _check(rc, "sylv_solve_noalloc")
    return X, info.as_dict()


def lyap(A, C, X=None, work=None, stream=None, **kw):
    """AX + XA^T = C on the GPU.  Returns (X, info dict)."""
    A, C = colmajor(A), colmajor(C)
    n = C.shape[0]
    if X is None:
        X = torch.empty((n, n), dtype=torch.float64, device=C.device).t()
    o = make_opts(**kw)
    info = Info()
    wp = ctypes.c_void_p(work.data_ptr()) if work is not None else None
    wb = work.numel() * work.element_size() if work is not None else 0
    rc = _lib.lyap_solve(n, A.data_ptr(), _ld(A), C.data_ptr(), _ld(C), X.data_ptr(), _ld(X),
                         ctypes.byref(o), ctypes.byref(info), wp, wb, _stream(stream))
    _check(rc, "lyap_solve")
    return X, info.as_dict()


def _iarr(v):
    return (ctypes.c_int * max(1, len(v)))(*[int(x) for x in v])


def _parr(ts):
    return (ctypes.c_void_p * max(1, len(ts)))(*[(t.data_ptr() if t is not None else None) for t in ts])


def batched_workspace_size(kinds, ms, ns, **kw):
    return int(_lib.sylv_batched_workspace_size(len(kinds), _iarr(kinds), _iarr(ms), _iarr(ns),
                                                ctypes.byref(make_opts(**kw))))


def solve_batched(eqs, Xs=None, work=None, stream=None, **kw):
    """Solve a list of equations in one call.  Each item is (A, C) for
    AX + XA^T = C or (A, B, C) for AX + XB = C.  Returns (list of X, list
    of info dicts)."""
    kinds, ms, ns, As, Bs, Cs, lda, ldb, ldc = [], [], [], [], [], [], [], [], []
    for e in eqs:
        if len(e) == 2:
            A, C = colmajor(e[0]), colmajor(e[1])
            kinds.append(1); As.append(A); Bs.append(None); Cs.append(C)
            lda.append(_ld(A)); ldb.append(1); ldc.append(_ld(C))
            ms.append(C.shape[0]); ns.append(C.shape[0])
        else:
            A, B, C = colmajor(e[0]), colmajor(e[1]), colmajor(e[2])
            kinds.append(0); As.append(A); Bs.append(B); Cs.append(C)
            lda.append(_ld(A)); ldb.append(_ld(B)); ldc.append(_ld(C))
            ms.append(C.shape[0]); ns.append(C.shape[1])
    if Xs is None:
        Xs = [torch.empty((C.shape[1], C.shape[0]), dtype=torch.float64, device=C.device).t() for C in Cs]
    Xs = [colmajor(X) for X in Xs]
    ldx = [_ld(X) for X in Xs]
    nb = len(eqs)
    o = make_opts(**kw)
    infos = (Info * max(1, nb))()
    wp = ctypes.c_void_p(work.data_ptr()) if work is not None else None
    wb = work.numel() * work.element_size() if work is not None else 0
    rc = _lib.sylv_solve_batched(nb, _iarr(kinds), _iarr(ms), _iarr(ns), _parr(As), _iarr(lda),
                                 _parr(Bs), _iarr(ldb), _parr(Cs), _iarr(ldc), _parr(Xs), _iarr(ldx),
                                 ctypes.byref(o), infos, wp, wb, _stream(stream))
    _check(rc, "sylv_solve_batched")
    return Xs, [infos[i].as_dict() for i in range(nb)]


def _prec_of(t):
    if t.dtype == torch.float64:
        return 0
    if t.dtype == torch.float32:
        return 1
    raise TypeError("float64 or float32 tensor expected")


def schur(A, stream=None):
    """Real Schur form on the GPU in A's precision: (T, U, status)."""
    A = colmajor(A)
    n = A.shape[0]
    T = torch.empty((n, n), dtype=A.dtype, device=A.device).t()
    U = torch.empty((n, n), dtype=A.dtype, device=A.device).t()
    st = ctypes.c_int(0)
    rc = _lib.sylv_schur(n, A.data_ptr(), _ld(A), T.data_ptr(), _ld(T), U.data_ptr(), _ld(U),
                         _prec_of(A), ctypes.byref(st), _stream(stream))
    _check(rc, "sylv_schur")
    return T, U, st.value


def cholqr(Q, stream=None):
    """CholQR2 of a nearly orthogonal float64 matrix: (Q factor, R, status)
    with positive diag(R); the input is not modified."""
    Qo = colmajor(Q).clone()
    Qo = Qo.t().contiguous().t()
    n = Qo.shape[0]
    R = torch.empty((n, n), dtype=torch.float64, device=Qo.device).t()
    st = ctypes.c_int(0)
    rc = _lib.sylv_cholqr(n, Qo.data_ptr(), _ld(Qo), R.data_ptr(), _ld(R), ctypes.byref(st), _stream(stream))
    _check(rc, "sylv_cholqr")
    return Qo, R, st.value


def sym_eig(S, stream=None):
    """Symmetric eigen-decomposition on the GPU in S's precision (block
    Jacobi on (S + S^T)/2): (d, Q, sweeps, status) with S = Q diag(d) Q^T."""
    S = colmajor(S)
    n = S.shape[0]
    d = torch.empty(n, dtype=S.dtype, device=S.device)
    Q = torch.empty((n, n), dtype=S.dtype, device=S.device).t()
    sw, st = ctypes.c_int(0), ctypes.c_int(0)
    rc = _lib.sylv_sym_eig(n, S.data_ptr(), _ld(S), d.data_ptr(), Q.data_ptr(), _ld(Q), _prec_of(S),
                           ctypes.byref(sw), ctypes.byref(st), _stream(stream))
    _check(rc, "sylv_sym_eig")
    return d, Q, sw.value, st.value


def trsyl(TA, TB, C, trans_b=False, stream=None):
    """TA Y + Y op(TB) = C (quasi-triangular) on the GPU: (Y, perturbed)."""
    TA, TB = colmajor(TA), colmajor(TB)
    Y = colmajor(C.clone())
    m, n = Y.shape
    pf = ctypes.c_int(0)
    rc = _lib.sylv_trsyl(m, n, TA.data_ptr(), _ld(TA), TB.data_ptr(), _ld(TB), int(bool(trans_b)),
                         Y.data_ptr(), _ld(Y), _prec_of(Y), ctypes.byref(pf), _stream(stream))
    _check(rc, "sylv_trsyl")
    return Y, pf.value


def residual(A, B, C, X, lyap=False, stream=None):
    """Binary64 R = C - AX - X op(B) and the relative residual of eq. (2.1)."""
    A, C, X = colmajor(A), colmajor(C), colmajor(X)
    B = A if lyap else colmajor(B)
    m, n = C.shape
    R = torch.empty((n, m), dtype=torch.float64, device=C.device).t()
    rr = ctypes.c_double(0.0)
    rc = _lib.sylv_residual(m, n, A.data_ptr(), _ld(A), B.data_ptr(), _ld(B), C.data_ptr(), _ld(C),
                            X.data_ptr(), _ld(X), R.data_ptr(), _ld(R), int(bool(lyap)),
                            ctypes.byref(rr), _stream(stream))
    _check(rc, "sylv_residual")
    return R, rr.value


def gemm(A, B, C=None, alpha=1.0, beta=0.0, ta=False, tb=False, stream=None):
    """C = alpha op(A) op(B) + beta C on MFMA (A's precision)."""
    A, B = colmajor(A), colmajor(B)
    m = A.shape[1] if ta else A.shape[0]
    k = A.shape[0] if ta else A.shape[1]
    n = B.shape[0] if tb else B.shape[1]
    if C is None:
        C = torch.zeros((n, m), dtype=A.dtype, device=A.device).t()
    C = colmajor(C)
    rc = _lib.sylv_gemm(_prec_of(A), int(ta), int(tb), m, n, k, float(alpha), A.data_ptr(), _ld(A),
                        B.data_ptr(), _ld(B), float(beta), C.data_ptr(), _ld(C), _stream(stream))
    _check(rc, "sylv_gemm")
    return C
