"""Graph capture: the solve calls check the stream and refuse, before any
call on it, when it is being captured (SYLV_ERR_CAPTURE_ALLOC for
work == NULL, SYLV_ERR_CAPTURE otherwise); the capture itself stays valid
and the library works normally afterwards."""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from gpu_common import binding, dev, say

pytestmark = pytest.mark.gpu

SYLV_ERR_CAPTURE_ALLOC = -2002
SYLV_ERR_CAPTURE = -2003


def test_solves_refuse_a_capturing_stream():
    sy = binding()
    L = sy.lib()
    A, B, C = workloads.sylv_random(77, 40, 30)
    dA, dB, dC = dev(A), dev(B), dev(C)
    X = torch.empty((30, 40), dtype=torch.float64, device="cuda").t()
    work = torch.empty(sy.workspace_size(40, 30), dtype=torch.uint8, device="cuda")
    o = sy.make_opts()
    info = sy.Info()
    y = torch.zeros(16, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()

    def call(wp, wb, st):
        return L.sylv_solve(40, 30, dA.data_ptr(), sy._ld(dA), dB.data_ptr(), sy._ld(dB), dC.data_ptr(),
                            sy._ld(dC), X.data_ptr(), sy._ld(X), ctypes.byref(o), ctypes.byref(info), wp, wb,
                            ctypes.c_void_p(st.cuda_stream))

    with torch.cuda.stream(s):
        g.capture_begin()
        try:
            y.add_(1.0)
            rc_alloc = call(None, 0, s)
            rc_work = call(ctypes.c_void_p(work.data_ptr()), work.numel(), s)
            rc_na = L.sylv_solve_noalloc(40, 30, dA.data_ptr(), sy._ld(dA), dB.data_ptr(), sy._ld(dB),
                                         dC.data_ptr(), sy._ld(dC), X.data_ptr(), sy._ld(X), ctypes.byref(o),
                                         ctypes.byref(info), ctypes.c_void_p(s.cuda_stream))
        finally:
            g.capture_end()
    say("capture codes", rc_alloc, rc_work, rc_na)
    assert rc_alloc == SYLV_ERR_CAPTURE_ALLOC
    assert rc_work == SYLV_ERR_CAPTURE
    # sylv_solve_noalloc: refused as well (its init check comes first when
    # sylv_init has not run in this process)
    assert rc_na in (SYLV_ERR_CAPTURE, -2001)
    g.replay()
    torch.cuda.synchronize()
    assert float(y[0]) == 1.0
    # the library still solves normally
    Xg, inf = sy.solve(dA, dB, dC)
    torch.cuda.synchronize()
    assert inf["status"] == 0 and inf["rel_res"] <= 1e-14
