"""Selector network kernels (FP32 forward, cross-entropy gradient, Adam) on
the GPU against the FP64 analytic oracle (oracle/mlp.py, itself pinned to
central finite differences on the CPU)."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from gpu_common import binding

pytestmark = pytest.mark.gpu


def _theta(seed):
    rs = np.random.RandomState(seed)
    parts = []
    for shp in omlp.SIZES:
        fan = shp[1] if len(shp) == 2 else 16
        parts.append(rs.standard_normal(shp) * np.sqrt(2.0 / fan))
    return omlp.pack(parts)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("n", [1, 7, 300, 1000])
def test_forward_matches_oracle(n):
    sy = binding()
    th = _theta(n)
    X = np.random.RandomState(10 + n).standard_normal((n, 16))
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Td = torch.tensor(th, dtype=torch.float32, device="cuda")
    P = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    rc = sy.lib().sylv_mlp_forward(n, ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(Td.data_ptr()),
                                   ctypes.c_void_p(P.data_ptr()), _stream())
    torch.cuda.synchronize()
    assert rc == 0
    # reference on the binary32-rounded inputs
    Po, _ = omlp.forward(th.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64))
    assert np.abs(P.cpu().numpy() - Po).max() <= 1e-5


@pytest.mark.parametrize("n", [5, 64, 513])
def test_train_step_gradient_loss_and_adam(n):
    sy = binding()
    th = _theta(100 + n)
    rs = np.random.RandomState(200 + n)
    X = rs.standard_normal((n, 16))
    y = rs.randint(0, 3, size=n)
    th32 = th.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    m0 = rs.standard_normal(th.size) * 1e-3
    v0 = np.abs(rs.standard_normal(th.size)) * 1e-6
    t = 3
    lr = 1e-3
    Td = torch.tensor(th, dtype=torch.float32, device="cuda")
    Md = torch.tensor(m0, dtype=torch.float32, device="cuda")
    Vd = torch.tensor(v0, dtype=torch.float32, device="cuda")
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    yd = torch.tensor(y, dtype=torch.int32, device="cuda")
    G = torch.empty(th.size, dtype=torch.float32, device="cuda")
    loss = ctypes.c_float(0.0)
    rc = sy.lib().sylv_mlp_train_step(n, ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(yd.data_ptr()),
                                      ctypes.c_void_p(Td.data_ptr()), ctypes.c_void_p(Md.data_ptr()),
                                      ctypes.c_void_p(Vd.data_ptr()), t, ctypes.c_float(lr),
                                      ctypes.c_void_p(G.data_ptr()), ctypes.byref(loss), _stream())
    torch.cuda.synchronize()
    assert rc == 0
    go = omlp.backward(th32, X32, y)
    g = G.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    assert abs(loss.value - omlp.loss(th32, X32, y)) <= 1e-5 * max(1.0, omlp.loss(th32, X32, y))
    # Adam from the GPU's own gradient: the update rule alone
    th_o, m_o, v_o = omlp.adam_step(th32, g, m0.astype(np.float32).astype(np.float64),
                                    v0.astype(np.float32).astype(np.float64), t, lr=lr)
    assert np.abs(Td.cpu().numpy() - th_o).max() <= 1e-6
    assert np.abs(Md.cpu().numpy() - m_o).max() <= 1e-7
    assert np.abs(Vd.cpu().numpy() - v_o).max() <= 1e-10 + 1e-5 * np.abs(v_o).max()


def test_training_reduces_loss_on_separable_data():
    """A few hundred GPU steps fit a linearly separable 3-class problem."""
    binding()
    from paper_2503_03456_amd import selector
    rs = np.random.RandomState(7)
    F = rs.standard_normal((2000, 16)).astype(np.float32)
    y = np.where(F[:, 6] < -0.5, 0, np.where(F[:, 6] > 0.5, 2, 1)).astype(np.int32)
    params, mean, std, hist = selector.train(F, y, epochs=20, batch=256, lr=3e-3)
    P = selector.predict(params, mean, std, F)
    assert hist[-1] < 0.5 * hist[0]
    assert np.mean(P.argmax(1) == y) > 0.95
