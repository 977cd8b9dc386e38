"""Shared helpers of the GPU tests (loading the binding, moving arrays)."""
import sys

import numpy as np
import pytest
import torch

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def binding():
    need_gpu()
    import paper_2503_03456_amd as sy
    return sy


def dev(a, dtype=torch.float64):
    """numpy (any order) -> column-major CUDA tensor."""
    t = torch.from_numpy(np.asfortranarray(a)).to(dtype)
    return t.t().contiguous().t().cuda() if t.dim() == 2 else t.cuda()


def host(t):
    return t.detach().cpu().double().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relerr(X, Y):
    return np.linalg.norm(X - Y) / max(np.linalg.norm(Y), 1e-300)


def check_schur(A, T, Uq, u, mult=20):
    """Schur invariants with unit roundoff u of the working precision."""
    n = A.shape[0]
    na = max(np.linalg.norm(A), 1e-300)
    res = np.linalg.norm(A - Uq @ T @ Uq.T) / na
    orth = np.linalg.norm(Uq.T @ Uq - np.eye(n))
    assert res <= mult * n * u, ("backward error", res)
    assert orth <= mult * n * u, ("orthogonality", orth)
    assert np.all(np.tril(T, -2) == 0)
    sub = np.diag(T, -1)
    assert not np.any((sub[:-1] != 0) & (sub[1:] != 0)), "consecutive subdiagonals"
    for i in np.nonzero(sub)[0]:
        a, b, c, d = T[i, i], T[i, i + 1], T[i + 1, i], T[i + 1, i + 1]
        assert (0.5 * (a - d)) ** 2 + b * c < 0, "2x2 block with real eigenvalues"
    return res, orth
