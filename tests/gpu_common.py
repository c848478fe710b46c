"""Shared helpers for the GPU parity tests (imported by tests marked ``gpu``)."""
import sys

import numpy as np
import pytest

U64 = 2.0 ** -53


def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def lib():
    torch_gpu()
    import paper_1806_01036_amd as borth
    from paper_1806_01036_amd import _lib
    _lib.load()  # raises if the HIP library is missing (no fallback)
    return borth


def dev(a, dtype=None):
    torch = torch_gpu()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_fro(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
