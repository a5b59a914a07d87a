"""Helpers for the GPU parity tests (device transfer, error metrics)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def case(name):
    """Name the case on stdout before a GPU step."""
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def t(a, dtype=None):
    a = np.ascontiguousarray(a)
    if dtype is None:
        dtype = torch.complex64 if np.iscomplexobj(a) else torch.float32
    return torch.from_numpy(a).to(dtype).to(dev())


def h(x):
    torch.cuda.synchronize()
    return x.detach().cpu().numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rng_c(shape, seed):
    g = np.random.default_rng(seed)
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)) / np.sqrt(2)
