"""Shared helpers for the GPU parity tests (test-only)."""
from __future__ import annotations

import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda", 0)


def to_dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=torch_dev())


def to_np(t):
    return t.detach().cpu().numpy()


def rel_err(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    den = np.abs(ref).max()
    if den == 0:
        return float(np.abs(x).max())
    return float(np.abs(x - ref).max() / den)


def gpu_all(system, D, V, precision="fp64", tau=None):
    """rho (list), M, grad from the HIP path through the C ABI."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    g = GPW(system, precision=precision, tau=tau)
    Dd = to_dev(D)
    Vd = [to_dev(v) for v in V]
    rho = g.rho(Dd)
    M = g.mat(Vd)
    grad = g.grad(Dd, Vd)
    torch.cuda.synchronize()
    out = ([to_np(r) for r in rho], to_np(M), to_np(grad), g.info)
    g.close()
    return out
