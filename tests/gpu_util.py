"""Helpers for the GPU tests: device transfer and the shared library context."""
import numpy as np
import pytest


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(a, dtype=None):
    torch = torch_cuda()
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def ctx():
    torch_cuda()
    from paper_2004_05756_amd import binding
    return binding.context(0)


def problem_tensors(p, rho):
    torch = torch_cuda()
    return dev(rho, torch.float64), dev(p.mask, torch.uint8), dev(p.f, torch.float64)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
