"""Helpers for the GPU tests: move seeded inputs to the device, call the C ABI
through the package binding, bring results back as float64 numpy arrays."""
import sys

import numpy as np


def torch_mod():
    import torch
    return torch


def dev():
    torch = torch_mod()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda", 0)


def to_dev(a, dtype=None):
    torch = torch_mod()
    dtype = dtype or torch.float32
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev()).to(dtype)


def to_np(t):
    """float64 numpy copy (exact for every storage type, float64 included)."""
    torch = torch_mod()
    return t.detach().to(torch.float64).cpu().numpy()


def geometry(desc):
    import paper_2110_13526_amd as kct
    return kct.Geometry.from_desc(desc, device=dev())


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
