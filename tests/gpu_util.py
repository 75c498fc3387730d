"""Helpers shared by the GPU tests (device transfer, error measures)."""
import sys

import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_max(a, b):
    """max |a - b| / max |b|."""
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_fro(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def announce(*parts):
    """Name the case on stdout before a GPU step (survives a lost box)."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()
