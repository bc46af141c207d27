"""Helpers shared by the GPU tests: device tensors and error measures."""
import sys

import numpy as np
import torch


def dev(a):
    """numpy array -> contiguous device tensor (same dtype)."""
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def empty(shape, dtype=torch.float32, fill=None):
    t = torch.empty(shape, dtype=dtype, device="cuda")
    if fill is not None:
        t.fill_(fill)
    return t


def say(*args):
    """Name the case on stdout before GPU work (flushes)."""
    print(*args, flush=True)
    sys.stdout.flush()


def normwise(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref)) if ref.size else 0.0
    num = np.max(np.abs(x - ref)) if ref.size else 0.0
    return float(num / den) if den > 0 else float(num)


TOL_FP32 = 1e-5  # normwise max relative error bound for FP32 results
