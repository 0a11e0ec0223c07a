"""Helpers shared by the GPU tests: tensor marshalling and relative errors."""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n > 0 else d


def to_gpu(x, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda:0", dtype=dtype).contiguous()


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().to("cpu", dtype=torch.float64).numpy()


def say(*args):
    print(*args, flush=True)
