"""Helpers shared by the GPU tests (marshalling and comparison only)."""
import numpy as np


def device():
    import torch
    from paper_2508_13386_amd import ms
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a GPU")
    return ms.TorchDevice(0)


def e_rel(x_gpu, x_orc, x_t):
    u_g = x_gpu - x_t
    u_o = x_orc - x_t
    return float(np.linalg.norm(u_g - u_o) / np.linalg.norm(u_o))


def say(*a):
    print(*a, flush=True)
