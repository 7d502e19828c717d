"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np


def torch_dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a, dtype="float64"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0",
                                                       dtype=getattr(torch, dtype))


def print_case(*args):
    print("[case]", *args, flush=True)
