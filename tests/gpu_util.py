"""Helpers for the GPU parity tests (host <-> device copies and error norms)."""
import numpy as np
import torch

DEV = "cuda:0"

# Per-order tolerance of max_k ||C^(k) - C_ref^(k)||_F / ||C_ref^(k)||_F against
# the FP64 oracle, by precision of the mode-wise products.
TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-4}


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def order_errors(c, ref):
    num = np.sqrt(np.sum(np.abs(c - ref) ** 2, axis=(-2, -1)))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=(-2, -1)))
    return num / np.where(den > 0, den, 1.0)
