"""Helpers shared by the GPU parity tests (inputs, tolerances, comparisons)."""
import math
import sys

import numpy as np

DX = math.pi / 4
# Tolerances (relative L2):
#   one FFT: FP64 1e-13, FP32 5e-6; 100 PFC steps: FP64 1e-12, FP32 1e-4.
TOL_FFT = {"f64": 1e-13, "f32": 5e-6}
TOL_STEP = {"f64": 1e-12, "f32": 1e-4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rounded(x, dtype):
    """The field as the GPU sees it (rounded once to FP32 for the FP32 path), widened to FP64."""
    return x.astype(np.float32).astype(np.float64) if dtype == "f32" else x.astype(np.float64)


def to_dev(x, dtype):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to(
        device="cuda:0", dtype=torch.float32 if dtype == "f32" else torch.float64)


def to_np(t):
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)
