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


def parity_errs(a, b):
    """(plain rel-L2, mean-removed rel-L2, max-abs) of `a` against the reference `b`.

    plain:        ||a - b|| / ||b|| over all values;
    mean-removed: the same after subtracting each array's mean (the mean of psi, about -0.3 against
                  +-0.1 fluctuations, holds most of ||psi||^2 and would hide errors in the
                  fluctuations); the plain value when b is (nearly) uniform;
    max-abs:      max |a - b| / max |b|, element by element."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    d = a - b
    nb = float(np.linalg.norm(b))
    plain = float(np.linalg.norm(d)) / nb
    bc = b - b.mean()
    nbc = float(np.linalg.norm(bc))
    centred = float(np.linalg.norm(d - d.mean())) / nbc if nbc > 1e-6 * nb else plain
    maxabs = float(np.max(np.abs(d))) / float(np.max(np.abs(b)))
    return plain, centred, maxabs


def parity_err(a, b):
    """The largest of the three measures of parity_errs: a parity assert `parity_err(a, b) < tol`
    bounds the plain and the mean-removed relative L2 error and the element-wise error at once."""
    return max(parity_errs(a, b))


def fmt_errs(errs):
    """Text of the three measures of parity_errs."""
    return "rel L2 %.2e, mean-removed %.2e, max-abs %.2e" % tuple(errs)


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
