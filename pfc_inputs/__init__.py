"""Seeded synthetic inputs shared by the tests, the oracle runs and the benchmark.

This module holds no arithmetic of the PFC method.  It only draws seeded random fields.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014), the 64-bit state version with Stafford's "variant 13" output mix.  The generator
seeded with ``seed`` adds the golden-ratio increment GAMMA to its state before each output, so
its i-th output (0-based) is ``mix64(seed + (i + 1) * GAMMA mod 2^64)``.  That closed form makes
the stream counter-based: element i of a C-order field is the i-th output, so any slice of a field
can be drawn independently and the numpy and torch versions agree bit for bit.

Doubles: ``u = (x >> 11) * 2^-53`` in [0, 1).  U(a, b) = a + (b - a) * u.  N(0, 1) by the
Box-Muller transform of the pair (u_{2i}, u_{2i+1}): sqrt(-2 ln(1 - u_{2i})) cos(2 pi u_{2i+1}).
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1
TWO_M53 = 2.0 ** -53


def splitmix64_sequential(seed: int, count: int) -> list[int]:
    """The generator as published: a running state, advanced by GAMMA before each output."""
    state = seed & MASK64
    out = []
    for _ in range(count):
        state = (state + GAMMA) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * M1) & MASK64
        z = ((z ^ (z >> 27)) * M2) & MASK64
        out.append(z ^ (z >> 31))
    return out


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the stream seeded with ``seed`` (uint64 array)."""
    idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & MASK64) + idx * np.uint64(GAMMA)
        return _mix64_np(state)


def unit_uniform(seed: int, start: int, count: int) -> np.ndarray:
    """Doubles in [0, 1) from outputs start .. start+count-1."""
    x = splitmix64(seed, start, count)
    return (x >> np.uint64(11)).astype(np.float64) * TWO_M53


def derive_seed(seed: int, index: int) -> int:
    """Seed of sub-stream ``index`` of ``seed``: that output of the parent stream."""
    return int(splitmix64(seed, index, 1)[0])


def uniform(seed: int, shape, lo: float, hi: float) -> np.ndarray:
    """C-order float64 field with entries U(lo, hi)."""
    count = int(np.prod(shape))
    return (lo + (hi - lo) * unit_uniform(seed, 0, count)).reshape(shape)


def normal(seed: int, shape) -> np.ndarray:
    """C-order float64 field with entries N(0, 1) (Box-Muller on consecutive output pairs)."""
    count = int(np.prod(shape))
    u = unit_uniform(seed, 0, 2 * count)
    a, b = u[0::2], u[1::2]
    return (np.sqrt(-2.0 * np.log1p(-a)) * np.cos(2.0 * math.pi * b)).reshape(shape)


def pfc_initial_field(seed: int, shape, mean: float, amplitude: float = 0.1) -> np.ndarray:
    """psi0 = mean + U(-amplitude, amplitude), the initial-condition recipe of the PFC runs."""
    return mean + uniform(seed, shape, -amplitude, amplitude)


# ---------------------------------------------------------------------------- torch (device) form
# Used where a field is too large to draw on the host (e.g. 2048^3).  Same stream, same values:
# int64 arithmetic wraps modulo 2^64 like uint64, and logical right shifts are arithmetic shifts
# with the sign-extended bits masked off.


def _as_i64(v: int) -> int:
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _lsr(z, s: int):
    return (z >> s) & ((1 << (64 - s)) - 1)


def _unit_uniform_torch(seed: int, start: int, count: int, device):
    import torch

    idx = torch.arange(start + 1, start + 1 + count, dtype=torch.int64, device=device)
    z = idx * _as_i64(GAMMA) + _as_i64(seed)
    z = (z ^ _lsr(z, 30)) * _as_i64(M1)
    z = (z ^ _lsr(z, 27)) * _as_i64(M2)
    z = z ^ _lsr(z, 31)
    return _lsr(z, 11).to(torch.float64) * TWO_M53


def uniform_torch(seed: int, shape, lo: float, hi: float, dtype, device, offset: float = 0.0,
                  chunk: int = 1 << 26):
    """Same values as ``offset + uniform(...)`` (float64, rounded once to ``dtype``), drawn on
    ``device`` in chunks."""
    import torch

    count = int(np.prod(shape))
    out = torch.empty(count, dtype=dtype, device=device)
    for s in range(0, count, chunk):
        c = min(chunk, count - s)
        u = _unit_uniform_torch(seed, s, c, device)
        out[s : s + c] = (offset + (lo + (hi - lo) * u)).to(dtype)
        del u
    return out.view(*shape)


def normal_torch(seed: int, shape, dtype, device, chunk: int = 1 << 25):
    """Same values as ``normal`` (rounded once to ``dtype``), drawn on ``device`` in chunks."""
    import torch

    count = int(np.prod(shape))
    out = torch.empty(count, dtype=dtype, device=device)
    for s in range(0, count, chunk):
        c = min(chunk, count - s)
        u = _unit_uniform_torch(seed, 2 * s, 2 * c, device)
        a, b = u[0::2], u[1::2]
        out[s : s + c] = (torch.sqrt(-2.0 * torch.log1p(-a)) * torch.cos(2.0 * math.pi * b)).to(dtype)
        del u, a, b
    return out.view(*shape)


def pfc_initial_field_torch(seed: int, shape, mean: float, dtype, device, amplitude: float = 0.1):
    """Same values as ``pfc_initial_field`` (rounded once to ``dtype``), drawn on ``device``."""
    return uniform_torch(seed, shape, -amplitude, amplitude, dtype, device, offset=mean)


# ---------------------------------------------------------------------------- amplitude fields
# Inputs of the complex-amplitude form: principal reciprocal-lattice vectors (components along the
# grid axes, slowest axis first; unit length for the first shell) and seeded complex amplitudes.

_S3 = math.sqrt(3.0) / 2.0
_R2 = 1.0 / math.sqrt(2.0)
_R3 = 1.0 / math.sqrt(3.0)
LATTICES = {
    # 2D (y, x): one shell of the triangular lattice (k1 + k2 + k3 = 0), and the square lattice
    "triangular": [(-0.5, -_S3), (1.0, 0.0), (-0.5, _S3)],
    "square": [(1.0, 0.0), (0.0, 1.0)],
    # 2D two shells of the triangular lattice: |k| = 1 and |k| = sqrt(3)
    "triangular2": [(-0.5, -_S3), (1.0, 0.0), (-0.5, _S3), (1.5, _S3), (-1.5, _S3), (0.0, -2.0 * _S3)],
    # 3D (z, y, x): bcc, the six <110> vectors of unit length
    "bcc": [(0.0, _R2, _R2), (0.0, _R2, -_R2), (_R2, 0.0, _R2), (_R2, 0.0, -_R2), (_R2, _R2, 0.0),
            (_R2, -_R2, 0.0)],
    # 3D fcc, two shells: four <111> of unit length and three <200> of length 2/sqrt(3)
    "fcc2": [(_R3, _R3, _R3), (_R3, -_R3, -_R3), (-_R3, _R3, -_R3), (-_R3, -_R3, _R3),
             (2 * _R3, 0.0, 0.0), (0.0, 2 * _R3, 0.0), (0.0, 0.0, 2 * _R3)],
}


def triangular_reciprocal(count: int) -> np.ndarray:
    """The ``count`` shortest reciprocal vectors i (1, 0) + j (-1/2, sqrt(3)/2) (components (y, x))
    of the triangular lattice, one of each +- pair, ordered by length, then by angle in [0, pi)."""
    out = []
    for i in range(-12, 13):
        for j in range(-12, 13):
            y, x = i - 0.5 * j, _S3 * j
            r2 = y * y + x * x
            ang = math.atan2(x, y)
            if r2 < 1e-12 or not (0.0 <= ang < math.pi - 1e-9):
                continue
            out.append((round(r2, 9), round(ang, 9), y, x))
    out.sort()
    return np.array([(y, x) for _, _, y, x in out[:count]], dtype=np.float64)


def lattice_vectors(name: str) -> np.ndarray:
    """[N][ndim] principal wave vectors of a named lattice ("triangular<N>": the N shortest
    reciprocal vectors of the triangular lattice)."""
    if name.startswith("triangular") and name[10:].isdigit() and int(name[10:]) > 2:
        return triangular_reciprocal(int(name[10:]))
    return np.array(LATTICES[name], dtype=np.float64)


def amplitude_fields(seed: int, nfields: int, shape, mean: float, amplitude: float = 0.02) -> np.ndarray:
    """[nfields, *shape] complex amplitudes: mean + U(-a, a) + i U(-a, a), field j drawn from the
    sub-streams 2j (real part) and 2j + 1 (imaginary part) of ``seed``."""
    out = np.empty((nfields,) + tuple(shape), np.complex128)
    for j in range(nfields):
        out[j].real = mean + uniform(derive_seed(seed, 2 * j), shape, -amplitude, amplitude)
        out[j].imag = uniform(derive_seed(seed, 2 * j + 1), shape, -amplitude, amplitude)
    return out


def amplitude_fields_torch(seed: int, nfields: int, shape, mean: float, cdtype, device, amplitude: float = 0.02):
    """Same values as ``amplitude_fields`` (each part rounded once), drawn on ``device``."""
    import torch

    rdt = torch.float32 if cdtype == torch.complex64 else torch.float64
    out = torch.empty((nfields,) + tuple(shape), dtype=cdtype, device=device)
    for j in range(nfields):
        re = uniform_torch(derive_seed(seed, 2 * j), shape, -amplitude, amplitude, rdt, device, offset=mean)
        im = uniform_torch(derive_seed(seed, 2 * j + 1), shape, -amplitude, amplitude, rdt, device)
        out[j] = torch.complex(re, im)
        del re, im
    return out


def batch_workload():
    """Descriptors of the batched workload: 48 independent 2D runs, {128^2, 256^2, 512^2, 1024^2} x
    12, six one-mode and six two-mode (Q1^2 = 2, R1 = 0.05) per size, r_i ~ U(-0.35, -0.15) from
    sub-stream (4, i), dt = 0.25, FP32.  The initial field of instance i is drawn from sub-stream
    (4, 1000 + i) with mean r_i (``pfc_initial_field``)."""
    out = []
    i = 0
    for n in (128, 256, 512, 1024):
        for j in range(12):
            two = j >= 6
            r = float(uniform(derive_seed(4, i), (1,), -0.35, -0.15)[0])
            out.append(dict(shape=(n, n), dtype="f32", model=1 if two else 0, r=r, dt=0.25,
                            q1sq=2.0 if two else 4.0 / 3.0, R1=0.05 if two else 0.0))
            i += 1
    return out

