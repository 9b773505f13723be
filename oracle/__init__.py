"""FP64 CPU oracle for the pseudo-spectral PFC step -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may import this
package.  It wraps ``liboracle.so`` (plain C, ``pfc_oracle.c``), which shares no code with the HIP
library.  What each function computes, and which passage of arxiv 2603.26818 it follows, is
stated in ``pfc_oracle.c``; this file only marshals numpy arrays.

All arrays are float64 (real) or complex128 (half spectra ``[n0][n1][n2/2+1]``), C-order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile liboracle.so with the C compiler (always recompiles)."""
    subprocess.run(["make", "-B", "-s", "-C", _HERE, "liboracle.so"], check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    i64p = P(ctypes.c_int64)
    dp = P(ctypes.c_double)
    lib.or_fft_c2c.argtypes = [ctypes.c_int, i64p, dp, ctypes.c_int]
    lib.or_rfftn.argtypes = [ctypes.c_int, i64p, dp, dp]
    lib.or_irfftn.argtypes = [ctypes.c_int, i64p, dp, dp]
    pp = P(_OrParams)
    lib.or_state_init.argtypes = [pp, dp, dp]
    lib.or_step.argtypes = [pp, dp, dp, ctypes.c_int64]
    lib.or_energy.argtypes = [pp, dp, dp, dp]
    lib.or_step_backward.argtypes = [pp, dp, dp, dp, dp, dp]
    lib.or_num_threads.argtypes = []
    lib.or_set_num_threads.argtypes = [ctypes.c_int]
    lib.or_hydro_step.argtypes = [pp, ctypes.POINTER(_OrHydro), dp, dp, dp, dp, ctypes.c_int64]
    ap = P(_OrApfc)
    lib.or_apfc_nonlinear.argtypes = [ap, dp, dp]
    lib.or_apfc_counts.argtypes = [ap, ctypes.c_int, P(ctypes.c_int)]
    lib.or_apfc_state_init.argtypes = [ap, dp, dp]
    lib.or_apfc_step.argtypes = [ap, dp, dp, ctypes.c_int64]
    for f in ("or_fft_c2c", "or_rfftn", "or_irfftn", "or_state_init", "or_step", "or_energy",
              "or_step_backward", "or_num_threads", "or_set_num_threads", "or_hydro_step", "or_apfc_nonlinear", "or_apfc_counts",
              "or_apfc_state_init", "or_apfc_step"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


class _OrHydro(ctypes.Structure):
    _fields_ = [("rho0", ctypes.c_double), ("gamma", ctypes.c_double), ("a0", ctypes.c_double)]


class _OrParams(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double * 3),
        ("model", ctypes.c_int),
        ("r", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("q1sq", ctypes.c_double),
        ("R1", ctypes.c_double),
        ("linear_only", ctypes.c_int),
        ("no_projection", ctypes.c_int),
    ]


@dataclass
class Params:
    """Grid and model.  ``shape`` is C-order (slowest axis first, x last)."""

    shape: tuple
    dx: float | tuple = np.pi / 4
    model: int = 0  # 0 one-mode, 1 two-mode
    r: float = -0.25
    dt: float = 0.5
    q1sq: float = 4.0 / 3.0
    R1: float = 0.0
    linear_only: bool = False
    no_projection: bool = False
    _c: _OrParams = field(default=None, repr=False, compare=False)

    def c(self) -> _OrParams:
        p = _OrParams()
        p.ndim = len(self.shape)
        dx = self.dx if isinstance(self.dx, (tuple, list)) else (self.dx,) * len(self.shape)
        for a in range(3):
            p.n[a] = int(self.shape[a]) if a < len(self.shape) else 1
            p.dx[a] = float(dx[a]) if a < len(self.shape) else 1.0
        p.model = int(self.model)
        p.r, p.dt, p.q1sq, p.R1 = float(self.r), float(self.dt), float(self.q1sq), float(self.R1)
        p.linear_only = int(bool(self.linear_only))
        p.no_projection = int(bool(self.no_projection))
        return p

    @property
    def half_shape(self):
        return tuple(self.shape[:-1]) + (self.shape[-1] // 2 + 1,)


def _dims(shape):
    return (ctypes.c_int64 * 3)(*(list(shape) + [1] * (3 - len(shape))))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def fft_c2c(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Full complex nd DFT (sign -1 forward, +1 inverse without 1/N)."""
    y = np.ascontiguousarray(x, dtype=np.complex128).copy()
    _check(_load().or_fft_c2c(y.ndim, _dims(y.shape), _dp(y.view(np.float64)), sign), "fft_c2c")
    return y


def rfftn(x: np.ndarray) -> np.ndarray:
    """Half spectrum [.., n/2+1] of a real field, self-conjugate planes projected."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    h = np.zeros(x.shape[:-1] + (x.shape[-1] // 2 + 1,), np.complex128)
    _check(_load().or_rfftn(x.ndim, _dims(x.shape), _dp(x), _dp(h.view(np.float64))), "rfftn")
    return h


def irfftn(h: np.ndarray, shape) -> np.ndarray:
    """Real field of a half spectrum, scaled by 1/N."""
    h = np.ascontiguousarray(h, dtype=np.complex128)
    x = np.zeros(tuple(shape), np.float64)
    _check(_load().or_irfftn(len(shape), _dims(shape), _dp(h.view(np.float64)), _dp(x)), "irfftn")
    return x


def state_init(p: Params, psi0: np.ndarray) -> np.ndarray:
    psi0 = np.ascontiguousarray(psi0, dtype=np.float64)
    s = np.zeros(p.half_shape, np.complex128)
    _check(_load().or_state_init(ctypes.byref(p.c()), _dp(psi0), _dp(s.view(np.float64))), "state_init")
    return s


def step(p: Params, psi: np.ndarray, state: np.ndarray, nsteps: int):
    """Returns (psi^{n+nsteps}, state^{n+nsteps}); inputs are not modified."""
    psi = np.array(psi, dtype=np.float64, order="C", copy=True)
    state = np.array(state, dtype=np.complex128, order="C", copy=True)
    _check(_load().or_step(ctypes.byref(p.c()), _dp(psi), _dp(state.view(np.float64)), int(nsteps)), "step")
    return psi, state


def energy(p: Params, psi: np.ndarray, state: np.ndarray):
    """(F from the spectrum, F from real space, mean of psi)."""
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    state = np.ascontiguousarray(state, dtype=np.complex128)
    out = np.zeros(3, np.float64)
    _check(_load().or_energy(ctypes.byref(p.c()), _dp(psi), _dp(state.view(np.float64)), _dp(out)), "energy")
    return float(out[0]), float(out[1]), float(out[2])


def step_backward(p: Params, psi_n, psi_np1, lam_np1):
    """(lambda^n, contribution of this step to dL/dr)."""
    psi_n = np.ascontiguousarray(psi_n, dtype=np.float64)
    psi_np1 = np.ascontiguousarray(psi_np1, dtype=np.float64)
    lam_np1 = np.ascontiguousarray(lam_np1, dtype=np.float64)
    lam_n = np.zeros_like(psi_n)
    acc = np.zeros(1, np.float64)
    _check(_load().or_step_backward(ctypes.byref(p.c()), _dp(psi_n), _dp(psi_np1), _dp(lam_np1),
                                    _dp(lam_n), _dp(acc)), "step_backward")
    return lam_n, float(acc[0])


def rollout(p: Params, psi0: np.ndarray, nsteps: int):
    """All fields psi^0..psi^nsteps of a run started from psi0 (state from psi0)."""
    psi = np.array(psi0, dtype=np.float64, copy=True)
    s = state_init(p, psi)
    out = [psi.copy()]
    for _ in range(nsteps):
        psi, s = step(p, psi, s, 1)
        out.append(psi.copy())
    return out


def loss_and_grad(p: Params, psi0: np.ndarray, target: np.ndarray, nsteps: int):
    """L = sum (psi^T - target)^2 and its gradients (dL/dpsi0, dL/dr) by the adjoint sweep."""
    traj = rollout(p, psi0, nsteps)
    diff = traj[-1] - target
    L = float(np.sum(diff * diff))
    lam = 2.0 * diff
    dLdr = 0.0
    for n in range(nsteps - 1, -1, -1):
        lam, g = step_backward(p, traj[n], traj[n + 1], lam)
        dLdr += g
    return L, lam, dLdr


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of later oracle calls."""
    _check(_load().or_set_num_threads(int(n)), "set_num_threads")


@dataclass
class Hydro:
    """Hydrodynamic PFC parameters (multiphysics section, Eq. (5)-(6)): mass density rho0,
    viscosity gamma, Gaussian averaging width a0."""

    rho0: float = 1.0
    gamma: float = 1.0
    a0: float = 1.0

    def c(self) -> _OrHydro:
        return _OrHydro(float(self.rho0), float(self.gamma), float(self.a0))


def hydro_step(p: Params, h: Hydro, psi: np.ndarray, psi_state: np.ndarray, v: np.ndarray, v_state: np.ndarray,
               nsteps: int):
    """nsteps hydrodynamic PFC steps.  v: [ndim, *shape] velocity components (axis order as the
    grid: component j is the velocity along axis j); v_state: their half spectra.  Returns new
    (psi, psi_state, v, v_state)."""
    psi = np.ascontiguousarray(psi, dtype=np.float64).copy()
    S = np.ascontiguousarray(psi_state, dtype=np.complex128).copy()
    v = np.ascontiguousarray(v, dtype=np.float64).copy()
    V = np.ascontiguousarray(v_state, dtype=np.complex128).copy()
    assert v.shape == (len(p.shape),) + tuple(p.shape) and V.shape == (len(p.shape),) + p.half_shape
    hc = h.c()
    _check(_load().or_hydro_step(ctypes.byref(p.c()), ctypes.byref(hc), _dp(psi), _dp(S.view(np.float64)), _dp(v),
                                 _dp(V.view(np.float64)), int(nsteps)), "hydro_step")
    return psi, S, v, V


APFC_MAX = 32


class _OrApfc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double * 3),
        ("nfields", ctypes.c_int),
        ("kvec", (ctypes.c_double * 3) * APFC_MAX),
        ("dB", ctypes.c_double),
        ("Bx", ctypes.c_double),
        ("t", ctypes.c_double),
        ("v", ctypes.c_double),
        ("dt", ctypes.c_double),
    ]


@dataclass
class Apfc:
    """Complex-amplitude PFC (equations in pfc_oracle.c): grid ``shape`` (C order), spacing ``dx``,
    principal wave vectors ``kvec`` [N][ndim] (components along the grid axes, slowest first),
    coefficients dB, Bx, t, v and time step dt."""

    shape: tuple
    kvec: np.ndarray
    dx: float | tuple = np.pi / 2
    dB: float = -0.15
    Bx: float = 1.0
    t: float = 0.0
    v: float = 1.0
    dt: float = 0.5

    @property
    def nfields(self) -> int:
        return int(np.asarray(self.kvec).shape[0])

    @property
    def field_shape(self):
        return (self.nfields,) + tuple(self.shape)

    def c(self) -> _OrApfc:
        a = _OrApfc()
        nd = len(self.shape)
        a.ndim = nd
        dx = self.dx if isinstance(self.dx, (tuple, list)) else (self.dx,) * nd
        for i in range(3):
            a.n[i] = int(self.shape[i]) if i < nd else 1
            a.dx[i] = float(dx[i]) if i < nd else 1.0
        k = np.asarray(self.kvec, dtype=np.float64)
        assert k.ndim == 2 and k.shape[1] == nd and 1 <= k.shape[0] <= APFC_MAX
        a.nfields = k.shape[0]
        for j in range(k.shape[0]):
            for i in range(nd):
                a.kvec[j][i] = float(k[j, i])
        a.dB, a.Bx, a.t, a.v, a.dt = (float(self.dB), float(self.Bx), float(self.t), float(self.v),
                                      float(self.dt))
        return a


def _cfields(a: Apfc, x) -> np.ndarray:
    x = np.array(x, dtype=np.complex128, order="C", copy=True)
    assert x.shape == a.field_shape, (x.shape, a.field_shape)
    return x


def apfc_nonlinear(a: Apfc, eta) -> np.ndarray:
    """N_j (the resonant part of -t psi^2 + v psi^3 at k_j) at every point, [N][grid] complex."""
    eta = _cfields(a, eta)
    out = np.zeros_like(eta)
    _check(_load().or_apfc_nonlinear(ctypes.byref(a.c()), _dp(eta.view(np.float64)), _dp(out.view(np.float64))),
           "apfc_nonlinear")
    return out


def apfc_counts(a: Apfc, j: int):
    """(resonant ordered pairs, resonant ordered triples) of field j."""
    c = (ctypes.c_int * 2)()
    _check(_load().or_apfc_counts(ctypes.byref(a.c()), int(j), c), "apfc_counts")
    return int(c[0]), int(c[1])


def apfc_state_init(a: Apfc, eta) -> np.ndarray:
    eta = _cfields(a, eta)
    out = np.zeros_like(eta)
    _check(_load().or_apfc_state_init(ctypes.byref(a.c()), _dp(eta.view(np.float64)), _dp(out.view(np.float64))),
           "apfc_state_init")
    return out


def apfc_step(a: Apfc, eta, eta_hat, nsteps: int):
    """nsteps amplitude steps; returns new (eta, eta_hat); inputs are not modified."""
    eta = _cfields(a, eta)
    S = _cfields(a, eta_hat)
    _check(_load().or_apfc_step(ctypes.byref(a.c()), _dp(eta.view(np.float64)), _dp(S.view(np.float64)),
                                int(nsteps)), "apfc_step")
    return eta, S
