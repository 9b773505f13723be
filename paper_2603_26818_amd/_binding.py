"""ctypes binding of libpfc.so.  Argument marshalling only (see include/pfc.h for semantics)."""
from __future__ import annotations

import ctypes
import math
import os

PFC_F32, PFC_F64 = 0, 1
PFC_ONE_MODE, PFC_TWO_MODE = 0, 1
PFC_FLAG_LINEAR_ONLY = 1
PFC_FLAG_XROWS_BLOCK = 0x80


def PFC_FLAG_ZBLOCK(s: int) -> int:
    """Layout hint: blocks of 2^s z planes in the native state (3D; see include/pfc.h)."""
    return 0x10 | ((int(s) & 3) << 5)

_STATUS = {
    0: "PFC_OK",
    1: "PFC_ERR_INVALID_ARG",
    2: "PFC_ERR_UNSUPPORTED",
    3: "PFC_ERR_ALIGNMENT",
    4: "PFC_ERR_WORKSPACE",
    5: "PFC_ERR_HIP",
    6: "PFC_ERR_DIVERGED",
    7: "PFC_ERR_INTERNAL",
}

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def library_path() -> str:
    return os.path.join(_HERE, "libpfc.so")


class PfcError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {detail}")


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double * 3),
        ("dtype", ctypes.c_int),
        ("model", ctypes.c_int),
        ("r", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("q1sq", ctypes.c_double),
        ("R1", ctypes.c_double),
        ("device", ctypes.c_int),
        ("flags", ctypes.c_uint32),
    ]


APFC_MAX_FIELDS = 32


class ApfcDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double * 3),
        ("dtype", ctypes.c_int),
        ("nfields", ctypes.c_int),
        ("k", (ctypes.c_double * 3) * APFC_MAX_FIELDS),
        ("dB", ctypes.c_double),
        ("Bx", ctypes.c_double),
        ("t", ctypes.c_double),
        ("v", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("device", ctypes.c_int),
    ]


_SIGS = {
    "pfc_plan_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(PlanDesc)]),
    "pfc_plan_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "pfc_plan_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "pfc_plan_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]),
    "pfc_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pfc_plan_real_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "pfc_plan_half_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "pfc_plan_state_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "pfc_plan_x_fused": (ctypes.c_int, [ctypes.c_void_p]),
    "pfc_fft_r2c": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "pfc_fft_c2r": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "pfc_state_init": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "pfc_state_export": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "pfc_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "pfc_step_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p]),
    "pfc_step_watched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "pfc_step_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
    "pfc_step_backward": (ctypes.c_int, [ctypes.c_void_p] * 7),
    "pfc_plan_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "pfc_plan_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "pfc_plan_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "pfc_energy": (ctypes.c_int, [ctypes.c_void_p] * 5),
    "pfc_hydro_work_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "pfc_hydro_state_init": (ctypes.c_int, [ctypes.c_void_p] * 6),
    "pfc_hydro_step": (ctypes.c_int, [ctypes.c_void_p] * 7 + [ctypes.c_size_t, ctypes.c_int64, ctypes.c_void_p]),
    "pfc_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(PlanDesc), ctypes.c_int]),
    "pfc_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "pfc_batch_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.c_void_p, ctypes.c_size_t]),
    "pfc_batch_state_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pfc_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "pfc_batch_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pfc_batch_grid": (ctypes.c_int, [ctypes.c_void_p]),
    "pfc_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "pfc_batch_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "pfc_batch_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "pfc_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pfc_apfc_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ApfcDesc)]),
    "pfc_apfc_field_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "pfc_apfc_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "pfc_apfc_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "pfc_apfc_terms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int)]),
    "pfc_apfc_fft": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "pfc_apfc_nonlinear": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "pfc_apfc_state_init": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "pfc_apfc_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "pfc_apfc_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pfc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "pfc_last_error": (ctypes.c_char_p, []),
}


def load_library():
    """Load libpfc.so (raises if it has not been built).

    torch is imported first when it is installed: its wheel carries its own HIP runtime with the
    same soname as the system one, so loading it first makes libpfc.so bind to that runtime and the
    process holds a single HIP runtime (device memory and streams from torch are then valid here)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; build it with make -C paper_2603_26818_amd/csrc")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        raise PfcError(status, where, load_library().pfc_last_error().decode())


def _torch():
    import torch

    return torch


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_desc(shape, dtype="f32", model=PFC_ONE_MODE, r=-0.25, dt=0.5, dx=math.pi / 4, q1sq=4.0 / 3.0, R1=0.0,
              device=0, flags=0) -> PlanDesc:
    shape = tuple(int(v) for v in shape)
    d = PlanDesc()
    d.ndim = len(shape)
    dxs = tuple(dx) if isinstance(dx, (tuple, list)) else (dx,) * len(shape)
    for a in range(3):
        d.n[a] = shape[a] if a < len(shape) else 1
        d.dx[a] = float(dxs[a]) if a < len(shape) else 1.0
    d.dtype = PFC_F64 if dtype in ("f64", "float64", PFC_F64) else PFC_F32
    d.model = int(model)
    d.r, d.dt, d.q1sq, d.R1 = float(r), float(dt), float(q1sq), float(R1)
    d.device = int(device)
    d.flags = int(flags)
    return d


class Plan:
    """A pfc_plan with its workspace (a torch uint8 tensor on the plan's device)."""

    def __init__(self, shape, dtype="f32", model=PFC_ONE_MODE, r=-0.25, dt=0.5, dx=math.pi / 4, q1sq=4.0 / 3.0,
                 R1=0.0, device=0, flags=0):
        torch = _torch()
        lib = load_library()
        shape = tuple(int(s) for s in shape)
        d = PlanDesc()
        d.ndim = len(shape)
        dxs = tuple(dx) if isinstance(dx, (tuple, list)) else (dx,) * len(shape)
        for a in range(3):
            d.n[a] = shape[a] if a < len(shape) else 1
            d.dx[a] = float(dxs[a]) if a < len(shape) else 1.0
        self.f64 = dtype in ("f64", "float64", PFC_F64)
        d.dtype = PFC_F64 if self.f64 else PFC_F32
        d.model = int(model)
        d.r, d.dt, d.q1sq, d.R1 = float(r), float(dt), float(q1sq), float(R1)
        d.device = int(device)
        d.flags = int(flags)
        h = ctypes.c_void_p()
        _check(lib.pfc_plan_create(ctypes.byref(h), ctypes.byref(d)), "pfc_plan_create")
        self._h = h
        self._lib = lib
        self.r, self.dt = float(r), float(dt)
        self.shape = shape
        self.device = torch.device("cuda", int(device))
        self.real_dtype = torch.float64 if self.f64 else torch.float32
        self.complex_dtype = torch.complex128 if self.f64 else torch.complex64
        self.half_shape = shape[:-1] + (shape[-1] // 2 + 1,)
        # the native state is opaque: rows of a pitch >= n_x / 2 (3D grids pad rows to whole 128-byte
        # lines and may interleave blocks of z planes); its size comes from the library
        cbytes = 16 if self.f64 else 8
        rows = math.prod(shape[:-1])
        self.state_shape = shape[:-1] + (int(lib.pfc_plan_state_bytes(h)) // (cbytes * rows),)
        nbytes = lib.pfc_plan_workspace_bytes(h)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise PfcError(3, "Plan", "workspace tensor is not 256-byte aligned")
        _check(lib.pfc_plan_set_workspace(h, ctypes.c_void_p(self.workspace.data_ptr()), nbytes),
               "pfc_plan_set_workspace")

    # ---------------------------------------------------------------- helpers
    def _tensor(self, t, shape, dtype, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, plan is on {self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return ctypes.c_void_p(t.data_ptr())

    def empty_real(self):
        return _torch().empty(self.shape, dtype=self.real_dtype, device=self.device)

    def empty_half(self):
        return _torch().empty(self.half_shape, dtype=self.complex_dtype, device=self.device)

    @property
    def x_fused(self):
        """Whether step() fuses the x passes between steps (pfc_plan_x_fused)."""
        return bool(self._lib.pfc_plan_x_fused(self._h))

    def empty_state(self):
        return _torch().empty(self.state_shape, dtype=self.complex_dtype, device=self.device)

    # ---------------------------------------------------------------- entry points
    def fft_r2c(self, real, out=None):
        out = self.empty_half() if out is None else out
        _check(self._lib.pfc_fft_r2c(self._h, self._tensor(real, self.shape, self.real_dtype, "real_in"),
                                     self._tensor(out, self.half_shape, self.complex_dtype, "half_out"),
                                     _stream_ptr(self.device)), "pfc_fft_r2c")
        return out

    def fft_c2r(self, half, out=None):
        out = self.empty_real() if out is None else out
        _check(self._lib.pfc_fft_c2r(self._h, self._tensor(half, self.half_shape, self.complex_dtype, "half_in"),
                                     self._tensor(out, self.shape, self.real_dtype, "real_out"),
                                     _stream_ptr(self.device)), "pfc_fft_c2r")
        return out

    def state_init(self, psi0, state=None):
        state = self.empty_state() if state is None else state
        _check(self._lib.pfc_state_init(self._h, self._tensor(psi0, self.shape, self.real_dtype, "psi0"),
                                        self._tensor(state, self.state_shape, self.complex_dtype, "state"),
                                        _stream_ptr(self.device)), "pfc_state_init")
        return state

    def state_export(self, state, out=None):
        out = self.empty_half() if out is None else out
        _check(self._lib.pfc_state_export(self._h, self._tensor(state, self.state_shape, self.complex_dtype, "state"),
                                          self._tensor(out, self.half_shape, self.complex_dtype, "half_natural"),
                                          _stream_ptr(self.device)), "pfc_state_export")
        return out

    def step(self, psi, state, nsteps=1):
        _check(self._lib.pfc_step(self._h, self._tensor(psi, self.shape, self.real_dtype, "psi"),
                                  self._tensor(state, self.state_shape, self.complex_dtype, "state"),
                                  int(nsteps), _stream_ptr(self.device)), "pfc_step")
        return psi, state

    def step_noalloc(self, psi, state, nsteps=1):
        """pfc_step_noalloc: pfc_step with the library's static device scratch (no allocation)."""
        _check(self._lib.pfc_step_noalloc(self._h, self._tensor(psi, self.shape, self.real_dtype, "psi"),
                                          self._tensor(state, self.state_shape, self.complex_dtype, "state"),
                                          int(nsteps), _stream_ptr(self.device)), "pfc_step_noalloc")
        return psi, state

    def step_watched(self, psi, state, nsteps, check_every=50):
        """pfc_step_watched: raises PfcError (PFC_ERR_DIVERGED) on a non-finite energy; returns the
        number of steps run."""
        done = ctypes.c_int64(0)
        st = self._lib.pfc_step_watched(self._h, self._tensor(psi, self.shape, self.real_dtype, "psi"),
                                        self._tensor(state, self.state_shape, self.complex_dtype, "state"),
                                        int(nsteps), int(check_every), _stream_ptr(self.device), ctypes.byref(done))
        _check(st, f"pfc_step_watched (after {done.value} steps)")
        return done.value

    def step_timed(self, psi, state, nsteps=1):
        """pfc_step_timed: returns the summed milliseconds of each pass (list)."""
        ms = (ctypes.c_double * 5)()
        npass = ctypes.c_int(0)
        _check(self._lib.pfc_step_timed(self._h, self._tensor(psi, self.shape, self.real_dtype, "psi"),
                                        self._tensor(state, self.state_shape, self.complex_dtype, "state"),
                                        int(nsteps), _stream_ptr(self.device), ms, ctypes.byref(npass)),
               "pfc_step_timed")
        return [ms[i] for i in range(npass.value)]

    def step_backward(self, psi_n, psi_np1, lambda_np1, lambda_n=None, dLdr=None):
        torch = _torch()
        lambda_n = self.empty_real() if lambda_n is None else lambda_n
        if dLdr is None:
            dLdr = torch.zeros(1, dtype=torch.float64, device=self.device)
        if dLdr.dtype != torch.float64 or dLdr.device != self.device or dLdr.numel() < 1:
            raise ValueError("dLdr must be a float64 tensor with >= 1 element on the plan's device")
        _check(self._lib.pfc_step_backward(
            self._h, self._tensor(psi_n, self.shape, self.real_dtype, "psi_n"),
            self._tensor(psi_np1, self.shape, self.real_dtype, "psi_np1"),
            self._tensor(lambda_np1, self.shape, self.real_dtype, "lambda_np1"),
            self._tensor(lambda_n, self.shape, self.real_dtype, "lambda_n"),
            ctypes.c_void_p(dLdr.data_ptr()), _stream_ptr(self.device)), "pfc_step_backward")
        return lambda_n, dLdr

    def hydro_state_init(self, psi, v, psi_state=None, v_state=None):
        """States of the density and of the ndim velocity components (v: [ndim, *shape])."""
        torch = _torch()
        d = len(self.shape)
        psi_state = self.empty_state() if psi_state is None else psi_state
        v_state = (torch.empty((d,) + tuple(self.state_shape), dtype=self.complex_dtype, device=self.device)
                   if v_state is None else v_state)
        _check(self._lib.pfc_hydro_state_init(
            self._h, self._tensor(psi, self.shape, self.real_dtype, "psi"),
            self._tensor(psi_state, self.state_shape, self.complex_dtype, "psi_state"),
            self._tensor(v, (d,) + tuple(self.shape), self.real_dtype, "v"),
            self._tensor(v_state, (d,) + tuple(self.state_shape), self.complex_dtype, "v_state"),
            _stream_ptr(self.device)), "pfc_hydro_state_init")
        return psi_state, v_state

    def hydro_step(self, psi, psi_state, v, v_state, nsteps=1, rho0=1.0, gamma=1.0, a0=1.0, work=None):
        """nsteps hydrodynamic PFC steps, all four fields updated in place; `work` (uint8 device tensor
        of pfc_hydro_work_bytes) is allocated here when not given."""
        torch = _torch()
        d = len(self.shape)
        nbytes = int(self._lib.pfc_hydro_work_bytes(self._h))
        if work is None:
            work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        hp = HydroParams(float(rho0), float(gamma), float(a0))
        _check(self._lib.pfc_hydro_step(
            self._h, ctypes.byref(hp), self._tensor(psi, self.shape, self.real_dtype, "psi"),
            self._tensor(psi_state, self.state_shape, self.complex_dtype, "psi_state"),
            self._tensor(v, (d,) + tuple(self.shape), self.real_dtype, "v"),
            self._tensor(v_state, (d,) + tuple(self.state_shape), self.complex_dtype, "v_state"),
            ctypes.c_void_p(work.data_ptr()), ctypes.c_size_t(work.numel()), int(nsteps),
            _stream_ptr(self.device)), "pfc_hydro_step")
        return psi, psi_state, v, v_state

    def energy(self, psi, state, out=None):
        torch = _torch()
        out = torch.empty(2, dtype=torch.float64, device=self.device) if out is None else out
        if out.dtype != torch.float64 or out.device != self.device or out.numel() < 2:
            raise ValueError("out must be a float64 tensor with >= 2 elements on the plan's device")
        _check(self._lib.pfc_energy(self._h, self._tensor(psi, self.shape, self.real_dtype, "psi"),
                                    self._tensor(state, self.state_shape, self.complex_dtype, "state"),
                                    ctypes.c_void_p(out.data_ptr()), _stream_ptr(self.device)), "pfc_energy")
        return out

    # ---------------------------------------------------------------- autotuner
    def get_tuning(self):
        v = (ctypes.c_int * 5)()
        n = ctypes.c_int(0)
        _check(self._lib.pfc_plan_get_tuning(self._h, v, ctypes.byref(n)), "pfc_plan_get_tuning")
        return [v[i] for i in range(n.value)]

    def set_tuning(self, variants):
        v = (ctypes.c_int * 5)(*list(variants))
        _check(self._lib.pfc_plan_set_tuning(self._h, v, len(variants)), "pfc_plan_set_tuning")

    def tuning_key(self):
        arch = _torch().cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        return f"{arch}|{'x'.join(map(str, self.shape))}|{'f64' if self.f64 else 'f32'}"

    def autotune(self, reps=5, cache_path=None):
        """Pick the candidate schedules of the step passes by whole-step timing (pfc_plan_autotune,
        coordinate descent from the defaults) on scratch fields; with cache_path, reuse / record the
        choice in a JSON file keyed by GPU arch, shape and dtype.  Returns (variants, ms per pass of
        the choice, or None when taken from the cache)."""
        import json

        torch = _torch()
        key = self.tuning_key()
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
            if key in cache:
                self.set_tuning(cache[key]["variants"])
                return cache[key]["variants"], None
        g = torch.Generator(device=self.device).manual_seed(0)
        psi = (-0.3 + 0.2 * (torch.rand(self.shape, generator=g, device=self.device, dtype=torch.float64) - 0.5))
        psi = psi.to(self.real_dtype)
        state = self.state_init(psi)
        best = (ctypes.c_double * 5)()
        _check(self._lib.pfc_plan_autotune(self._h, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(state.data_ptr()),
                                           _stream_ptr(self.device), int(reps), best), "pfc_plan_autotune")
        variants = self.get_tuning()
        best_ms = [best[i] for i in range(len(variants))]
        if cache_path:
            cache[key] = {"variants": variants, "best_ms": best_ms}
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
        return variants, best_ms

    def set_params(self, r, dt):
        _check(self._lib.pfc_plan_set_params(self._h, float(r), float(dt)), "pfc_plan_set_params")
        self.r, self.dt = float(r), float(dt)

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.pfc_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Batch:
    """A pfc_batch: many independent 2D runs advanced together by one persistent launch.

    instances: list of dicts with the Plan keywords (shape, dtype, model, r, dt, dx, q1sq, R1, flags)."""

    def __init__(self, instances, device=0):
        torch = _torch()
        lib = load_library()
        self._lib = lib
        self.instances = [dict(i) for i in instances]
        descs = (PlanDesc * len(instances))()
        for k, inst in enumerate(self.instances):
            descs[k] = make_desc(device=device, **inst)
        h = ctypes.c_void_p()
        _check(lib.pfc_batch_create(ctypes.byref(h), descs, len(instances)), "pfc_batch_create")
        self._h = h
        self.device = torch.device("cuda", int(device))
        self.f64 = descs[0].dtype == PFC_F64
        self.real_dtype = torch.float64 if self.f64 else torch.float32
        self.complex_dtype = torch.complex128 if self.f64 else torch.complex64
        self.psi = self.state = None

    def bind(self, psis, states=None):
        """Attach the fields (psi[i]: real (n0, n1), state[i]: complex (n0, n1/2)); allocates states
        when not given, and the workspace."""
        torch = _torch()
        if states is None:
            states = [torch.empty(tuple(p.shape[:-1]) + (p.shape[-1] // 2,), dtype=self.complex_dtype,
                                  device=self.device) for p in psis]
        n = len(self.instances)
        if len(psis) != n or len(states) != n:
            raise ValueError("one psi and one state per instance")
        for k, (p, s_, inst) in enumerate(zip(psis, states, self.instances)):
            shp = tuple(inst["shape"])
            if tuple(p.shape) != shp or p.dtype != self.real_dtype or p.device != self.device or not p.is_contiguous():
                raise ValueError(f"psi[{k}] must be a contiguous {self.real_dtype} tensor of shape {shp}")
            sshp = shp[:-1] + (shp[-1] // 2,)
            if tuple(s_.shape) != sshp or s_.dtype != self.complex_dtype or not s_.is_contiguous():
                raise ValueError(f"state[{k}] must be a contiguous {self.complex_dtype} tensor of shape {sshp}")
        nbytes = self._lib.pfc_batch_workspace_bytes(self._h)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        pp = (ctypes.c_void_p * n)(*[p.data_ptr() for p in psis])
        sp = (ctypes.c_void_p * n)(*[s_.data_ptr() for s_ in states])
        _check(self._lib.pfc_batch_bind(self._h, pp, sp, ctypes.c_void_p(self.workspace.data_ptr()), nbytes),
               "pfc_batch_bind")
        self.psi, self.state = list(psis), list(states)
        return self

    @property
    def grid(self):
        return self._lib.pfc_batch_grid(self._h)

    def state_init(self):
        _check(self._lib.pfc_batch_state_init(self._h, _stream_ptr(self.device)), "pfc_batch_state_init")

    def step(self, nsteps):
        _check(self._lib.pfc_batch_step(self._h, int(nsteps), _stream_ptr(self.device)), "pfc_batch_step")

    def check(self):
        _check(self._lib.pfc_batch_check(self._h, _stream_ptr(self.device)), "pfc_batch_check")

    def get_tuning(self):
        n = 3 * len(self.instances)
        v = (ctypes.c_int * n)()
        _check(self._lib.pfc_batch_get_tuning(self._h, v, n), "pfc_batch_get_tuning")
        return [list(v[3 * i:3 * i + 3]) for i in range(len(self.instances))]

    def set_tuning(self, per_instance):
        flat = [int(x) for t in per_instance for x in t]
        v = (ctypes.c_int * len(flat))(*flat)
        _check(self._lib.pfc_batch_set_tuning(self._h, v, len(flat)), "pfc_batch_set_tuning")

    def tuning_key(self):
        arch = _torch().cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        dt = "f64" if self.f64 else "f32"
        return arch + "|batch|" + dt + "|" + ",".join("x".join(map(str, i["shape"])) for i in self.instances)

    def autotune(self, steps=5, cache_path=None):
        """Choose candidate schedules per pass and length (pfc_batch_autotune) on a scratch batch with
        the same instances, then apply the choice here.  With cache_path, reuse / record it in a JSON
        file.  Returns (per-instance variants, ms per step of the choice or None from the cache)."""
        import json

        torch = _torch()
        key = self.tuning_key()
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
            if key in cache:
                self.set_tuning(cache[key]["variants"])
                return cache[key]["variants"], None
        scratch = Batch(self.instances, device=self.device.index)
        g = torch.Generator(device=self.device).manual_seed(0)
        psis = [(i["r"] + 0.2 * (torch.rand(tuple(i["shape"]), generator=g, device=self.device,
                                            dtype=torch.float64) - 0.5)).to(self.real_dtype) for i in self.instances]
        scratch.bind(psis)
        scratch.state_init()
        ms = ctypes.c_double(0.0)
        _check(self._lib.pfc_batch_autotune(scratch._h, _stream_ptr(self.device), int(steps), ctypes.byref(ms)),
               "pfc_batch_autotune")
        variants = scratch.get_tuning()
        scratch.destroy()
        self.set_tuning(variants)
        if cache_path:
            cache[key] = {"variants": variants, "ms_per_step": ms.value}
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
        return variants, ms.value

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.pfc_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class HydroParams(ctypes.Structure):
    """pfc_hydro_params: mass density, viscosity, width of the Gaussian average."""

    _fields_ = [("rho0", ctypes.c_double), ("gamma", ctypes.c_double), ("a0", ctypes.c_double)]


# Module-level functions with the C names (same arguments, Plan in place of the handle).
def pfc_plan_create(shape, **kw) -> Plan:
    return Plan(shape, **kw)


def pfc_plan_destroy(plan: Plan):
    plan.destroy()


def pfc_plan_set_params(plan: Plan, r, dt):
    plan.set_params(r, dt)


def pfc_fft_r2c(plan: Plan, real_in, half_out=None):
    return plan.fft_r2c(real_in, half_out)


def pfc_fft_c2r(plan: Plan, half_in, real_out=None):
    return plan.fft_c2r(half_in, real_out)


def pfc_state_init(plan: Plan, psi0, state=None):
    return plan.state_init(psi0, state)


def pfc_state_export(plan: Plan, state, half_natural=None):
    return plan.state_export(state, half_natural)


def pfc_step(plan: Plan, psi, state, nsteps=1):
    return plan.step(psi, state, nsteps)


def pfc_step_timed(plan: Plan, psi, state, nsteps=1):
    return plan.step_timed(psi, state, nsteps)


def pfc_step_backward(plan: Plan, psi_n, psi_np1, lambda_np1, lambda_n=None, dLdr=None):
    return plan.step_backward(psi_n, psi_np1, lambda_np1, lambda_n, dLdr)


def pfc_energy(plan: Plan, psi, state, out=None):
    return plan.energy(psi, state, out)


def pfc_hydro_state_init(plan: Plan, psi, v, psi_state=None, v_state=None):
    return plan.hydro_state_init(psi, v, psi_state, v_state)


def pfc_hydro_step(plan: Plan, psi, psi_state, v, v_state, nsteps=1, rho0=1.0, gamma=1.0, a0=1.0, work=None):
    return plan.hydro_step(psi, psi_state, v, v_state, nsteps, rho0, gamma, a0, work)


class Apfc:
    """A pfc_apfc object (complex-amplitude form) with its workspace (a torch uint8 tensor).
    Fields and spectra are complex tensors of shape (N, *shape)."""

    def __init__(self, shape, kvec, dtype="f32", dx=math.pi / 2, dB=-0.15, Bx=1.0, t=0.0, v=1.0, dt=0.5, device=0):
        torch = _torch()
        lib = load_library()
        shape = tuple(int(s) for s in shape)
        kvec = [[float(c) for c in row] for row in kvec]
        d = ApfcDesc()
        d.ndim = len(shape)
        dxs = tuple(dx) if isinstance(dx, (tuple, list)) else (dx,) * len(shape)
        for a in range(3):
            d.n[a] = shape[a] if a < len(shape) else 1
            d.dx[a] = float(dxs[a]) if a < len(shape) else 1.0
        self.f64 = dtype in ("f64", "float64", PFC_F64)
        d.dtype = PFC_F64 if self.f64 else PFC_F32
        if not 1 <= len(kvec) <= APFC_MAX_FIELDS:
            raise ValueError(f"need 1..{APFC_MAX_FIELDS} wave vectors")
        d.nfields = len(kvec)
        for j, row in enumerate(kvec):
            if len(row) != len(shape):
                raise ValueError("each wave vector needs one component per grid axis")
            for a, c in enumerate(row):
                d.k[j][a] = c
        d.dB, d.Bx, d.t, d.v, d.dt = float(dB), float(Bx), float(t), float(v), float(dt)
        d.device = int(device)
        h = ctypes.c_void_p()
        _check(lib.pfc_apfc_create(ctypes.byref(h), ctypes.byref(d)), "pfc_apfc_create")
        self._h, self._lib = h, lib
        self.shape = shape
        self.nfields = len(kvec)
        self.field_shape = (self.nfields,) + shape
        self.device = torch.device("cuda", int(device))
        self.complex_dtype = torch.complex128 if self.f64 else torch.complex64
        nbytes = lib.pfc_apfc_workspace_bytes(h)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise PfcError(3, "Apfc", "workspace tensor is not 256-byte aligned")
        _check(lib.pfc_apfc_set_workspace(h, ctypes.c_void_p(self.workspace.data_ptr()), nbytes),
               "pfc_apfc_set_workspace")

    def _fields(self, x, name):
        torch = _torch()
        if not isinstance(x, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if x.device != self.device or x.dtype != self.complex_dtype:
            raise TypeError(f"{name} must be {self.complex_dtype} on {self.device}")
        if tuple(x.shape) != self.field_shape or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous tensor of shape {self.field_shape}")
        return ctypes.c_void_p(x.data_ptr())

    def empty(self):
        return _torch().empty(self.field_shape, dtype=self.complex_dtype, device=self.device)

    def terms(self, j):
        np_, nt_ = ctypes.c_int(), ctypes.c_int()
        _check(self._lib.pfc_apfc_terms(self._h, int(j), ctypes.byref(np_), ctypes.byref(nt_)), "pfc_apfc_terms")
        return np_.value, nt_.value

    def fft(self, x, dir=-1, out=None):
        out = self.empty() if out is None else out
        _check(self._lib.pfc_apfc_fft(self._h, self._fields(x, "in"), self._fields(out, "out"), int(dir),
                                      _stream_ptr(self.device)), "pfc_apfc_fft")
        return out

    def nonlinear(self, eta, out=None):
        out = self.empty() if out is None else out
        _check(self._lib.pfc_apfc_nonlinear(self._h, self._fields(eta, "eta"), self._fields(out, "out"),
                                            _stream_ptr(self.device)), "pfc_apfc_nonlinear")
        return out

    def state_init(self, eta, eta_hat=None):
        eta_hat = self.empty() if eta_hat is None else eta_hat
        _check(self._lib.pfc_apfc_state_init(self._h, self._fields(eta, "eta"), self._fields(eta_hat, "eta_hat"),
                                             _stream_ptr(self.device)), "pfc_apfc_state_init")
        return eta_hat

    def step(self, eta, eta_hat, nsteps=1):
        _check(self._lib.pfc_apfc_step(self._h, self._fields(eta, "eta"), self._fields(eta_hat, "eta_hat"),
                                       int(nsteps), _stream_ptr(self.device)), "pfc_apfc_step")
        return eta, eta_hat

    def destroy(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.pfc_apfc_destroy(h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def pfc_apfc_create(shape, kvec, **kw) -> Apfc:
    return Apfc(shape, kvec, **kw)


def pfc_apfc_state_init(obj: Apfc, eta, eta_hat=None):
    return obj.state_init(eta, eta_hat)


def pfc_apfc_step(obj: Apfc, eta, eta_hat, nsteps=1):
    return obj.step(eta, eta_hat, nsteps)


def pfc_apfc_fft(obj: Apfc, x, dir=-1, out=None):
    return obj.fft(x, dir, out)


def pfc_apfc_nonlinear(obj: Apfc, eta, out=None):
    return obj.nonlinear(eta, out)
