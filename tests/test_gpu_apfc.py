"""Complex-amplitude form on the GPU against the FP64 oracle (equations in pfc_oracle.c, pinned in
test_oracle_apfc.py): batched complex FFTs of all amplitudes, the resonant nonlinearity, and the
semi-implicit step, in 2D and 3D, FP32 and FP64, on power-of-two and mixed-radix grids (x rows of
6 to 2048 points, y and last-axis pencils of 6 to 2048 points, including the spread and grouped
tiles of the 1024-, 1400- and 2048-point pencils); then the benchmark workload (6 bcc amplitudes
on 256^3, FP32) stepped against the oracle, and a uniform crystal relaxing to its equilibrium
amplitude on a 2048^2 grid."""
import numpy as np
import pytest

import oracle
import pfc_inputs as P
from gpu_common import TOL_FFT, TOL_STEP, parity_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pfc():
    import paper_2603_26818_amd as m

    m.load_library()
    return m


def cdev(x, dtype):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to(
        device="cuda:0", dtype=torch.complex64 if dtype == "f32" else torch.complex128)


def chost(t):
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def crounded(x, dtype):
    return x.astype(np.complex64).astype(np.complex128) if dtype == "f32" else x


FFT_SHAPES = [(32, 64), (64, 16), (16, 32, 8), (8, 16, 64), (30, 20, 12), (750, 20), (6, 10, 14), (4, 8, 2048),
              (2048, 4, 8), (1024, 6, 10), (1400, 4, 6), (10, 1400)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", FFT_SHAPES)
def test_apfc_fft_vs_oracle(pfc, shape, dtype):
    nf = 3
    say(f"[apfc fft] shape={shape} dtype={dtype} fields={nf} seed=81")
    k = P.lattice_vectors("triangular") if len(shape) == 2 else P.lattice_vectors("bcc")[:nf]
    x = crounded(P.amplitude_fields(81, nf, shape, 0.0, 1.0), dtype)
    obj = pfc.Apfc(shape, k, dtype=dtype)
    xd = cdev(x, dtype)
    X = chost(obj.fft(xd, -1))
    Xin = chost(obj.fft(xd, -1, out=xd))  # in place: the same bits as out of place
    assert np.array_equal(X, Xin)
    ref = np.stack([oracle.fft_c2c(x[j], -1) for j in range(nf)])
    e_fwd = parity_err(X, ref)
    y = chost(obj.fft(cdev(ref, dtype), +1))
    e_inv = parity_err(y, x)
    say(f"      forward rel L2 {e_fwd:.2e}  inverse {e_inv:.2e}")
    assert e_fwd < TOL_FFT[dtype] and e_inv < TOL_FFT[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("lattice,shape", [("triangular", (16, 32)), ("square", (8, 64)), ("triangular2", (30, 20)),
                                           ("bcc", (8, 16, 32)), ("fcc2", (6, 10, 12)), ("triangular30", (8, 16)),
                                           ("triangular32", (8, 16))])
def test_apfc_nonlinearity_vs_oracle(pfc, lattice, shape, dtype):
    k = P.lattice_vectors(lattice)
    say(f"[apfc nonlinear] {lattice} shape={shape} dtype={dtype} seed=82")
    eta = crounded(P.amplitude_fields(82, len(k), shape, 0.1, 0.3), dtype)
    obj = pfc.Apfc(shape, k, dtype=dtype, t=0.35, v=0.8, dt=0.1)  # dt only has to pass validation here
    got = chost(obj.nonlinear(cdev(eta, dtype)))
    ref = oracle.apfc_nonlinear(oracle.Apfc(shape, k, t=0.35, v=0.8), eta)
    e = parity_err(got, ref)
    say(f"      rel L2 {e:.2e}")
    assert e < (1e-14 if dtype == "f64" else 1e-6)


STEP_CASES = [
    # (lattice, shape, dtype, nsteps, seed)
    ("triangular", (64, 64), "f64", 100, 83),
    ("triangular", (64, 64), "f32", 100, 83),
    ("triangular2", (32, 60), "f64", 60, 84),
    ("square", (128, 32), "f32", 60, 85),
    ("bcc", (32, 32, 32), "f64", 30, 86),
    ("bcc", (16, 32, 64), "f32", 30, 87),
    ("fcc2", (30, 20, 12), "f64", 30, 88),
    ("bcc", (2048, 4, 8), "f32", 5, 89),
    ("bcc", (2048, 32, 64), "f32", 2, 95),  # 768 pencil tiles: the full-width 2048-point tile
    ("bcc", (1024, 6, 10), "f32", 5, 90),
    ("bcc", (1400, 4, 6), "f32", 5, 91),
    ("bcc", (1400, 4, 6), "f64", 5, 91),
    ("triangular", (10, 1400), "f64", 10, 92),
    # tens of coupled amplitudes: 30 and 32 (the maximum) triangular reciprocal vectors, |k| up to 4.4
    ("triangular30", (16, 32), "f64", 10, 93),
    ("triangular30", (16, 32), "f32", 10, 93),
    ("triangular32", (12, 20), "f64", 6, 94),
]


def _many(lattice):
    return lattice.startswith("triangular3")


def _params(lattice):
    # coefficients of a crystal that relaxes (dB < 0), with the resonant quadratic term on; with
    # 30 or more amplitudes (thousands of resonant triples per field) the explicit nonlinearity needs
    # small amplitudes and dt = 0.1 to stay bounded
    return dict(dB=-0.15, Bx=1.0, t=0.3, v=1.0, dt=0.1 if _many(lattice) else 0.5)


def _initial(seed, lattice, nf, shape, dtype):
    mean, amp = (0.01, 0.005) if _many(lattice) else (0.1, 0.05)
    return crounded(P.amplitude_fields(seed, nf, shape, mean, amp), dtype)


@pytest.mark.parametrize("lattice,shape,dtype,nsteps,seed", STEP_CASES)
def test_apfc_step_vs_oracle(pfc, lattice, shape, dtype, nsteps, seed):
    k = P.lattice_vectors(lattice)
    say(f"[apfc step] {lattice} shape={shape} dtype={dtype} nsteps={nsteps} seed={seed}")
    kw = _params(lattice)
    eta0 = _initial(seed, lattice, len(k), shape, dtype)
    obj = pfc.Apfc(shape, k, dtype=dtype, **kw)
    eta = cdev(eta0, dtype)
    S = obj.state_init(eta)
    obj.step(eta, S, nsteps)
    a = oracle.Apfc(shape, k, **kw)
    ref_eta, ref_S = oracle.apfc_step(a, eta0, oracle.apfc_state_init(a, eta0), nsteps)
    e, eS = parity_err(chost(eta), ref_eta), parity_err(chost(S), ref_S)
    change = parity_err(eta0, ref_eta)
    say(f"      eta rel L2 {e:.2e}  spectra {eS:.2e}  (change over the run {change:.2e})")
    assert change > 1e-3  # the run moves the fields
    assert e < TOL_STEP[dtype] and eS < TOL_STEP[dtype]


def test_apfc_bench_workload_vs_oracle(pfc):
    """The benchmark workload: 6 bcc amplitudes on 256^3, FP32, in the benchmark's launch
    configuration, two steps against the FP64 oracle (all 100M complex values compared)."""
    import torch

    shape, k = (256, 256, 256), P.lattice_vectors("bcc")
    kw = _params("bcc")
    say("[apfc 256^3 bcc] FP32, 2 steps vs the oracle")
    eta = P.amplitude_fields_torch(7, 6, shape, 0.1, torch.complex64, "cuda:0", 0.05)
    eta0 = chost(eta)
    obj = pfc.Apfc(shape, k, dtype="f32", **kw)
    S = obj.state_init(eta)
    obj.step(eta, S, 2)
    got = chost(eta)
    del eta, S
    a = oracle.Apfc(shape, k, **kw)
    ref, _ = oracle.apfc_step(a, eta0, oracle.apfc_state_init(a, eta0), 2)
    e = parity_err(got, ref)
    say(f"      eta rel L2 {e:.2e}")
    assert e < 1e-5


def test_apfc_uniform_crystal_equilibrium_at_2048sq(pfc):
    """Uniform real amplitudes on a 2048^2 triangular grid relax to
    phi* = (t + sqrt(t^2 - 15 v dB)) / (15 v) at every point (FP64)."""
    import torch

    dB, t, v = 0.02, 0.5, 1.0 / 3.0
    shape = (2048, 2048)
    say("[apfc 2048^2 equilibrium] FP64, 450 steps")
    obj = pfc.Apfc(shape, P.lattice_vectors("triangular"), dtype="f64", dB=dB, t=t, v=v, dt=0.5)
    eta = torch.full((3,) + shape, 0.1, dtype=torch.complex128, device="cuda:0")
    S = obj.state_init(eta)
    obj.step(eta, S, 450)
    phi = (t + np.sqrt(t * t - 15 * v * dB)) / (15 * v)
    err = float((eta - phi).abs().max())
    say(f"      max |eta - phi*| {err:.2e}")
    assert err < 1e-12
