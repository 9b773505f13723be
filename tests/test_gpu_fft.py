"""GPU parity of the r2c / c2r transforms (pfc_fft_r2c, pfc_fft_c2r) against the FP64 oracle.

The oracle's DFT is pinned in test_oracle_pins.py.  Shapes span 2D and 3D, cubic and non-cubic
grids, several workgroup tiles and the smallest sizes, FP32 and FP64."""
import numpy as np
import pytest

import oracle
import pfc_inputs as P
from gpu_common import TOL_FFT, parity_err, rounded, say, to_dev, to_np

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4), (8, 8), (16, 64), (64, 16), (128, 128), (256, 32), (4, 4, 4), (8, 8, 8), (16, 8, 32), (4, 16, 8),
          (32, 32, 32), (64, 64, 64), (128, 64, 32), (32, 256, 16), (1024, 32, 32), (2048, 16, 32),
          # long x rows (256, 512 and 1024 packed points: the padded LDS rows of the x r2c)
          (4, 4, 512), (8, 1024), (4, 2048)]


@pytest.fixture(scope="module")
def pfc():
    import paper_2603_26818_amd as m

    m.load_library()
    return m


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_r2c_c2r_vs_oracle(pfc, shape, dtype):
    say(f"[fft] shape={shape} dtype={dtype} seed=21")
    x = rounded(P.normal(21, shape), dtype)
    plan = pfc.Plan(shape, dtype=dtype)
    X = plan.fft_r2c(to_dev(x, dtype))
    ref = oracle.rfftn(x)
    e_fwd = parity_err(to_np(X), ref)
    # c2r of the oracle's spectrum (exactly Hermitian planes) against the oracle's c2r
    import torch

    H = torch.from_numpy(ref).to("cuda:0", plan.complex_dtype)
    y = plan.fft_c2r(H)
    e_inv = parity_err(to_np(y), oracle.irfftn(ref, shape))
    say(f"      r2c rel L2 {e_fwd:.2e}   c2r rel L2 {e_inv:.2e}")
    assert e_fwd < TOL_FFT[dtype] and e_inv < TOL_FFT[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c2r_projects_self_conjugate_planes(pfc, dtype):
    """Anti-Hermitian content in the kx = 0 and kx = n/2 planes is discarded, as in the oracle."""
    shape = (16, 8, 32)
    say(f"[fft] c2r projection shape={shape} dtype={dtype}")
    rng_re, rng_im = P.normal(31, shape[:-1] + (17,)), P.normal(32, shape[:-1] + (17,))
    H = rng_re + 1j * rng_im  # not Hermitian anywhere
    if dtype == "f32":
        H = H.astype(np.complex64).astype(np.complex128)
    plan = pfc.Plan(shape, dtype=dtype)
    import torch

    y = plan.fft_c2r(torch.from_numpy(H).to("cuda:0", plan.complex_dtype))
    e = parity_err(to_np(y), oracle.irfftn(H, shape))
    say(f"      rel L2 {e:.2e}")
    assert e < TOL_FFT[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_single_mode_exact(pfc, dtype):
    shape = (32, 16, 64)
    say(f"[fft] single mode shape={shape} dtype={dtype}")
    m = (5, 3, 7)
    g = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    x = np.cos(sum(2 * np.pi * mi * gi / n for mi, gi, n in zip(m, g, shape)))
    plan = pfc.Plan(shape, dtype=dtype)
    X = to_np(plan.fft_r2c(to_dev(x, dtype)))
    expect = np.zeros_like(X)
    expect[m] = np.prod(shape) / 2
    tol = (1e-13 if dtype == "f64" else 2e-6) * np.prod(shape)
    assert np.abs(X - expect).max() < tol


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [256, 512])
def test_roundtrip_full_size(pfc, n, dtype):
    """Standalone 3D r2c -> c2r round trip on seeded N(0,1) fields (seed 21 at 256^3, 22 at 512^3),
    plus Parseval, at the full sizes."""
    import torch

    import pfc_inputs

    shape = (n, n, n)
    seed = 21 if n == 256 else 22
    say(f"[fft] round trip shape={shape} dtype={dtype} seed={seed}")
    plan = pfc.Plan(shape, dtype=dtype)
    x = pfc_inputs.normal_torch(seed, shape, plan.real_dtype, "cuda:0")
    X = plan.fft_r2c(x)
    y = plan.fft_c2r(X)
    torch.cuda.synchronize()
    e = (torch.linalg.vector_norm((y - x).double()) / torch.linalg.vector_norm(x.double())).item()
    # Parseval with half-spectrum weights (computed in FP64 from the GPU spectrum)
    w = torch.full((n // 2 + 1,), 2.0, dtype=torch.float64, device="cuda:0")
    w[0] = 1.0
    w[-1] = 1.0
    lhs = torch.sum(x.double() ** 2).item()
    rhs = (torch.sum(w * X.abs().double() ** 2) / n**3).item()
    say(f"      round trip rel L2 {e:.2e}, Parseval rel {abs(lhs - rhs) / lhs:.2e}")
    tol = 1e-14 if dtype == "f64" else 1e-6
    assert e < tol * 10 and abs(lhs - rhs) / lhs < tol * 10


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_512_spectrum_of_tiled_field_vs_oracle(pfc, dtype):
    """A 512^3 field made of 4x4x4 copies of a 128^3 field g has spectrum 64 G(k/4) at indices that
    are multiples of 4 on every axis and zero elsewhere.  G comes from the oracle at 128^3."""
    import torch

    n, m = 512, 128
    say(f"[fft] tiled 512^3 vs oracle 128^3, dtype={dtype}")
    g = rounded(P.normal(23, (m, m, m)), dtype)
    G = oracle.rfftn(g)
    plan = pfc.Plan((n, n, n), dtype=dtype)
    x = to_dev(g, dtype).repeat(4, 4, 4)
    X = plan.fft_r2c(x)
    sub = to_np(X[::4, ::4, ::4])
    e = parity_err(sub, 64 * G)
    off = X.clone()
    off[::4, ::4, ::4] = 0
    leak = (off.abs().max() / X.abs().max()).item()
    say(f"      rel L2 on the lattice {e:.2e}, max off-lattice {leak:.2e}")
    assert e < TOL_FFT[dtype] and leak < (1e-13 if dtype == "f64" else 1e-5)
