"""Parity at the full sizes of the 3D runs, where the FP64 oracle cannot run the whole case.

* 2048^3 FP32 (r = -0.30, dt = 0.5, psi0 seed 3): a field made of 8 x 8 x 8 copies of a 256^3 field
  stays tiled under the step (the spectrum lives on every 8th wavenumber, where q is the same as on
  the 256^3 grid), so the 2048^3 run must equal the tiled 256^3 run; the 256^3 run is compared with
  the oracle.  Both GPU runs are FP32 with different FFT lengths, so they agree to FP32 rounding
  amplified over the steps (bounded below).
* 256^3 (r = -0.30, dt = 0.5, psi0 seed 2): FP64 and FP32 against the oracle after 100 steps (the
  gates: 1e-12 FP64, 1e-4 FP32, on the plain and mean-removed relative L2 and the element-wise
  error); then 1000 FP64 steps with the energy checked at every 50th step (non-increasing while the sufficient
  condition holds) and the FP32 run against the FP64 run at step 1000."""
import math

import numpy as np
import pytest

import oracle
import pfc_inputs as P
from gpu_common import TOL_STEP, fmt_errs, parity_err, parity_errs, rounded, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pfc():
    import paper_2603_26818_amd as m

    m.load_library()
    return m


def test_2048_cube_tiled_equals_256_cube(pfc):
    import torch

    n, m, steps = 2048, 256, 20
    say(f"[fullsize] 2048^3 FP32 tiled from 256^3, {steps} steps")
    g = rounded(P.pfc_initial_field(3, (m, m, m), -0.30), "f32")
    ps = pfc.Plan((m, m, m), dtype="f32", r=-0.30, dt=0.5)
    xs = to_dev(g, "f32")
    ss = ps.state_init(xs)
    ps.step(xs, ss, steps)
    p = oracle.Params((m, m, m), r=-0.30, dt=0.5)
    ref, _ = oracle.step(p, g, oracle.state_init(p, g), steps)
    e_small = parity_err(to_np(xs), ref)
    say(f"           256^3 vs oracle: rel L2 {e_small:.2e}")
    assert e_small < TOL_STEP["f32"]
    pb = pfc.Plan((n, n, n), dtype="f32", r=-0.30, dt=0.5)
    xb = to_dev(g, "f32").repeat(8, 8, 8)
    sb = pb.state_init(xb)
    pb.step(xb, sb, steps)
    torch.cuda.synchronize()
    num = 0.0
    for k in range(8):  # compare one z-slab of copies at a time
        blk = xb[k * m:(k + 1) * m].view(m, 8, m, 8, m)
        d = (blk - xs.view(m, 1, m, 1, m)).double()
        num += float(torch.sum(d * d))
        del blk, d
    e_big = math.sqrt(num / 512) / float(torch.linalg.vector_norm(xs.double()))
    F = pb.energy(xb, sb).cpu().tolist()
    Fs = ps.energy(xs, ss).cpu().tolist()
    say(f"           2048^3 vs tiled 256^3: rel L2 {e_big:.2e}; energy {F[0]:.8e} vs 512 x {Fs[0]:.8e}")
    assert e_big < 1e-5
    assert abs(F[0] - 512 * Fs[0]) < 1e-5 * abs(F[0])
    del xb, sb, pb


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_256_cube_vs_oracle(pfc, dtype):
    shape, steps = (256, 256, 256), 100
    say(f"[fullsize] 256^3 {dtype} vs oracle, {steps} steps")
    psi0 = rounded(P.pfc_initial_field(2, shape, -0.30), dtype)
    p = oracle.Params(shape, r=-0.30, dt=0.5)
    ref, refS = oracle.step(p, psi0, oracle.state_init(p, psi0), steps)
    plan = pfc.Plan(shape, dtype=dtype, r=-0.30, dt=0.5)
    x = to_dev(psi0, dtype)
    s = plan.state_init(x)
    plan.step(x, s, steps)
    errs = parity_errs(to_np(x), ref)
    F = plan.energy(x, s).cpu().tolist()
    Fr = oracle.energy(p, ref, refS)
    say(f"           psi {fmt_errs(errs)}; energy {F[0]:.12g} vs {Fr[0]:.12g}")
    assert max(errs) < TOL_STEP[dtype] and abs(F[0] - Fr[0]) < TOL_STEP[dtype] * abs(Fr[0])


def test_256_cube_1000_steps_energy_and_fp32(pfc):
    import torch

    shape, steps, every = (256, 256, 256), 1000, 50
    say(f"[fullsize] 256^3 FP64 {steps} steps, energy every {every}; FP32 against FP64")
    psi0 = rounded(P.pfc_initial_field(2, shape, -0.30), "f32")  # the same start for both precisions
    q = None
    p64 = pfc.Plan(shape, dtype="f64", r=-0.30, dt=0.5)
    p32 = pfc.Plan(shape, dtype="f32", r=-0.30, dt=0.5)
    x64, x32 = to_dev(psi0, "f64"), to_dev(psi0, "f32")
    s64, s32 = p64.state_init(x64), p32.state_init(x32)
    # sufficient condition for a non-increasing energy: min_{q>0} [2/(dt q) + r + L(q)] >= 3 max|psi|^2
    qmax = 3 * (math.pi / (math.pi / 4)) ** 2
    qs = np.linspace(qmax / 1e5, qmax, 200001)
    bound = float(np.min(2.0 / (0.5 * qs) - 0.30 + (1 - qs) ** 2))
    F_prev = p64.energy(x64, s64).cpu().tolist()[0]
    checked = 0
    for k in range(steps // every):
        m0 = float(x64.abs().max())
        p64.step(x64, s64, every)
        p32.step(x32, s32, every)
        F = p64.energy(x64, s64).cpu().tolist()[0]
        m1 = float(x64.abs().max())
        assert math.isfinite(F)
        if bound >= 3 * max(m0, m1) ** 2:
            assert F <= F_prev + 1e-12 * abs(F_prev), (k, F, F_prev)
            checked += 1
        F_prev = F
    e = float(torch.linalg.vector_norm((x32.double() - x64)) / torch.linalg.vector_norm(x64))
    say(f"           energy non-increasing at {checked}/{steps // every} checks (bound {bound:.3f}, "
        f"max|psi| {float(x64.abs().max()):.3f}); FP32 vs FP64 at step {steps}: rel L2 {e:.2e}")
    assert checked >= 10
    assert e < 1e-3


def test_512_cube_bench_workload_vs_oracle(pfc):
    """The benchmark's headline workload itself: 512^3 FP32, r = -0.30, dt = 0.5, dx = pi/4, psi0
    seed 23, drawn on the device as the benchmark draws it, the plan launched as the benchmark
    launches it; 3 steps and one r2c against the FP64 oracle on the same (FP32-rounded) field."""
    import torch

    shape, r = (512, 512, 512), -0.30
    say("[fullsize] 512^3 FP32 bench workload: 3 steps and one r2c vs the oracle")
    psi = P.pfc_initial_field_torch(23, shape, r, torch.float32, "cuda:0")
    psi0 = to_np(psi)
    plan = pfc.Plan(shape, dtype="f32", r=r, dt=0.5)
    half = to_np(plan.fft_r2c(psi))
    ref_half = oracle.rfftn(psi0)
    e_fft = parity_errs(half, ref_half)
    del half
    state = plan.state_init(psi)
    plan.step(psi, state, 3)
    got = to_np(psi)
    del psi, state, plan
    torch.cuda.empty_cache()
    p = oracle.Params(shape, r=r, dt=0.5)
    ref, _ = oracle.step(p, psi0, oracle.state_init(p, psi0), 3)
    e = parity_errs(got, ref)
    say(f"      r2c {fmt_errs(e_fft)}; psi after 3 steps {fmt_errs(e)}")
    assert max(e_fft) < 5e-6 and max(e) < 1e-5
