"""Grids whose lengths have factors 3, 5 and 7 (the paper's grids 750^3 and 1400^3 are of this
kind: 750 = 2 3 5^3).  GPU transforms and PFC steps against the FP64 oracle, whose mixed-radix
recursion is pinned in test_oracle_pins.py.  Shapes cover every compiled non-power-of-two length on
each pass kind (x half-lengths 6, 10, 14, 15, 375, 700; y and last-axis lengths 6, 10, 12, 14, 20,
30, 60, 150, 700, 750, 1400), partial column tiles (M = 375 is not a multiple of the 16-column tile), 2D and 3D,
FP32 and FP64; then one step at 750^3, the paper's smaller 3D grid."""
import numpy as np
import pytest

import oracle
import pfc_inputs as P
from gpu_common import TOL_FFT, TOL_STEP, parity_err, rounded, say, to_dev, to_np

pytestmark = pytest.mark.gpu

FFT_SHAPES = [(30, 20, 12), (14, 10, 28), (750, 6, 20), (10, 750, 12), (6, 10, 750), (150, 60, 30), (12, 14, 20),
              (750, 20), (20, 750), (60, 300), (30, 28),
              # 1400 and 700: 50 threads per pencil, stages of 14, 10, 10 (or 7, 10, 10) butterflies
              # that do not divide evenly among the threads
              (1400, 6, 20), (10, 1400, 12), (6, 10, 1400), (700, 12, 20), (1400, 20), (20, 1400)]
STEP_CASES = [
    # (shape, dtype, nsteps, seed)
    ((30, 20, 12), "f64", 40, 41),
    ((30, 20, 12), "f32", 40, 41),
    ((14, 10, 28), "f64", 30, 42),
    ((750, 6, 20), "f64", 20, 43),
    ((750, 6, 20), "f32", 20, 43),
    ((6, 10, 750), "f64", 20, 44),
    ((10, 750, 12), "f32", 20, 45),
    ((150, 60, 30), "f64", 20, 46),
    ((750, 20), "f64", 40, 47),
    ((20, 750), "f32", 40, 48),
    ((60, 300), "f64", 40, 49),
    ((1400, 6, 20), "f64", 20, 54),
    ((1400, 6, 20), "f32", 20, 54),
    ((6, 10, 1400), "f64", 20, 55),
    ((10, 1400, 12), "f32", 20, 56),
    ((20, 1400), "f64", 30, 57),
    ((1400, 20), "f32", 30, 58),
]


@pytest.fixture(scope="module")
def pfc():
    import paper_2603_26818_amd as m

    m.load_library()
    return m


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", FFT_SHAPES)
def test_mixed_r2c_c2r_vs_oracle(pfc, shape, dtype):
    import torch

    say(f"[mixed fft] shape={shape} dtype={dtype} seed=51")
    x = rounded(P.normal(51, shape), dtype)
    plan = pfc.Plan(shape, dtype=dtype)
    ref = oracle.rfftn(x)
    e_fwd = parity_err(to_np(plan.fft_r2c(to_dev(x, dtype))), ref)
    y = plan.fft_c2r(torch.from_numpy(ref).to("cuda:0", plan.complex_dtype))
    e_inv = parity_err(to_np(y), oracle.irfftn(ref, shape))
    say(f"      r2c rel L2 {e_fwd:.2e}   c2r rel L2 {e_inv:.2e}")
    assert e_fwd < TOL_FFT[dtype] and e_inv < TOL_FFT[dtype]


@pytest.mark.parametrize("shape,dtype,nsteps,seed", STEP_CASES)
def test_mixed_step_vs_oracle(pfc, shape, dtype, nsteps, seed):
    say(f"[mixed step] shape={shape} dtype={dtype} nsteps={nsteps} seed={seed}")
    r = -0.30 if len(shape) == 3 else -0.25
    psi0 = rounded(P.pfc_initial_field(seed, shape, r), dtype)
    plan = pfc.Plan(shape, dtype=dtype, r=r, dt=0.5)
    psi = to_dev(psi0, dtype)
    state = plan.state_init(psi)
    plan.step(psi, state, nsteps)
    F = to_np(plan.energy(psi, state))
    p = oracle.Params(shape, r=r, dt=0.5)
    ref_psi, ref_state = oracle.step(p, psi0, oracle.state_init(p, psi0), nsteps)
    ref_F = oracle.energy(p, ref_psi, ref_state)
    e = parity_err(to_np(psi), ref_psi)
    es = parity_err(to_np(plan.state_export(state)), ref_state)
    eF = abs(F[0] - ref_F[0]) / abs(ref_F[0])
    say(f"      psi rel L2 {e:.2e}  state {es:.2e}  energy {eF:.2e}")
    assert e < TOL_STEP[dtype] and es < TOL_STEP[dtype] and eF < TOL_STEP[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mixed_mass_is_conserved_bitwise(pfc, dtype):
    shape = (30, 20, 12)
    psi0 = rounded(P.pfc_initial_field(52, shape, -0.3), dtype)
    plan = pfc.Plan(shape, dtype=dtype, r=-0.3, dt=0.5)
    psi = to_dev(psi0, dtype)
    state = plan.state_init(psi)
    s0 = to_np(plan.state_export(state))[0, 0, 0]
    plan.step(psi, state, 25)
    s1 = to_np(plan.state_export(state))[0, 0, 0]
    say(f"[mixed mass] {dtype}: k = 0 mode {s0} -> {s1}")
    assert s0 == s1


@pytest.fixture(scope="module")
def oracle_750():
    """Two FP64 oracle steps at 750^3 (several seconds on the host)."""
    shape = (750, 750, 750)
    psi0 = P.pfc_initial_field(53, shape, -0.30)
    p = oracle.Params(shape, r=-0.30, dt=0.5)
    ref_psi, _ = oracle.step(p, psi0, oracle.state_init(p, psi0), 2)
    return psi0, ref_psi


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_750_cube_two_steps_vs_oracle(pfc, oracle_750, dtype):
    shape = (750, 750, 750)
    psi0, ref_psi = oracle_750
    say(f"[mixed 750^3] dtype={dtype}, 2 steps")
    plan = pfc.Plan(shape, dtype=dtype, r=-0.30, dt=0.5)
    psi = to_dev(rounded(psi0, dtype), dtype)
    state = plan.state_init(psi)
    plan.step(psi, state, 2)
    e = parity_err(to_np(psi), ref_psi)
    say(f"      psi rel L2 {e:.2e}")
    assert e < (1e-12 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mixed_adjoint_rollout_vs_oracle(pfc, dtype):
    """Gradient of L = sum (psi(T) - target)^2 with respect to psi0 and r through 60 steps on a
    30 x 20 grid, against the oracle's adjoint sweep."""
    shape, nsteps, r0, rt = (30, 20), 60, -0.25, -0.30
    say(f"[mixed adjoint] shape={shape} dtype={dtype} nsteps={nsteps}")
    psi0 = rounded(P.pfc_initial_field(59, shape, r0), dtype)
    target = oracle.rollout(oracle.Params(shape, r=rt, dt=0.5), psi0, nsteps)[-1]
    L_ref, g_ref, dr_ref = oracle.loss_and_grad(oracle.Params(shape, r=r0, dt=0.5), psi0, target, nsteps)
    plan = pfc.Plan(shape, dtype=dtype, r=r0, dt=0.5)
    L, g, dr = pfc.loss_and_grad(plan, to_dev(psi0, dtype), r0, to_dev(target, dtype), nsteps, 20)
    eg = parity_err(to_np(g), g_ref)
    say(f"      L {L:.10g} vs {L_ref:.10g}; grad rel L2 {eg:.2e}; dL/dr {dr:.8g} vs {dr_ref:.8g}")
    tol = 1e-10 if dtype == "f64" else 1e-3
    assert abs(L - L_ref) < tol * abs(L_ref) and eg < tol and abs(dr - dr_ref) < tol * abs(dr_ref)
