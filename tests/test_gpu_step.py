"""GPU parity of the PFC step, state, energy and adjoint entry points against the FP64 oracle.

Workloads follow the PFC runs of the benchmark configurations: dx = pi/4, psi0 = mean + U(-0.1, 0.1)
from a seeded SplitMix64 stream, dt = 0.5 (0.25 for the two-mode model).  Tolerance after 100
steps: relative L2 <= 1e-12 (FP64), <= 1e-4 (FP32)."""
import numpy as np
import pytest

import oracle
import pfc_inputs as P
from gpu_common import TOL_STEP, parity_err, rounded, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pfc():
    import paper_2603_26818_amd as m

    m.load_library()
    return m


def _run(pfc, shape, dtype, nsteps, seed, r, dt=0.5, model=0, q1sq=4.0 / 3.0, R1=0.0, flags=0, chunks=1):
    psi0 = rounded(P.pfc_initial_field(seed, shape, r), dtype)
    plan = pfc.Plan(shape, dtype=dtype, r=r, dt=dt, model=model, q1sq=q1sq, R1=R1, flags=flags)
    psi = to_dev(psi0, dtype)
    state = plan.state_init(psi)
    for _ in range(chunks):
        plan.step(psi, state, nsteps // chunks)
    F = plan.energy(psi, state)
    p = oracle.Params(shape, r=r, dt=dt, model=model, q1sq=q1sq, R1=R1, linear_only=bool(flags & 1))
    ref_psi, ref_state = oracle.step(p, psi0, oracle.state_init(p, psi0), nsteps)
    ref_F = oracle.energy(p, ref_psi, ref_state)
    return plan, psi0, psi, state, F, ref_psi, ref_state, ref_F


CASES = [
    # (shape, dtype, nsteps, seed, r)
    ((128, 128), "f64", 100, 1, -0.25),  # the 2D 128^2 FP64 configuration
    ((128, 128), "f32", 100, 1, -0.25),
    ((64, 64, 64), "f64", 100, 2, -0.30),
    ((64, 64, 64), "f32", 100, 2, -0.30),
    ((16, 32, 8), "f64", 60, 3, -0.30),
    ((8, 64), "f64", 60, 4, -0.25),
    ((4, 4), "f64", 20, 5, -0.25),
    ((4, 8, 4), "f64", 20, 6, -0.30),
    ((256, 64), "f32", 50, 7, -0.25),
    ((32, 128, 64), "f32", 40, 8, -0.30),
    # long x rows: the fused x pass (M = 256, 512) and the separate passes (M = 1024) on padded LDS rows
    ((4, 4, 512), "f64", 20, 12, -0.30),
    ((8, 1024), "f32", 40, 13, -0.25),
    ((4, 2048), "f64", 20, 14, -0.25),
]


@pytest.mark.parametrize("shape,dtype,nsteps,seed,r", CASES)
def test_step_vs_oracle(pfc, shape, dtype, nsteps, seed, r):
    say(f"[step] shape={shape} dtype={dtype} nsteps={nsteps} seed={seed} r={r}")
    plan, psi0, psi, state, F, ref_psi, ref_state, ref_F = _run(pfc, shape, dtype, nsteps, seed, r, chunks=2)
    e = parity_err(to_np(psi), ref_psi)
    F = to_np(F)
    eF = abs(F[0] - ref_F[0]) / abs(ref_F[0])
    es = parity_err(to_np(plan.state_export(state)), ref_state)
    say(f"       psi rel L2 {e:.2e}  state rel L2 {es:.2e}  energy rel {eF:.2e}  F={F[0]:.10g}")
    assert e < TOL_STEP[dtype] and es < TOL_STEP[dtype] and eF < TOL_STEP[dtype]
    assert abs(F[1] - ref_F[2]) < (1e-15 if dtype == "f64" else 1e-7)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_mode_operator(pfc, dtype):
    shape = (64, 128)
    say(f"[step] two-mode shape={shape} dtype={dtype}")
    plan, psi0, psi, state, F, ref_psi, ref_state, ref_F = _run(
        pfc, shape, dtype, 100, 9, -0.30, dt=0.25, model=1, q1sq=2.0, R1=0.05)
    e = parity_err(to_np(psi), ref_psi)
    say(f"       psi rel L2 {e:.2e}")
    assert e < TOL_STEP[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_linear_only_closed_form(pfc, dtype):
    """Nonlinearity off: every mode decays by 1/(1 + dt q (r + L(q))) per step."""
    shape = (16, 32, 64)
    say(f"[step] linear-only shape={shape} dtype={dtype}")
    plan, psi0, psi, state, F, ref_psi, ref_state, _ = _run(pfc, shape, dtype, 12, 10, -0.3, flags=1)
    e = parity_err(to_np(plan.state_export(state)), ref_state)
    say(f"       state rel L2 {e:.2e}")
    assert e < (1e-13 if dtype == "f64" else 5e-6)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mass_mode_bitwise_and_zero_steps(pfc, dtype):
    import torch

    shape = (32, 16, 32)
    say(f"[step] mass shape={shape} dtype={dtype}")
    psi0 = rounded(P.pfc_initial_field(11, shape, -0.3), dtype)
    plan = pfc.Plan(shape, dtype=dtype, r=-0.3, dt=0.5)
    psi = to_dev(psi0, dtype)
    state = plan.state_init(psi)
    s0 = state.clone()
    # the k = 0 mode comes from an FP64 sum of psi0, rounded once
    expect = np.float32(psi0.sum()) if dtype == "f32" else psi0.sum()
    assert abs(to_np(state)[0, 0, 0].real - expect) <= abs(expect) * (1e-7 if dtype == "f32" else 1e-13)
    plan.step(psi, state, 0)
    assert torch.equal(state, s0)
    assert np.array_equal(to_np(psi), psi0)
    plan.step(psi, state, 30)
    torch.cuda.synchronize()
    assert state[0, 0, 0].real.item() == s0[0, 0, 0].real.item()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_energy_vs_oracle_random_state(pfc, dtype):
    shape = (32, 64, 16)
    say(f"[energy] shape={shape} dtype={dtype}")
    psi0 = rounded(P.pfc_initial_field(12, shape, -0.3), dtype)
    p = oracle.Params(shape, r=-0.3)
    plan = pfc.Plan(shape, dtype=dtype, r=-0.3)
    psi = to_dev(psi0, dtype)
    state = plan.state_init(psi)
    F = to_np(plan.energy(psi, state))
    ref = oracle.energy(p, psi0, oracle.state_init(p, psi0))
    say(f"       F {F[0]:.12g} vs {ref[0]:.12g}")
    assert abs(F[0] - ref[0]) < (1e-13 if dtype == "f64" else 1e-6) * abs(ref[0])
    assert abs(F[1] - ref[2]) < (1e-15 if dtype == "f64" else 1e-7)


@pytest.mark.parametrize("shape,dtype", [((16, 16), "f64"), ((64, 32), "f32"), ((8, 16, 32), "f64"),
                                         ((32, 32, 32), "f32")])
def test_step_backward_vs_oracle(pfc, shape, dtype):
    import torch

    say(f"[adjoint] one step shape={shape} dtype={dtype}")
    psi_n = rounded(P.pfc_initial_field(13, shape, -0.25), dtype)
    lam = rounded(P.normal(14, shape), dtype)
    p = oracle.Params(shape, r=-0.25, dt=0.5)
    psi_np1, _ = oracle.step(p, psi_n, oracle.rfftn(psi_n), 1)
    psi_np1 = rounded(psi_np1, dtype)
    ref_lam, ref_g = oracle.step_backward(p, psi_n, psi_np1, lam)
    plan = pfc.Plan(shape, dtype=dtype, r=-0.25, dt=0.5)
    dl = torch.full((1,), 0.5, dtype=torch.float64, device="cuda:0")
    out, dl = plan.step_backward(to_dev(psi_n, dtype), to_dev(psi_np1, dtype), to_dev(lam, dtype), dLdr=dl)
    e = parity_err(to_np(out), ref_lam)
    eg = abs(to_np(dl)[0] - 0.5 - ref_g) / abs(ref_g)
    say(f"       lambda rel L2 {e:.2e}  dL/dr rel {eg:.2e}")
    tol = 1e-13 if dtype == "f64" else 5e-6
    assert e < tol and eg < tol * 10
    # in place: lambda_n may be the lambda_np1 buffer
    lam_d = to_dev(lam, dtype)
    out2, _ = plan.step_backward(to_dev(psi_n, dtype), to_dev(psi_np1, dtype), lam_d, lambda_n=lam_d)
    assert parity_err(to_np(out2), ref_lam) < tol


def test_watchdog_reports_divergence(pfc):
    """A NaN planted in psi0 (forced from the host) is caught at the first check; a finite run
    passes and ends like pfc_step."""
    import torch

    shape = (32, 64)
    say("[watchdog] NaN in psi0")
    psi0 = P.pfc_initial_field(15, shape, -0.25)
    plan = pfc.Plan(shape, dtype="f64", r=-0.25, dt=0.5)
    x = to_dev(psi0, "f64")
    s = plan.state_init(x)
    x2, s2 = x.clone(), s.clone()
    assert plan.step_watched(x, s, 40, check_every=7) == 40
    plan.step(x2, s2, 40)
    torch.cuda.synchronize()
    assert torch.equal(x, x2)
    bad = psi0.copy()
    bad[3, 5] = np.nan
    xb = to_dev(bad, "f64")
    sb = plan.state_init(xb)
    with pytest.raises(pfc.PfcError) as ei:
        plan.step_watched(xb, sb, 40, check_every=10)
    assert ei.value.status == 6 and "after 10 steps" in str(ei.value)
