"""GPU parity of the hydrodynamic PFC step (pfc_hydro_step: density and Gaussian-averaged velocity,
Eq. (5)-(6), Listing 2) against the FP64 oracle, whose hydrodynamic step is pinned in
test_oracle_hydro.py.  psi0 = mean + U(-0.1, 0.1), v0 = U(-0.05, 0.05) per component (seeded), dx =
pi/4, dt = 0.5 (0.25 in 3D).  Tolerances after the stated steps: relative L2 1e-12 (FP64), 1e-4
(FP32) on psi and on every velocity component."""
import numpy as np
import pytest

import oracle
import pfc_inputs as P
from gpu_common import TOL_STEP, fmt_errs, parity_err, parity_errs, rounded, say, to_dev, to_np

pytestmark = pytest.mark.gpu

CASES = [
    # (shape, dtype, nsteps, seed, (rho0, gamma, a0))
    ((64, 64), "f64", 30, 71, (1.0, 1.0, 1.0)),
    ((64, 64), "f32", 30, 71, (1.0, 1.0, 1.0)),
    ((32, 128), "f64", 20, 72, (0.5, 2.0, 0.8)),
    ((16, 32, 64), "f64", 12, 73, (1.0, 1.0, 1.0)),
    ((16, 32, 64), "f32", 12, 73, (1.0, 1.0, 1.0)),
    ((30, 20, 12), "f64", 10, 74, (1.0, 0.5, 1.2)),  # mixed radix
    ((8, 16, 8), "f64", 10, 75, (2.0, 1.0, 0.0)),  # a0 = 0: no averaging
]


@pytest.fixture(scope="module")
def pfc():
    import paper_2603_26818_amd as m

    m.load_library()
    return m


@pytest.mark.parametrize("shape,dtype,nsteps,seed,hp", CASES)
def test_hydro_step_vs_oracle(pfc, shape, dtype, nsteps, seed, hp):
    d = len(shape)
    r, dt = (-0.25, 0.5) if d == 2 else (-0.30, 0.25)
    say(f"[hydro] shape={shape} dtype={dtype} nsteps={nsteps} seed={seed} rho0,gamma,a0={hp}")
    psi0 = rounded(P.pfc_initial_field(seed, shape, r), dtype)
    v0 = np.stack([rounded(P.uniform(seed * 10 + j, shape, -0.05, 0.05), dtype) for j in range(d)])
    p = oracle.Params(shape, r=r, dt=dt)
    h = oracle.Hydro(*hp)
    ref = oracle.hydro_step(p, h, psi0, oracle.rfftn(psi0), v0, np.stack([oracle.rfftn(x) for x in v0]), nsteps)
    plan = pfc.Plan(shape, dtype=dtype, r=r, dt=dt)
    psi, v = to_dev(psi0, dtype), to_dev(v0, dtype)
    S, V = plan.hydro_state_init(psi, v)
    plan.hydro_step(psi, S, v, V, nsteps, *hp)
    e = parity_err(to_np(psi), ref[0])
    ev = [parity_err(to_np(v[j]), ref[2][j]) for j in range(d)]
    es = parity_err(to_np(plan.state_export(S)), ref[1])
    say(f"      psi rel L2 {e:.2e}  state {es:.2e}  v {' '.join(f'{x:.2e}' for x in ev)}")
    tol = TOL_STEP[dtype]
    assert e < tol and es < tol and max(ev) < tol


def _hydro_full(pfc, n, dtype, seed, nsteps):
    """The benchmark's hydrodynamic workload at n^3 (rho0 = gamma = a0 = 1, r = -0.30, dt = 0.25,
    psi0 = -0.30 + U(-0.1, 0.1) and v0 = U(-0.05, 0.05) per component, drawn on the device as the
    benchmark draws them), nsteps steps with the benchmark's launches, against the oracle's
    hydrodynamic step from the same (rounded) fields: psi, its state and every velocity component."""
    import torch

    shape, r, dt, hp = (n, n, n), -0.30, 0.25, (1.0, 1.0, 1.0)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    say(f"[hydro] {n}^3 {dtype} seed {seed}: {nsteps} steps vs the oracle")
    plan = pfc.Plan(shape, dtype=dtype, r=r, dt=dt)
    psi = P.pfc_initial_field_torch(seed, shape, r, tdt, "cuda:0")
    v = torch.stack([P.uniform_torch(seed * 10 + j, shape, -0.05, 0.05, tdt, "cuda:0") for j in range(3)])
    psi0, v0 = to_np(psi), to_np(v)
    S, V = plan.hydro_state_init(psi, v)
    work = torch.empty(int(plan._lib.pfc_hydro_work_bytes(plan._h)), dtype=torch.uint8, device="cuda:0")
    plan.hydro_step(psi, S, v, V, nsteps, work=work)
    got_psi, got_v, got_S = to_np(psi), to_np(v), to_np(plan.state_export(S))
    state_bytes = int(plan._lib.pfc_plan_state_bytes(plan._h))
    del psi, v, S, V, work, plan
    torch.cuda.empty_cache()
    p = oracle.Params(shape, r=r, dt=dt)
    ref = oracle.hydro_step(p, oracle.Hydro(*hp), psi0, oracle.rfftn(psi0), v0,
                            np.stack([oracle.rfftn(x) for x in v0]), nsteps)
    e = parity_errs(got_psi, ref[0])
    es = parity_errs(got_S, ref[1])
    ev = [parity_errs(got_v[j], ref[2][j]) for j in range(3)]
    say(f"      psi {fmt_errs(e)}\n      state {fmt_errs(es)}")
    for j in range(3):
        say(f"      v{j} {fmt_errs(ev[j])}")
    return state_bytes, max(max(e), max(es), max(max(x) for x in ev))


def test_hydro_bench_workload_512_fp32_vs_oracle(pfc):
    """512^3 FP32, the benchmark's seed 9: 2 steps (the 512-point last-axis derivative schedules,
    the spectral updates, the multiply-accumulate epilogue and the non-temporal x and y passes of
    states over 128 MiB, as the benchmark runs them)."""
    _, err = _hydro_full(pfc, 512, "f32", 9, 2)
    assert err < TOL_STEP["f32"]


def test_hydro_256_fp64_nontemporal_vs_oracle(pfc):
    """256^3 FP64: a 128 MiB state, so the passes take their non-temporal loads and stores."""
    state_bytes, err = _hydro_full(pfc, 256, "f64", 19, 2)
    assert state_bytes >= 128 << 20
    assert err < TOL_STEP["f64"]


def test_hydro_rejects_bad_arguments(pfc):
    import torch

    plan = pfc.Plan((16, 16), dtype="f64")
    psi = torch.zeros((16, 16), dtype=torch.float64, device="cuda:0")
    v = torch.zeros((2, 16, 16), dtype=torch.float64, device="cuda:0")
    S, V = plan.hydro_state_init(psi, v)
    with pytest.raises(pfc.PfcError):
        plan.hydro_step(psi, S, v, V, 1, rho0=0.0)
    with pytest.raises(pfc.PfcError):
        plan.hydro_step(psi, S, v, V, 1, work=torch.empty(64, dtype=torch.uint8, device="cuda:0"))
