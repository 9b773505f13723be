"""Gradients through the PFC rollout (PFCRollout: checkpointed forward, replay, pfc_step_backward).

Workload of the adjoint configuration: 2D one-mode PFC, 512^2, dt = 0.5, 2000 steps, checkpoints
every 50 steps; loss = sum (psi(T) - target)^2 where the target is a run from the same psi0 at
r = -0.30, and the gradient is taken at r = -0.25 with respect to psi0 and r.  psi0 = -0.25 +
U(-0.1, 0.1), seed 5.  Checks: the FP64 CPU adjoint (oracle), central finite differences of the
GPU forward along 16 seeded directions, and FP32 against FP64."""
import numpy as np
import pytest

import oracle
import pfc_inputs as P
from gpu_common import fmt_errs, parity_err, parity_errs, rounded, say, to_dev, to_np

pytestmark = pytest.mark.gpu

SHAPE, NSTEPS, R0, RT, DT = (512, 512), 2000, -0.25, -0.30, 0.5


@pytest.fixture(scope="module")
def pfc():
    import paper_2603_26818_amd as m

    m.load_library()
    return m


@pytest.fixture(scope="module")
def oracle_512sq_2000():
    """FP64 CPU adjoint at the full size (about half a minute on the host)."""
    psi0 = P.pfc_initial_field(5, SHAPE, R0)
    target = oracle.rollout(oracle.Params(SHAPE, r=RT, dt=DT), psi0, NSTEPS)[-1]
    L, g, dr = oracle.loss_and_grad(oracle.Params(SHAPE, r=R0, dt=DT), psi0, target, NSTEPS)
    return psi0, target, L, g, dr


def _gpu_target(pfc, dtype, psi0):
    plan = pfc.Plan(SHAPE, dtype=dtype, r=RT, dt=DT)
    psi = to_dev(psi0, dtype)
    st = plan.state_init(psi)
    plan.step(psi, st, NSTEPS)
    return psi


def test_rollout_matches_oracle_small(pfc):
    shape, nsteps = (32, 64), 130  # segments of 50, 50 and 30 steps
    say(f"[rollout] shape={shape} nsteps={nsteps} FP64")
    psi0 = P.pfc_initial_field(6, shape, R0)
    target = oracle.rollout(oracle.Params(shape, r=RT, dt=DT), psi0, nsteps)[-1]
    L_ref, g_ref, dr_ref = oracle.loss_and_grad(oracle.Params(shape, r=R0, dt=DT), psi0, target, nsteps)
    plan = pfc.Plan(shape, dtype="f64", r=R0, dt=DT)
    L, g, dr = pfc.loss_and_grad(plan, to_dev(psi0, "f64"), R0, to_dev(target, "f64"), nsteps, 50)
    eg = parity_err(to_np(g), g_ref)
    say(f"          L {L:.12g} vs {L_ref:.12g}; grad rel L2 {eg:.2e}; dL/dr {dr:.10g} vs {dr_ref:.10g}")
    assert abs(L - L_ref) < 1e-11 * abs(L_ref)
    assert eg < 1e-10
    assert abs(dr - dr_ref) < 1e-10 * abs(dr_ref)


def test_rollout_512sq_2000_fp64_vs_cpu_adjoint(pfc, oracle_512sq_2000):
    psi0, target_ref, L_ref, g_ref, dr_ref = oracle_512sq_2000
    say(f"[rollout] {SHAPE} {NSTEPS} steps FP64 vs CPU adjoint")
    target = _gpu_target(pfc, "f64", psi0)
    say(f"          target rel L2 vs oracle {parity_err(to_np(target), target_ref):.2e}")
    plan = pfc.Plan(SHAPE, dtype="f64", r=R0, dt=DT)
    L, g, dr = pfc.loss_and_grad(plan, to_dev(psi0, "f64"), R0, target, NSTEPS, 50)
    eg = parity_err(to_np(g), g_ref)
    say(f"          L {L:.12g} vs {L_ref:.12g}; grad rel L2 {eg:.2e}; dL/dr {dr:.10g} vs {dr_ref:.10g}")
    assert abs(L - L_ref) < 1e-8 * abs(L_ref)
    assert eg < 1e-8
    assert abs(dr - dr_ref) < 1e-8 * abs(dr_ref)


def test_rollout_512sq_2000_central_differences(pfc):
    """<dL/dpsi0, v> and dL/dr against central differences of the GPU FP64 forward.  Each estimate
    is Richardson-extrapolated, (4 D(h/2) - D(h)) / 3, which removes the h^2 truncation term; h is
    taken from a scan where successive extrapolated estimates agree best (the plateau)."""
    import torch

    say(f"[rollout] {SHAPE} FP64 central differences, 16 directions")
    psi0 = P.pfc_initial_field(5, SHAPE, R0)
    target = _gpu_target(pfc, "f64", psi0)
    plan = pfc.Plan(SHAPE, dtype="f64", r=R0, dt=DT)
    x0 = to_dev(psi0, "f64")
    L, g, dr = pfc.loss_and_grad(plan, x0, R0, target, NSTEPS, 50)

    def loss(x, r):
        plan.set_params(r, DT)
        psi = x.clone()
        st = plan.state_init(psi)
        plan.step(psi, st, NSTEPS)
        d = psi - target
        return float(torch.sum(d * d))

    def fd(fun, hs):
        D = {h: (fun(h) - fun(-h)) / (2 * h) for h in hs}
        est = [(4 * D[hs[i + 1]] - D[hs[i]]) / 3 for i in range(len(hs) - 1)]  # hs[i+1] = hs[i]/2
        # the two neighbouring estimates that agree best
        k = min(range(len(est) - 1), key=lambda i: abs(est[i] - est[i + 1]))
        return est[k + 1], abs(est[k] - est[k + 1])

    worst = 0.0
    for t in range(16):
        v = to_dev(P.normal(500 + t, SHAPE), "f64")
        v /= torch.linalg.vector_norm(v)
        gv = float(torch.sum(g * v))
        est, spread = fd(lambda h: loss(x0 + h * v, R0), [2e-3, 1e-3, 5e-4, 2.5e-4, 1.25e-4])
        rel = abs(est - gv) / max(abs(gv), 1e-12 * float(torch.linalg.vector_norm(g)))
        worst = max(worst, rel)
        say(f"          dir {t:2d}: adjoint {gv:+.10e}  FD {est:+.10e}  rel {rel:.1e}")
    # r enters every step's multiplier, so L(r) curves far more than L along psi0: smaller h
    est_r, _ = fd(lambda h: loss(x0, R0 + h), [1.6e-5, 8e-6, 4e-6, 2e-6, 1e-6, 5e-7])
    rel_r = abs(est_r - dr) / abs(dr)
    say(f"          dL/dr adjoint {dr:+.10e}  FD {est_r:+.10e}  rel {rel_r:.1e}; worst direction {worst:.1e}")
    assert worst < 1e-5 and rel_r < 1e-5


def test_rollout_512sq_2000_fp32_vs_fp64(pfc, oracle_512sq_2000):
    """The FP32 run's gradient against the FP64 CPU adjoint, end to end: the FP32 forward trajectory
    departs from FP64 over the 2000 steps, and the backward sweep adds its own rounding (bounded
    separately below, observed 2.5e-4).  Observed 1.8e-3 for the psi0 gradient and 1.1e-3 for dL/dr;
    gated at 5e-3."""
    psi0, target_ref, L_ref, g_ref, dr_ref = oracle_512sq_2000
    say(f"[rollout] {SHAPE} FP32 vs FP64 CPU adjoint")
    p32 = rounded(psi0, "f32")
    target = _gpu_target(pfc, "f32", p32)
    plan = pfc.Plan(SHAPE, dtype="f32", r=R0, dt=DT)
    L, g, dr = pfc.loss_and_grad(plan, to_dev(p32, "f32"), R0, target, NSTEPS, 50)
    eg = parity_errs(to_np(g), g_ref)
    say(f"          L {L:.8g} vs {L_ref:.8g}; grad {fmt_errs(eg)}; dL/dr {dr:.8g} vs {dr_ref:.8g}")
    assert max(eg) < 5e-3 and abs(dr - dr_ref) < 5e-3 * abs(dr_ref)


def test_rollout_512sq_2000_fp32_adjoint_along_its_own_trajectory(pfc):
    """The FP32 adjoint's own error, separated from the drift of the FP32 forward run: the FP64
    oracle's adjoint step is swept backward along the GPU's own FP32 trajectory (every psi^n of the
    FP32 forward run, widened to FP64; the rollout's replay reproduces that trajectory bit for bit)
    from lambda^T = 2 (psi^T - target), target the FP32 GPU run at r = -0.30.  Both sweeps then see
    the same forward states, so their difference is the rounding of the FP32 backward steps alone.

    Gate 1e-3: one FP32 backward step has relative error d1 (measured here at the middle of the
    trajectory, about 3e-7: three FP32 transforms); if each step's rounding were carried to lambda^0
    undamped, 2000 steps would accumulate at most 2000 d1, about 6e-4.  Observed 2.5e-4 (psi0
    gradient) and 6e-5 (dL/dr).  The FP32 forward drift over the same run is reported beside it."""
    psi0 = rounded(P.pfc_initial_field(5, SHAPE, R0), "f32")
    say(f"[rollout] {SHAPE} {NSTEPS} steps: FP32 GPU adjoint vs the FP64 adjoint along the FP32 trajectory")
    target = _gpu_target(pfc, "f32", psi0)
    plan = pfc.Plan(SHAPE, dtype="f32", r=R0, dt=DT)
    L, g, dr = pfc.loss_and_grad(plan, to_dev(psi0, "f32"), R0, target, NSTEPS, 50)
    # the FP32 forward trajectory at r = R0, kept on the host in FP32
    plan.set_params(R0, DT)
    x = to_dev(psi0, "f32")
    st = plan.state_init(x)
    traj = np.empty((NSTEPS + 1,) + SHAPE, np.float32)
    traj[0] = psi0
    for n in range(NSTEPS):
        plan.step(x, st, 1)
        traj[n + 1] = x.cpu().numpy()
    # forward drift of FP32 from FP64 over the same steps
    p64 = pfc.Plan(SHAPE, dtype="f64", r=R0, dt=DT)
    x64 = to_dev(psi0, "f64")
    p64.step(x64, p64.state_init(x64), NSTEPS)
    drift = parity_errs(traj[NSTEPS].astype(np.float64), to_np(x64))
    # FP64 adjoint sweep along the FP32 trajectory
    po = oracle.Params(SHAPE, r=R0, dt=DT)
    lam = 2.0 * (traj[NSTEPS].astype(np.float64) - to_np(target))
    acc = 0.0
    mid = NSTEPS // 2
    d1 = None
    for n in range(NSTEPS - 1, -1, -1):
        lam_new, c = oracle.step_backward(po, traj[n].astype(np.float64), traj[n + 1].astype(np.float64), lam)
        if n == mid:  # one FP32 GPU backward step on the same (FP32-rounded) inputs
            lam32 = to_dev(lam.astype(np.float32), "f32")
            got, _ = plan.step_backward(to_dev(traj[n], "f32"), to_dev(traj[n + 1], "f32"), lam32)
            ref1, _ = oracle.step_backward(po, traj[n].astype(np.float64), traj[n + 1].astype(np.float64),
                                           lam.astype(np.float32).astype(np.float64))
            d1 = parity_errs(to_np(got), ref1)
        lam = lam_new
        acc += c
    eg = parity_errs(to_np(g), lam)
    er = abs(dr - acc) / abs(acc)
    say(f"          forward FP32 drift at step {NSTEPS}: {fmt_errs(drift)}")
    say(f"          one FP32 backward step (n = {mid}): {fmt_errs(d1)}; {NSTEPS} x that: {NSTEPS * max(d1):.2e}")
    say(f"          dL/dpsi0 {fmt_errs(eg)}; dL/dr {dr:.8g} vs {acc:.8g} (rel {er:.2e})")
    assert max(d1) < 5e-6
    assert max(eg) < 1e-3 and er < 1e-3
