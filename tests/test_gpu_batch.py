"""Batched persistent form (pfc_batch_*): every instance equals its own single-plan run.

The batched kernel runs the same per-element arithmetic as the single-plan path (same FFT
schedules, same twiddle values, same update), so each instance must match pfc_step bit for bit,
after every replay of the captured graph; the single-plan path is checked against the oracle in
test_gpu_step.py, and one instance is also checked against the oracle here."""
import numpy as np
import pytest

import oracle
import pfc_inputs as P
from gpu_common import fmt_errs, parity_err, parity_errs, rounded, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pfc():
    import paper_2603_26818_amd as m

    m.load_library()
    return m


def _instances(dtype):
    sizes = [(1024, 1024), (512, 512), (256, 128), (128, 256), (64, 64), (32, 1024), (128, 128), (512, 64)]
    out = []
    for i, shp in enumerate(sizes):
        two = i % 2 == 1
        r = float(P.uniform(P.derive_seed(4, i), (1,), -0.35, -0.15)[0])
        out.append(dict(shape=shp, dtype=dtype, model=1 if two else 0, r=r, dt=0.25,
                        q1sq=2.0 if two else 4.0 / 3.0, R1=0.05 if two else 0.0))
    return out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_matches_single_plans_every_replay(pfc, dtype):
    import torch

    insts = _instances(dtype)
    say(f"[batch] {len(insts)} instances dtype={dtype}")
    psi0 = [rounded(P.pfc_initial_field(P.derive_seed(4, 100 + i), d["shape"], d["r"]), dtype) for i, d in enumerate(insts)]
    b = pfc.Batch(insts)
    psis = [to_dev(x, dtype) for x in psi0]
    b.bind(psis)
    b.state_init()
    say(f"        grid {b.grid} workgroups")
    # single-plan runs of the same instances (eager launches)
    plans = [pfc.Plan(d["shape"], dtype=dtype, model=d["model"], r=d["r"], dt=d["dt"], q1sq=d["q1sq"], R1=d["R1"])
             for d in insts]
    ref_psi = [to_dev(x, dtype) for x in psi0]
    ref_state = [p.state_init(x) for p, x in zip(plans, ref_psi)]
    torch.cuda.synchronize()
    for k in range(len(insts)):
        assert torch.equal(b.state[k], ref_state[k]), f"state_init differs for instance {k}"
    # launches of 7 steps (graph replays; every step after the first runs the fused x c2r + x r2c
    # pass), then of 1 and 2 steps (no fused pass, and one)
    for rep, n in enumerate((7, 7, 7, 1, 2)):
        b.step(n)
        b.check()
        for p, x, s in zip(plans, ref_psi, ref_state):
            p.step(x, s, n)
        torch.cuda.synchronize()
        for k in range(len(insts)):
            same = torch.equal(b.psi[k], ref_psi[k]) and torch.equal(b.state[k], ref_state[k])
            if not same:
                e = parity_err(to_np(b.psi[k]), to_np(ref_psi[k]))
                raise AssertionError(f"replay {rep}: instance {k} {insts[k]['shape']} differs (rel L2 {e:.2e})")
        say(f"        replay {rep}: all instances bitwise equal to their single-plan runs")


def test_batch_instance_vs_oracle(pfc):
    insts = _instances("f64")[4:6]  # 64 x 64 one-mode and 32 x 1024 two-mode
    say(f"[batch] oracle check of {[d['shape'] for d in insts]}")
    psi0 = [P.pfc_initial_field(P.derive_seed(4, 200 + i), d["shape"], d["r"]) for i, d in enumerate(insts)]
    b = pfc.Batch(insts)
    b.bind([to_dev(x, "f64") for x in psi0])
    b.state_init()
    b.step(60)
    b.check()
    for k, d in enumerate(insts):
        p = oracle.Params(d["shape"], model=d["model"], r=d["r"], dt=d["dt"], q1sq=d["q1sq"], R1=d["R1"])
        ref, _ = oracle.step(p, psi0[k], oracle.state_init(p, psi0[k]), 60)
        e = parity_err(to_np(b.psi[k]), ref)
        say(f"        instance {d['shape']}: rel L2 {e:.2e}")
        assert e < 1e-12


def test_batch_bench_workload_after_autotune(pfc):
    """The benchmark's batched workload itself: 48 FP32 instances {128^2 .. 1024^2} x 12, one- and
    two-mode, seeded as the benchmark seeds them, on the schedules the autotuner picks.  After 100
    steps (one graph launch) every instance equals its single-plan run on the same schedules bit for
    bit, and one one-mode and one two-mode instance of each size equals its own FP64 oracle run
    (started from the same FP32-rounded field) within the FP32 step gate."""
    import torch

    insts = P.batch_workload()
    nsteps = 100
    say(f"[batch] benchmark workload: {len(insts)} FP32 instances, autotuned, {nsteps} steps")
    psi0 = [P.pfc_initial_field_torch(P.derive_seed(4, 1000 + i), d["shape"], d["r"], torch.float32, "cuda:0")
            for i, d in enumerate(insts)]
    b = pfc.Batch(insts).bind([x.clone() for x in psi0])
    variants, ms = b.autotune(steps=5)
    say(f"        chosen schedules by size: " + ", ".join(f"{d['shape'][0]}^2 {v}" for d, v in
                                                       list(zip(insts, variants))[::6]))
    b.state_init()
    b.step(nsteps)
    b.check()
    torch.cuda.synchronize()
    for k, d in enumerate(insts):
        p = pfc.Plan(d["shape"], dtype="f32", model=d["model"], r=d["r"], dt=d["dt"], q1sq=d["q1sq"], R1=d["R1"])
        p.set_tuning(variants[k])
        x = psi0[k].clone()
        s_ = p.state_init(x)
        p.step(x, s_, nsteps)
        torch.cuda.synchronize()
        assert torch.equal(b.psi[k], x), f"instance {k} {d['shape']} differs from its single-plan run"
    say("        all 48 instances bitwise equal to their single-plan runs on the same schedules")
    worst = 0.0
    for k in range(0, len(insts), 6):  # instances 0, 6, 12, ...: one one-mode, one two-mode per size
        d = insts[k]
        p = oracle.Params(d["shape"], model=d["model"], r=d["r"], dt=d["dt"], q1sq=d["q1sq"], R1=d["R1"])
        x0 = to_np(psi0[k])
        ref, _ = oracle.step(p, x0, oracle.state_init(p, x0), nsteps)
        errs = parity_errs(to_np(b.psi[k]), ref)
        say(f"        instance {k} {d['shape']} {'two' if d['model'] else 'one'}-mode r={d['r']:.4f}: {fmt_errs(errs)}")
        worst = max(worst, max(errs))
    assert worst < 1e-4


@pytest.mark.parametrize("choice", [1])
def test_batch_candidates_match_single_plans(pfc, choice):
    """Every instance on its alternative candidate schedules (where a pass has one) still equals the
    single-plan run on the same candidates, bit for bit."""
    import torch

    insts = _instances("f32")
    b = pfc.Batch(insts)
    psi0 = [rounded(P.pfc_initial_field(P.derive_seed(4, 300 + i), d["shape"], d["r"]), "f32") for i, d in enumerate(insts)]
    b.bind([to_dev(x, "f32") for x in psi0])
    tuning = []
    for k in range(len(insts)):
        t = []
        for j in range(3):
            trial = [list(v) for v in b.get_tuning()]
            trial[k][j] = choice
            try:
                b.set_tuning(trial)
                t.append(choice)
            except Exception:
                t.append(0)
        tuning.append(t)
    b.set_tuning(tuning)
    say(f"[batch] candidates {tuning}")
    b.state_init()
    b.step(9)
    b.check()
    for k, d in enumerate(insts):
        p = pfc.Plan(d["shape"], dtype="f32", model=d["model"], r=d["r"], dt=d["dt"], q1sq=d["q1sq"], R1=d["R1"])
        p.set_tuning(tuning[k])
        x = to_dev(psi0[k], "f32")
        s = p.state_init(x)
        p.step(x, s, 9)
        torch.cuda.synchronize()
        assert torch.equal(b.psi[k], x), f"instance {k} {d['shape']} differs"


def test_batch_autotune_and_cache(pfc, tmp_path):
    import torch

    insts = _instances("f32")
    b = pfc.Batch(insts)
    psi0 = [rounded(P.pfc_initial_field(P.derive_seed(4, 400 + i), d["shape"], d["r"]), "f32") for i, d in enumerate(insts)]
    b.bind([to_dev(x, "f32") for x in psi0])
    cache = str(tmp_path / "bt.json")
    v, ms = b.autotune(steps=3, cache_path=cache)
    say(f"[batch] autotuned {v}, {ms:.4f} ms/step")
    assert b.get_tuning() == v
    b.state_init()
    b.step(5)
    b.check()
    b2 = pfc.Batch(insts)
    b2.bind([to_dev(x, "f32") for x in psi0])
    v2, ms2 = b2.autotune(cache_path=cache)
    assert v2 == v and ms2 is None
    b2.state_init()
    b2.step(5)
    b2.check()
    torch.cuda.synchronize()
    for k in range(len(insts)):
        assert torch.equal(b.psi[k], b2.psi[k])
