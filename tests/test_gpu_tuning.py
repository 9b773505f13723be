"""Every candidate schedule the autotuner can pick is correct: each pass of the step is forced to
each of its candidates (pfc_plan_set_tuning) and the run is compared with the FP64 oracle; the
shapes cover the lengths 16 .. 2048 on every pass kind.  Then the autotuner itself runs."""
import numpy as np
import pytest

import oracle
import pfc_inputs as P
from gpu_common import parity_err, rounded, say, to_dev, to_np

pytestmark = pytest.mark.gpu

SHAPES = [(16, 32, 64), (64, 128, 256), (256, 512, 32), (512, 16, 1024), (1024, 64, 16), (2048, 8, 8),
          (4, 2048, 64), (8, 8, 2048), (16, 1024, 128), (128, 32, 128),
          (2048, 64), (1024, 2048), (512, 512), (256, 1024), (128, 32), (32, 256), (750, 750, 12), (1400, 1400, 12),
          (12, 10, 750), (10, 12, 1400)]
NSTEPS = 6
MAX_CANDIDATES = 5  # the most any pass has (the 512-point z and y passes: schedules and tiles)


@pytest.fixture(scope="module")
def pfc():
    import paper_2603_26818_amd as m

    m.load_library()
    return m


@pytest.mark.parametrize("shape", SHAPES)
def test_every_candidate_matches_oracle(pfc, shape):
    psi0 = P.pfc_initial_field(31, shape, -0.3)
    p = oracle.Params(shape, r=-0.3, dt=0.5)
    ref, _ = oracle.step(p, psi0, oracle.state_init(p, psi0), NSTEPS)
    for dtype in ("f64", "f32"):
        plan = pfc.Plan(shape, dtype=dtype, r=-0.3, dt=0.5)
        npass = len(plan.get_tuning())
        seen = set()
        for choice in range(MAX_CANDIDATES):
            variants = []
            for k in range(npass):  # candidate `choice` where the pass has it, else 0
                v = [0] * npass
                v[k] = choice
                try:
                    plan.set_tuning(v)
                    variants.append(choice)
                except Exception:
                    variants.append(0)
            if choice > 0 and all(v == 0 for v in variants):
                continue
            if tuple(variants) in seen:
                continue
            seen.add(tuple(variants))
            plan.set_tuning(variants)
            x = to_dev(rounded(psi0, dtype), dtype)
            st = plan.state_init(x)
            plan.step(x, st, NSTEPS)
            e = parity_err(to_np(x), ref)
            say(f"[tuning] shape={shape} dtype={dtype} variants={variants} rel L2 {e:.2e}")
            assert e < (1e-12 if dtype == "f64" else 1e-5)


def test_autotune_and_cache(pfc, tmp_path):
    shape = (64, 128, 256)
    plan = pfc.Plan(shape, dtype="f32", r=-0.3, dt=0.5)
    cache = str(tmp_path / "tune.json")
    v, best = plan.autotune(reps=3, cache_path=cache)
    say(f"[tuning] autotune {shape}: variants {v}, best ms {best}")
    assert best is not None and len(v) == 5
    plan2 = pfc.Plan(shape, dtype="f32", r=-0.3, dt=0.5)
    v2, best2 = plan2.autotune(cache_path=cache)
    assert v2 == v and best2 is None and plan2.get_tuning() == v
