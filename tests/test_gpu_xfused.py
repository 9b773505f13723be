"""The fused x pass between steps (the x c2r of one step, the cube and the x r2c of the next in one
kernel, the real field in between kept in LDS): K steps in one call equal K calls of one step (which
never fuse) bit for bit, for power-of-two and mixed-radix rows, 2D and 3D, FP32 and FP64, and the
plane-block layout.  Runs of several steps in one call are also what the oracle comparisons of
test_gpu_step.py, test_gpu_mixed.py and test_gpu_fullsize.py time, so the fused pass is checked
against the oracle there."""
import pytest

import pfc_inputs as P
from gpu_common import rounded, say, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ((64, 32, 128), "f32"),
    ((64, 32, 128), "f64"),
    ((16, 8, 750), "f32"),  # 375-point rows over 32 threads
    ((12, 10, 1400), "f64"),  # 700-point rows over 64 threads
    ((8, 8, 2048), "f32"),  # 1024-point rows
    ((256, 128, 2048), "f32"),  # plane pairs (z >= 256, planes of 1 MiB)
    ((2048, 64), "f32"),  # 2D, 32-point rows
    ((32, 1024), "f64"),  # 2D, 512-point rows
]


@pytest.fixture(scope="module")
def pfc():
    import paper_2603_26818_amd as m

    m.load_library()
    return m


@pytest.mark.parametrize("shape,dtype", CASES)
def test_k_steps_in_one_call_equal_k_single_steps(pfc, shape, dtype):
    import torch

    nsteps = 4
    say(f"[xfused] shape={shape} dtype={dtype} {nsteps} steps")
    psi0 = rounded(P.pfc_initial_field(41, shape, -0.3), dtype)
    plan = pfc.Plan(shape, dtype=dtype, r=-0.3, dt=0.5)
    assert plan.x_fused == (shape[-1] // 2 < 1024)  # every default x schedule here fits a wavefront
    # zero-filled states: rows padded to whole lines keep their padding, which no kernel reads or
    # writes, so the raw buffers compare equal only if both start alike
    a = to_dev(psi0, dtype)
    sa = plan.state_init(a, torch.zeros_like(plan.empty_state()))
    plan.step(a, sa, nsteps)
    b = to_dev(psi0, dtype)
    sb = plan.state_init(b, torch.zeros_like(plan.empty_state()))
    for _ in range(nsteps):
        plan.step(b, sb, 1)
    torch.cuda.synchronize()
    assert torch.equal(a, b), "psi differs between one call of K steps and K calls of one step"
    assert torch.equal(sa, sb), "state differs between one call of K steps and K calls of one step"
